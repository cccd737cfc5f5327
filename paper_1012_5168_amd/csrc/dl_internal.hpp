// dl_internal.hpp -- host-side declarations shared by the library's sources:
// handle structs, kernel argument blocks and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "dl_common.hpp"
#include "dloops.h"

namespace dl {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);

struct Error {
    int code;
    std::string msg;
};

#define DL_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw ::dl::Error{DL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};            \
    } while (0)

#define DL_REQUIRE(cond, msg)                                                                          \
    do {                                                                                               \
        if (!(cond)) throw ::dl::Error{DL_EINVAL, (msg)};                                              \
    } while (0)

// ---------------------------------------------------------------- precision

enum Prec { P64 = DL_F64, P32 = DL_F32, P16 = DL_F16, PBF = DL_BF16 };

inline size_t elem_bytes(int p)  // bytes of one stored complex number
{
    return p == P64 ? 16 : p == P32 ? 8 : 4;
}

// ---------------------------------------------------------------- device buffers

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;  // the requested size: what callers may read or write
    size_t cap = 0;    // the size of the underlying block (>= bytes when it came from the cache)
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap) { o.p = nullptr; o.bytes = o.cap = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        release();
        p = o.p; bytes = o.bytes; cap = o.cap;
        o.p = nullptr; o.bytes = o.cap = 0;
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t n);
    void release() noexcept;
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// The stream of the entry point running on this thread, for the duration of
// the call: a device buffer released meanwhile enters the memory cache with an
// event recorded on it, instead of a device-wide synchronisation.
struct StreamScope {
    explicit StreamScope(void *stream);
    ~StreamScope();
    StreamScope(const StreamScope &) = delete;
    StreamScope &operator=(const StreamScope &) = delete;
    bool prev_known;
    void *prev;
};

// A call that must not allocate (dl_apply_noalloc), for the duration of the
// scope on this thread: the autotuner only looks up choices it already holds
// (timing candidates would create events and write its cache file) and no
// profiling events are created.
struct NoAllocScope {
    NoAllocScope();
    ~NoAllocScope();
    NoAllocScope(const NoAllocScope &) = delete;
    NoAllocScope &operator=(const NoAllocScope &) = delete;
    bool prev;
};
bool no_alloc_active();

// nrhs half-spinor fields of one parity in one precision
struct HalfField {
    int prec = P64;
    int64_t nrhs = 0, Vh = 0;
    DevBuf data, nrm;
    void alloc(int prec_, int64_t nrhs_, int64_t Vh_);
    Field view() const { return Field{data.p, nrm.as<float>()}; }
    Field view_rhs(int64_t r) const;  // the fields from right-hand side r on
    size_t bytes() const { return data.bytes + nrm.bytes; }
};

// ---------------------------------------------------------------- handles

}  // namespace dl

struct dl_lattice_s {
    int32_t dims[4];
    int32_t tap;
    int64_t V, Vh;
    dl::Geom geom() const;
};

struct dl_gauge_s {
    dl_lattice_s lat;
    int32_t recon;
    uint32_t prec_mask;
    dl::DevBuf links[4];  // per precision: [4][2][NE][Vh]
};

namespace dl {

// ---------------------------------------------------------------- profiling

enum ProfKind { PROF_DSLASH = 0, PROF_BLAS = 1, PROF_TRACE = 2, PROF_DSLASH_PLAIN = 3, PROF_SMEAR = 4, PROF_NKIND = 5 };
// Brackets a launch with events when profiling is on.  The algorithmic bytes
// of the launch are `bytes`, or, when `counter` is set, fixed_bytes (if any
// work ran) plus unit_bytes times the number of units the kernel counted
// into *counter divided by `units_div` (the hopping kernel counts live
// right-hand-side blocks, so masked-off right-hand sides move no bytes).
struct ProfPart {
    unsigned *counter;
    double unit_bytes, fixed_bytes, units_div;
};
struct ProfScope {
    ProfScope(int kind, double bytes, hipStream_t s, int kind2 = -1);
    ~ProfScope();
    int kind, kind2;
    double bytes;
    hipStream_t s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<ProfPart> parts;  // counted byte terms (replace `bytes` when present)
};
// a zeroed device counter for the next profiled launch (null when profiling is off)
unsigned *prof_counter();
bool prof_on();
bool capturing(hipStream_t s);  // the stream is recording a graph

// ---------------------------------------------------------------- dslash

enum Epi {
    EPI_PLAIN = 0,     // out = a D in
    EPI_XPAY = 1,      // out = x + a D in
    EPI_XPAY_DOT = 2,  // out = x + a D in; partial (y, out)            [2 doubles]
    EPI_XPAY_TS = 3,   // out = x + a D in; partials (out, x), |out|^2, (y, out)   [5 doubles]
    EPI_XPAY_NRM = 4,  // out = x + a D in; partial |out|^2              [1 double]
    EPI_XMY_NRM = 5,   // out = x - y + a D in; partial |out|^2          [1 double]
    EPI_CG_R = 6,      // q = x + a D in; out = y - alpha q (out = y in place, alpha from
                       // the solver state); partial |out|^2; q itself is not stored   [1 double]
};

inline int epi_nparts(int epi)
{
    switch (epi) {
    case EPI_XPAY_DOT: return 2;
    case EPI_XPAY_TS: return 5;
    case EPI_XPAY_NRM: return 1;
    case EPI_XMY_NRM: return 1;
    case EPI_CG_R: return 1;
    default: return 0;
    }
}

struct DslashCall {
    Geom g;
    int parity;           // output parity
    int prec;             // storage precision of fields and links
    int recon;            // 12 or 18
    bool dag;             // D^dagger
    int epi;
    Field in, out, x, y;  // in: parity 1-p; out, x, y: parity p
    const void *links;
    double a;
    int nrhs;
    double *partials;     // [nrhs][nblk][nparts] (epilogues with reductions)
    const int *active;    // per right-hand side flag or null
    unsigned *live_count = nullptr;  // profiling: live right-hand-side blocks
    const struct KState *st = nullptr;  // per right-hand side solver state (EPI_CG_R's alpha)
};

// launch with the tuned (or default) configuration; returns the number of
// site blocks per right-hand side (the partials' middle extent) of each call.
// A batch of calls (same precision, link format, adjoint flag and epilogue;
// one per lattice) runs as one launch.
int launch_dslash(const DslashCall &c, hipStream_t s);
std::vector<int> launch_dslash_batch(const std::vector<DslashCall> &calls, hipStream_t s);

// launch configuration of the hopping kernel.  kind 0 (item kernel):
// right-hand sides per thread, sites per workgroup and the persistent grid
// cap (0 = one block per item).  kind 1 (LDS-link kernel): nr wavefronts per
// workgroup, 64 sites per workgroup, regions of `persistent` site blocks.
struct TuneChoice {
    int kind, nr, bs, persistent;
};
TuneChoice tune_lookup(const std::vector<DslashCall> &c, hipStream_t s);
void launch_dslash_any(const std::vector<DslashCall> &c, const TuneChoice &t, hipStream_t s);
// whether the LDS-link kernel serves this precision and link format (its
// links must fit the LDS a workgroup may hold), and the sites per block a choice gives
bool dslash_lds_ok(int prec, int recon);
// LDS a workgroup may hold on gfx950
constexpr int LDS_WORKGROUP_BYTES = 163840;
// links in the LDS-link kernel's LDS: expanded to three rows in the arithmetic
// precision (0), or as stored (1: the variant that rebuilds them per use)
#ifndef LDS_COMPACT_LINKS
#define LDS_COMPACT_LINKS 0
#endif
// FP64: only the six spatial links in LDS, as stored (36 KiB per block with
// 12-parameter links, so four blocks per CU), the two temporal links of a
// wavefront's sites in its registers (1)
#ifndef LDS_TLINK_REGS
#define LDS_TLINK_REGS 1
#endif
// bytes of links one 64-site block of the LDS-link kernel keeps in LDS
inline int lds_link_block_bytes(int prec, int recon)
{
    if (LDS_TLINK_REGS && prec == P64) return 6 * (recon == 12 ? 6 : 9) * 64 * 16;
    return LDS_COMPACT_LINKS ? 8 * (recon == 12 ? 6 : 9) * 64 * (int)elem_bytes(prec)
                             : 8 * 9 * 64 * (prec == P64 ? 16 : 8);
}
int dslash_block_sites(const DslashCall &c, const TuneChoice &t);

// ---------------------------------------------------------------- Krylov vector kernels

// Per right-hand side solver state, device resident.  The iterate / update
// flags live in separate int arrays (act, upd, restart) so that kernels can
// take them as masks.
struct KState {
    double rho[2], alpha[2], omega[2], beta[2];
    double rr;      // |r|^2 of the iterated residual
    double b2;      // |b|^2 of the full-lattice source
    double stop2;   // tol^2 * b2
    double maxrr;   // max |r|^2 since the last reliable update
    double delta2;  // reliable-update trigger squared
    double true2;   // last FP64 true residual squared (Schur system)
    int iters;
    int updates;
    int done;       // converged: FP64 true residual below tolerance
    int nonfinite;
    int maxiter;
    int pad;
};

int blas_blocks(int64_t Vh);

// Operands of a Krylov vector kernel for one segment (lattice).
struct VSeg {
    Field f[5];
    const KState *st = nullptr;
    const int *mask = nullptr;  // per right-hand side flags selecting who acts (null = all)
    int64_t Vh = 0;
    int nrhs = 0;
    double *parts = nullptr;    // [nrhs][blas_blocks(Vh)][np] for the reducing operations
    unsigned *live = nullptr;   // profiling: incremented once per right-hand side processed
};
enum VOp { V_BICG_S = 0, V_BICG_XRP, V_CG_XR, V_CG_P, V_ZERO, V_NORM2, V_DOT };
void vec_launch(int op, int prec, const std::vector<VSeg> &segs, hipStream_t s);
void copy_launch(int prec_dst, int prec_src, const std::vector<VSeg> &segs, hipStream_t s);  // f0 = f1
void fold_launch(int prec, const std::vector<VSeg> &segs, hipStream_t s);   // f0 (FP64) += f1; f1 = 0
// measurement only: copy (mode 0) or read (mode 1) nwords 16-byte words with non-temporal accesses
void stream_launch(int mode, const void *src, void *dst, int64_t nwords, hipStream_t s);
void zero_launch(void *p, int64_t nwords, hipStream_t s);  // nwords 16-byte words
// reliable update of the residual: f0 (r, precision prec) = f1 (FP64 residual), and the search
// direction f2 (p, precision prec) += f1 - old f0, so that p = r + beta (p - omega v) holds for the
// replaced r
void replace_launch(int prec, const std::vector<VSeg> &segs, hipStream_t s);
void sub_launch(const std::vector<VSeg> &segs, hipStream_t s);              // f0 = f1 - f2 (FP64)

// Operands of a per-right-hand-side scalar kernel for one segment.
struct SSeg {
    KState *st = nullptr;
    int *act = nullptr, *upd = nullptr, *restart = nullptr;
    const int *mask = nullptr;
    const double *parts = nullptr, *parts2 = nullptr;
    int nblk = 0;   // site blocks of the producing kernel (partials' middle extent)
    int nblk2 = 0;  // the same for parts2 where another kernel produced them (0: nblk)
    int nrhs = 0;
    double *out = nullptr;
};
struct SParams {
    double tol2 = 0, delta2 = 0;
    int maxiter = 0, np = 0, mixed = 0, final_check = 0;
};
enum SOp {
    S_BICG_INIT = 0,  // parts (+ parts2): |b_e|^2 (+ |b_o|^2)
    S_BICG_RHO,       // (re)start: parts (rhat, r); rho = (rhat, r), alpha = omega = 1
    S_BICG_ALPHA,     // parts: (rhat, v)
    S_BICG_OMEGA,     // parts: (t, s), |t|^2, (rhat, t); parts2: (rhat, s): omega, rho, beta
    S_BICG_CHECK,     // parts: |r|^2: iteration count, convergence and reliable-update flags
    S_BICG_RESYNC,    // parts: (rhat, r) after a reliable update: rho
    S_TRUE_RES,       // parts (+ parts2): FP64 residual norms
    S_CG_INIT,        // parts: |r|^2
    S_CG_ALPHA,       // parts: |Mhat p|^2
    S_CG_BETA,        // parts: |r|^2
    S_SUM             // out[rhs * np + k] = sum of partials
};
void scalar_launch(int op, const std::vector<SSeg> &segs, const SParams &p, hipStream_t s);

// ---------------------------------------------------------------- fields, sources, traces

// canonical complex128 [nrhs][V][4][3] <-> parity fields
void k_pack(int prec, Field dst, int parity, const double *canon, const Geom &g, int nrhs, hipStream_t s);
void k_unpack(int prec, Field src, int parity, double *canon, const Geom &g, int nrhs, hipStream_t s);

// internal source kind: the source is a stored FP64 field pair (xe, xo), e.g.
// a smeared noise, instead of being regenerated from the counter stream
constexpr int SRC_STORED = 100;

struct SourceSpec {
    int kind;         // DL_SRC_Z2 / DL_SRC_POINT / SRC_STORED
    int scheme;       // dilution bits
    uint64_t seed;
    int64_t V;
    int T;            // time extent (time dilution: noise n lives on timeslice n mod T)
    int point_site;
    const int64_t *noise;  // [nrhs] noise number of each right-hand side (device)
    const int *cls;        // [nrhs] dilution class (device); point: 3*spin + colour
    Field xe = {nullptr, nullptr}, xo = {nullptr, nullptr};  // SRC_STORED: FP64 source per parity
};
void k_source(int prec, Field dst, int parity, const SourceSpec &src, const Geom &g, int nrhs, hipStream_t s);
// C[rhs][t][4][4] (complex) = sum_{x in t} sum_c conj(eta_{a c}(x)) s_{b c}(x)
void k_trace(int prec, Field se, Field so, const SourceSpec &src, const Geom &g, int nrhs, double *C,
             hipStream_t s);
// loops[n][g][t] = sum_{d} sum_{ab} Gamma_g[a][b] C[n*ncls + d][t][a][b]
// one step of gauge-covariant Gaussian smearing on both parities (FP64 fields,
// FP64 links [4][2][NE][Vh]): out = (in + alpha H in) / (1 + 6 alpha), H the
// spatial, spin-diagonal hopping term; in and out must not overlap
void k_smear(const void *links, int recon, Field ine, Field ino, Field oute, Field outo, const Geom &g, int nrhs,
             double alpha, hipStream_t s);
// disconnected correlator: out[dt] = -norm * sum over distinct noise pairs (sb, sa: [T] complex scratch)
// Eqs. 3-4 (dl_fit.cpp): the flavour-singlet combination and the ratio fit
void eta_prime_fit(const double *d, const double *c, int ncfg, int T, double m_pi, int tmin, int tmax, double *c_eta,
                   double *params, double *errors, double *chi2);
void k_correlator(const double *lb, const double *la, double *sb, double *sa, int n, int T, double norm, double *out,
                  hipStream_t s);
void k_gamma_contract(const double *C, int n_noise, int ncls, int T, const double *gam, const int *gidx,
                      int n_gamma, double *loops, hipStream_t s);
// adjoint source dst(x) = A[noise - first_noise][t(x)] eta(x), A as [noise][T][4][4] complex (FP64 field)
void k_adjoint_source(Field dst, int parity, const SourceSpec &src, const Geom &g, int nrhs, const double *A,
                      int64_t first_noise, hipStream_t s);
// grad [4][V][3][3] complex += link gradient of Re sum conj(W) L from forward
// solutions s and adjoint solutions a' (a = gamma5 a'), all FP64 parity fields
void k_link_grad(Field se, Field so, Field ae, Field ao, const Geom &g, int nrhs, double kappa, double *grad,
                 hipStream_t s);
// canonical device links [4][V][3][3] complex128 -> [4][2][9][Vh] complex128 (parity split)
void k_links_reorder(const double *canon, double *dst, const Geom &g, hipStream_t s);
// links canonical (host-reordered to [4][2][9][Vh] complex128 on the device) -> storage format
void k_links_convert(int prec, void *dst, int ne, const double *src64, int64_t Vh, hipStream_t s);

}  // namespace dl
