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
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        release();
        p = o.p; bytes = o.bytes;
        o.p = nullptr; o.bytes = 0;
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t n);
    void release();
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

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

enum ProfKind { PROF_DSLASH = 0, PROF_BLAS = 1, PROF_TRACE = 2, PROF_DSLASH_PLAIN = 3, PROF_NKIND = 4 };
// Brackets a launch with events when profiling is on.  The algorithmic bytes
// of the launch are `bytes`, or, when `counter` is set, fixed_bytes (if any
// work ran) plus unit_bytes times the number of units the kernel counted
// into *counter divided by `units_div` (the hopping kernel counts live
// right-hand-side blocks, so masked-off right-hand sides move no bytes).
struct ProfScope {
    ProfScope(int kind, double bytes, hipStream_t s, int kind2 = -1);
    ~ProfScope();
    int kind, kind2;
    double bytes;
    hipStream_t s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    unsigned *counter = nullptr;
    double unit_bytes = 0, fixed_bytes = 0, units_div = 1;
};
// a zeroed device counter for the next profiled launch (null when profiling is off)
unsigned *prof_counter();
bool prof_on();

// ---------------------------------------------------------------- dslash

enum Epi {
    EPI_PLAIN = 0,     // out = a D in
    EPI_XPAY = 1,      // out = x + a D in
    EPI_XPAY_DOT = 2,  // out = x + a D in; partial (y, out)            [2 doubles]
    EPI_XPAY_TS = 3,   // out = x + a D in; partials (out, x), |out|^2   [3 doubles]
    EPI_XPAY_NRM = 4,  // out = x + a D in; partial |out|^2              [1 double]
    EPI_XMY_NRM = 5,   // out = x - y + a D in; partial |out|^2          [1 double]
};

inline int epi_nparts(int epi)
{
    switch (epi) {
    case EPI_XPAY_DOT: return 2;
    case EPI_XPAY_TS: return 3;
    case EPI_XPAY_NRM: return 1;
    case EPI_XMY_NRM: return 1;
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
};

// launch with the tuned (or default) configuration; returns the number of
// site blocks per right-hand side (the partials' middle extent)
int launch_dslash(const DslashCall &c, hipStream_t s);

// launch configuration of the hopping kernel: right-hand sides per thread and
// sites per workgroup
struct TuneChoice {
    int nr, bs;
};
TuneChoice tune_lookup(const DslashCall &c, hipStream_t s);
void launch_dslash_any(const DslashCall &c, int nr, int bs, hipStream_t s);
int dslash_site_blocks(const Geom &g, int prec, int nrhs);

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

// BiCGStab scalar updates (one wave per right-hand side)
void k_bicg_init(KState *st, int *act, int *upd, int nrhs, const double *b2_parts_e, const double *b2_parts_o,
                 int nblk, double tol2, double delta2, int maxiter, hipStream_t s);
// rho_new from partials (rhat, r) [, |r|^2]; first = 1 restarts the recursion for
// right-hand sides selected by mask (null = all); mixed enables reliable-update triggers
void k_bicg_rho(KState *st, int *act, int *upd, const int *mask, int nrhs, const double *parts, int nblk, int np,
                int first, int mixed, hipStream_t s);
void k_bicg_alpha(KState *st, const int *act, int nrhs, const double *parts, int nblk, hipStream_t s);
void k_bicg_omega(KState *st, const int *act, int nrhs, const double *parts, int nblk, hipStream_t s);
// after an FP64 residual recomputation for the right-hand sides flagged in upd
void k_true_residual(KState *st, int *act, int *upd, int *restart, int nrhs, const double *parts_e,
                     const double *parts_o, int nblk, int final_check, hipStream_t s);
// CGNR scalar updates
void k_cg_init(KState *st, int *act, int nrhs, const double *parts, int nblk, int iters, hipStream_t s);
void k_cg_alpha(KState *st, int *act, int nrhs, const double *parts, int nblk, hipStream_t s);
void k_cg_beta(KState *st, int *act, int nrhs, const double *parts, int nblk, hipStream_t s);
void k_sum_parts(const double *parts, int nrhs, int nblk, int nparts, double *out, hipStream_t s);

// vector kernels (fields in storage precision `prec`; masked by act)
void k_bicg_p(int prec, Field p, Field r, Field v, const KState *st, const int *act, int64_t Vh, int nrhs,
              hipStream_t s);
void k_bicg_s(int prec, Field r, Field v, const KState *st, const int *act, int64_t Vh, int nrhs, hipStream_t s);
void k_bicg_xr(int prec, Field x, Field r, Field p, Field t, Field rh, const KState *st, const int *act, int64_t Vh,
               int nrhs, double *parts, hipStream_t s);
void k_cg_xr(int prec, Field x, Field r, Field p, Field q, const KState *st, const int *act, int64_t Vh, int nrhs,
             double *parts, hipStream_t s);
void k_cg_p(int prec, Field p, Field r, const KState *st, const int *act, int64_t Vh, int nrhs, hipStream_t s);

// generic field kernels (mask: per right-hand side flags selecting who acts; null = all)
void k_copy(int prec_dst, Field dst, int prec_src, Field src, int64_t Vh, int nrhs, const int *mask, hipStream_t s);
void k_zero(int prec, Field f, int64_t Vh, int nrhs, const int *mask, hipStream_t s);
void k_fold_x(Field x64, int prec, Field xlo, int64_t Vh, int nrhs, const int *mask, hipStream_t s);
void k_norm2_parts(int prec, Field f, int64_t Vh, int nrhs, const int *mask, double *parts, hipStream_t s);
void k_dot_parts(int prec, Field a, Field b, int64_t Vh, int nrhs, const int *mask, double *parts, hipStream_t s);
void k_sub(Field dst, Field a, Field b, int64_t Vh, int nrhs, const int *mask, hipStream_t s);

// ---------------------------------------------------------------- fields, sources, traces

// canonical complex128 [nrhs][V][4][3] <-> parity fields
void k_pack(int prec, Field dst, int parity, const double *canon, const Geom &g, int nrhs, hipStream_t s);
void k_unpack(int prec, Field src, int parity, double *canon, const Geom &g, int nrhs, hipStream_t s);

struct SourceSpec {
    int kind;         // DL_SRC_Z2 / DL_SRC_POINT
    int scheme;       // dilution bits
    uint64_t seed;
    int64_t V;
    int point_site;
    const int64_t *noise;  // [nrhs] noise number of each right-hand side (device)
    const int *cls;        // [nrhs] dilution class (device); point: 3*spin + colour
};
void k_source(int prec, Field dst, int parity, const SourceSpec &src, const Geom &g, int nrhs, hipStream_t s);
// C[rhs][t][4][4] (complex) = sum_{x in t} sum_c conj(eta_{a c}(x)) s_{b c}(x)
void k_trace(int prec, Field se, Field so, const SourceSpec &src, const Geom &g, int nrhs, double *C,
             hipStream_t s);
// loops[n][g][t] = sum_{d} sum_{ab} Gamma_g[a][b] C[n*ncls + d][t][a][b]
void k_gamma_contract(const double *C, int n_noise, int ncls, int T, const double *gam, const int *gidx,
                      int n_gamma, double *loops, hipStream_t s);
// adjoint source dst(x) = A[noise - first_noise][t(x)] eta(x), A as [noise][T][4][4] complex (FP64 field)
void k_adjoint_source(Field dst, int parity, const SourceSpec &src, const Geom &g, int nrhs, const double *A,
                      int64_t first_noise, hipStream_t s);
// grad [4][V][3][3] complex += link gradient of Re sum conj(W) L from forward
// solutions s and adjoint solutions a' (a = gamma5 a'), all FP64 parity fields
void k_link_grad(Field se, Field so, Field ae, Field ao, const Geom &g, int nrhs, double kappa, double *grad,
                 hipStream_t s);
// links canonical (host-reordered to [4][2][9][Vh] complex128 on the device) -> storage format
void k_links_convert(int prec, void *dst, int ne, const double *src64, int64_t Vh, hipStream_t s);

}  // namespace dl
