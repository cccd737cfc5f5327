// dl_api.cpp -- the C ABI: handles, validation, the even-odd solver drivers
// (BiCGStab with FP64 reliable updates, truncated CGNR) and the loop
// estimator.  Every step of the computation runs in the library's kernels;
// the host only orders launches, polls convergence flags and moves results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "dl_internal.hpp"

using namespace dl;

// ====================================================================== errors

namespace dl {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace dl

template <typename F>
static int guarded(F &&f)
{
    try {
        g_err.clear();
        return f();
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return DL_ENOMEM;
    } catch (...) {
        g_err = "unexpected internal error";
        return DL_EHIP;
    }
}

// ====================================================================== buffers

namespace dl {

void DevBuf::alloc(size_t n)
{
    release();
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Error{DL_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e)};
    }
    bytes = n;
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

void HalfField::alloc(int prec_, int64_t nrhs_, int64_t Vh_)
{
    prec = prec_;
    nrhs = nrhs_;
    Vh = Vh_;
    data.alloc((size_t)nrhs * 12 * Vh * elem_bytes(prec));
    if (prec == P16)
        nrm.alloc((size_t)nrhs * Vh * sizeof(float));
    else
        nrm.release();
}

Field HalfField::view_rhs(int64_t r) const
{
    Field f;
    f.d = static_cast<char *>(data.p) + (size_t)r * 12 * Vh * elem_bytes(prec);
    f.nrm = nrm.p ? nrm.as<float>() + r * Vh : nullptr;
    return f;
}

// ====================================================================== profiling

static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct ProfRec {
    int kind;
    double bytes;
    hipEvent_t e0, e1;
};
static std::vector<ProfRec> g_prof_pending;
static double g_prof_ms[PROF_NKIND], g_prof_bytes[PROF_NKIND];
static int64_t g_prof_n[PROF_NKIND];

ProfScope::ProfScope(int kind_, double bytes_, hipStream_t s_) : kind(kind_), bytes(bytes_), s(s_)
{
    if (!g_prof_on) return;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        e0 = e1 = nullptr;
        return;
    }
    (void)hipEventRecord(e0, s);
}

ProfScope::~ProfScope()
{
    if (!e0) return;
    (void)hipEventRecord(e1, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({kind, bytes, e0, e1});
}

static void prof_drain()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_pending) {
        float ms = 0;
        if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            g_prof_ms[r.kind] += ms;
            g_prof_bytes[r.kind] += r.bytes;
            g_prof_n[r.kind] += 1;
        }
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_prof_pending.clear();
}

// ====================================================================== dslash launch

int dslash_site_blocks(const Geom &g, int /*prec*/, int /*nrhs*/) { return (g.Vh + 63) / 64; }

template <typename S>
void launch_dslash_t(const DslashCall &c, int nr, int bs, hipStream_t s);

// algorithmic bytes of one launch: every operand moved once
static double dslash_bytes(const DslashCall &c)
{
    const double vh = c.g.Vh, e = (double)elem_bytes(c.prec), nrm = c.prec == P16 ? 4.0 : 0.0;
    const double field = vh * (12 * e + nrm) * c.nrhs;
    const double links = vh * 8.0 * (c.recon == 12 ? 6 : 9) * e;
    int nfield = 2;  // in, out
    if (c.epi != EPI_PLAIN) nfield += 1;                                        // x
    if (c.epi == EPI_XPAY_DOT || c.epi == EPI_XMY_NRM) nfield += 1;             // y
    return nfield * field + links;
}

struct TuneChoice {
    int nr, bs;
};
TuneChoice tune_lookup(const DslashCall &c, hipStream_t s);

int launch_dslash(const DslashCall &c, hipStream_t s)
{
    TuneChoice t = tune_lookup(c, s);
    ProfScope ps(PROF_DSLASH, dslash_bytes(c), s);
    switch (c.prec) {
    case P64: launch_dslash_t<double>(c, t.nr, t.bs, s); break;
    case P32: launch_dslash_t<float>(c, t.nr, t.bs, s); break;
    case P16: launch_dslash_t<__half>(c, t.nr, t.bs, s); break;
    default: launch_dslash_t<__hip_bfloat16>(c, t.nr, t.bs, s); break;
    }
    return (c.g.Vh + t.bs - 1) / t.bs;
}

// default launch configuration (the autotuner refines it when enabled)
TuneChoice tune_lookup(const DslashCall &c, hipStream_t)
{
    (void)c;
    return TuneChoice{1, 256};
}

}  // namespace dl

// ====================================================================== lattice

dl::Geom dl_lattice_s::geom() const
{
    Geom g;
    g.X = dims[0];
    g.Y = dims[1];
    g.Z = dims[2];
    g.T = dims[3];
    g.Xh = dims[0] / 2;
    g.Vh = (int)Vh;
    g.sY = g.Xh;
    g.sZ = g.Xh * g.Y;
    g.sT = g.Xh * g.Y * g.Z;
    g.tap = tap;
    return g;
}

extern "C" const char *dl_last_error(void) { return g_err.c_str(); }

extern "C" const char *dl_version(void) { return "dloops 0.1 (gfx950)"; }

extern "C" int dl_lattice_create(const int32_t dims[4], int32_t t_antiperiodic, dl_lattice *out)
{
    return guarded([&]() {
        DL_REQUIRE(dims != nullptr && out != nullptr, "dl_lattice_create: null pointer");
        int64_t V = 1;
        for (int mu = 0; mu < 4; ++mu) {
            DL_REQUIRE(dims[mu] >= 2 && dims[mu] % 2 == 0,
                       "dl_lattice_create: every extent must be even and >= 2 (got " + std::to_string(dims[mu]) + ")");
            V *= dims[mu];
        }
        DL_REQUIRE(V <= 0x7fffffff, "dl_lattice_create: volume exceeds 2^31 - 1");
        auto *L = new dl_lattice_s;
        std::memcpy(L->dims, dims, sizeof(L->dims));
        L->tap = t_antiperiodic ? 1 : 0;
        L->V = V;
        L->Vh = V / 2;
        *out = L;
        return DL_OK;
    });
}

extern "C" void dl_lattice_destroy(dl_lattice lat) { delete lat; }

extern "C" int64_t dl_lattice_volume(dl_lattice lat) { return lat ? lat->V : 0; }

// ====================================================================== gauge field

extern "C" int dl_gauge_create(dl_lattice lat, const double *links, uint32_t prec_mask, int32_t recon, void *stream,
                               dl_gauge *out)
{
    return guarded([&]() {
        DL_REQUIRE(lat && links && out, "dl_gauge_create: null pointer");
        DL_REQUIRE((prec_mask & 0xF) != 0 && (prec_mask & ~0xFu) == 0, "dl_gauge_create: prec_mask must be a "
                                                                        "non-empty subset of bits 0..3");
        DL_REQUIRE(recon == 12 || recon == 18, "dl_gauge_create: recon must be 12 or 18");
        hipStream_t s = static_cast<hipStream_t>(stream);
        auto G = std::make_unique<dl_gauge_s>();
        G->lat = *lat;
        G->recon = recon;
        G->prec_mask = prec_mask;
        const Geom g = G->lat.geom();
        const int64_t V = G->lat.V, Vh = G->lat.Vh;
        // host reorder: canonical [mu][V][3][3] -> [mu][parity][9][Vh]
        std::vector<double> re((size_t)4 * 2 * 9 * Vh * 2);
        for (int64_t i = 0; i < V; ++i) {
            int64_t r = i;
            const int x = (int)(r % g.X);
            r /= g.X;
            const int y = (int)(r % g.Y);
            r /= g.Y;
            const int z = (int)(r % g.Z);
            const int t = (int)(r / g.Z);
            const int par = (x + y + z + t) & 1;
            const int64_t cb = i >> 1;
            for (int mu = 0; mu < 4; ++mu)
                for (int e = 0; e < 9; ++e) {
                    const double *src = links + (((int64_t)mu * V + i) * 9 + e) * 2;
                    double *dst = re.data() + ((((int64_t)mu * 2 + par) * 9 + e) * Vh + cb) * 2;
                    dst[0] = src[0];
                    dst[1] = src[1];
                }
        }
        DevBuf stage(re.size() * sizeof(double));
        DL_HIP(hipMemcpyAsync(stage.p, re.data(), stage.bytes, hipMemcpyHostToDevice, s));
        const int ne = recon == 12 ? 6 : 9;
        for (int p = 0; p < 4; ++p) {
            if (!(prec_mask & (1u << p))) continue;
            G->links[p].alloc((size_t)4 * 2 * ne * Vh * elem_bytes(p));
            k_links_convert(p, G->links[p].p, ne, stage.as<double>(), Vh, s);
        }
        DL_HIP(hipGetLastError());
        DL_HIP(hipStreamSynchronize(s));
        *out = G.release();
        return DL_OK;
    });
}

extern "C" void dl_gauge_destroy(dl_gauge g) { delete g; }

// ====================================================================== gamma matrices

// Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3 in the chiral basis, as [16][4][4][re,im]
static std::vector<double> gamma_table()
{
    using C = std::complex<double>;
    const C I(0, 1);
    C sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    C gm[4][4][4] = {};
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                gm[k][r][2 + c] = -I * sig[k][r][c];
                gm[k][2 + r][c] = I * sig[k][r][c];
            }
    for (int r = 0; r < 2; ++r) gm[3][r][2 + r] = gm[3][2 + r][r] = 1;
    std::vector<double> out(16 * 32);
    for (int n = 0; n < 16; ++n) {
        C G[4][4] = {};
        for (int a = 0; a < 4; ++a) G[a][a] = 1;
        for (int mu = 0; mu < 4; ++mu) {
            if (!((n >> mu) & 1)) continue;
            C H[4][4] = {};
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    for (int k = 0; k < 4; ++k) H[a][b] += G[a][k] * gm[mu][k][b];
            std::memcpy(G, H, sizeof(G));
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                out[n * 32 + 2 * (4 * a + b)] = G[a][b].real();
                out[n * 32 + 2 * (4 * a + b) + 1] = G[a][b].imag();
            }
    }
    return out;
}

// ====================================================================== operators

namespace {

struct Ctx {
    dl_gauge G;
    Geom g;
    hipStream_t s;
    const void *links(int prec) const { return G->links[prec].p; }
};

DslashCall dcall(const Ctx &c, int prec, int parity, bool dag, int epi, Field in, Field out, Field x, Field y,
                 double a, int nrhs, double *parts, const int *active)
{
    DslashCall d;
    d.g = c.g;
    d.parity = parity;
    d.prec = prec;
    d.recon = c.G->recon;
    d.dag = dag;
    d.epi = epi;
    d.in = in;
    d.out = out;
    d.x = x;
    d.y = y;
    d.links = c.links(prec);
    d.a = a;
    d.nrhs = nrhs;
    d.partials = parts;
    d.active = active;
    return d;
}

const Field NOF = {nullptr, nullptr};

void check_prec(dl_gauge G, int prec)
{
    DL_REQUIRE(prec >= 0 && prec <= 3, "precision must be one of DL_F64, DL_F32, DL_F16, DL_BF16");
    DL_REQUIRE((G->prec_mask >> prec) & 1, "the gauge handle does not hold links in the requested precision");
}

}  // namespace

extern "C" int dl_apply(dl_gauge G, double kappa, int32_t op, int32_t prec, const void *in, void *out, int64_t nrhs,
                        void *stream)
{
    return guarded([&]() {
        DL_REQUIRE(G && in && out, "dl_apply: null pointer");
        DL_REQUIRE(nrhs >= 1 && nrhs <= 65535, "dl_apply: nrhs must be in [1, 65535]");
        DL_REQUIRE(op >= DL_OP_DHOP && op <= DL_OP_DHOPDAG, "dl_apply: unknown operator");
        check_prec(G, prec);
        DL_REQUIRE(in != out, "dl_apply: in and out must not overlap");
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        const int n = (int)nrhs;
        const int64_t Vh = G->lat.Vh;
        HalfField ie, io, oe, oo, tmp;
        ie.alloc(prec, n, Vh);
        io.alloc(prec, n, Vh);
        oe.alloc(prec, n, Vh);
        oo.alloc(prec, n, Vh);
        k_pack(prec, ie.view(), 0, static_cast<const double *>(in), c.g, n, c.s);
        k_pack(prec, io.view(), 1, static_cast<const double *>(in), c.g, n, c.s);
        const bool dag = op == DL_OP_MDAG || op == DL_OP_MHATDAG || op == DL_OP_DHOPDAG;
        switch (op) {
        case DL_OP_DHOP:
        case DL_OP_DHOPDAG:
            launch_dslash(dcall(c, prec, 0, dag, EPI_PLAIN, io.view(), oe.view(), NOF, NOF, 1.0, n, nullptr, nullptr),
                          c.s);
            launch_dslash(dcall(c, prec, 1, dag, EPI_PLAIN, ie.view(), oo.view(), NOF, NOF, 1.0, n, nullptr, nullptr),
                          c.s);
            break;
        case DL_OP_M:
        case DL_OP_MDAG:
            launch_dslash(
                dcall(c, prec, 0, dag, EPI_XPAY, io.view(), oe.view(), ie.view(), NOF, -kappa, n, nullptr, nullptr),
                c.s);
            launch_dslash(
                dcall(c, prec, 1, dag, EPI_XPAY, ie.view(), oo.view(), io.view(), NOF, -kappa, n, nullptr, nullptr),
                c.s);
            break;
        default:  // Schur complement on even sites
            tmp.alloc(prec, n, Vh);
            launch_dslash(dcall(c, prec, 1, dag, EPI_PLAIN, ie.view(), tmp.view(), NOF, NOF, 1.0, n, nullptr, nullptr),
                          c.s);
            launch_dslash(dcall(c, prec, 0, dag, EPI_XPAY, tmp.view(), oe.view(), ie.view(), NOF, -kappa * kappa, n,
                                nullptr, nullptr),
                          c.s);
            k_zero(prec, oo.view(), Vh, n, nullptr, c.s);
            break;
        }
        k_unpack(prec, oe.view(), 0, static_cast<double *>(out), c.g, n, c.s);
        k_unpack(prec, oo.view(), 1, static_cast<double *>(out), c.g, n, c.s);
        DL_HIP(hipGetLastError());
        DL_HIP(hipStreamSynchronize(c.s));
        return DL_OK;
    });
}

// ====================================================================== solvers

namespace {

// Workspace of a batched solve.  Sources b_e, b_o and the FP64 solution x_e,
// x_o live in FP64 for tolerance-driven solves; the Krylov vectors live in
// the iteration precision.
struct SolveWork {
    int n = 0;
    int prec = P64;
    HalfField be, bo, bhat, x64, xo, r64, tmp64;     // FP64 (BiCGStab)
    HalfField r, rh, p, v, t, tmpo, xlo;             // iteration precision
    DevBuf st, act, upd, restart, parts, parts2;
    int nblk_max = 0;

    void alloc_bicg(int prec_, int n_, int64_t Vh)
    {
        prec = prec_;
        n = n_;
        be.alloc(P64, n, Vh);
        bo.alloc(P64, n, Vh);
        bhat.alloc(P64, n, Vh);
        x64.alloc(P64, n, Vh);
        xo.alloc(P64, n, Vh);
        r64.alloc(P64, n, Vh);
        tmp64.alloc(P64, n, Vh);
        r.alloc(prec, n, Vh);
        rh.alloc(prec, n, Vh);
        p.alloc(prec, n, Vh);
        v.alloc(prec, n, Vh);
        t.alloc(prec, n, Vh);
        tmpo.alloc(prec, n, Vh);
        if (prec != P64) xlo.alloc(prec, n, Vh);
        alloc_common(Vh);
    }
    // truncated CGNR in one precision: be, bo, bhat, x(x64 slot), xo, r, p, t(=q), v(=t), tmpo
    void alloc_cgnr(int prec_, int n_, int64_t Vh)
    {
        prec = prec_;
        n = n_;
        be.alloc(prec, n, Vh);
        bo.alloc(prec, n, Vh);
        bhat.alloc(prec, n, Vh);
        x64.alloc(prec, n, Vh);
        xo.alloc(prec, n, Vh);
        r.alloc(prec, n, Vh);
        p.alloc(prec, n, Vh);
        v.alloc(prec, n, Vh);
        t.alloc(prec, n, Vh);
        tmpo.alloc(prec, n, Vh);
        alloc_common(Vh);
    }
    void alloc_common(int64_t Vh)
    {
        nblk_max = (int)((Vh + 63) / 64);
        st.alloc(sizeof(KState) * n);
        act.alloc(sizeof(int) * n);
        upd.alloc(sizeof(int) * n);
        restart.alloc(sizeof(int) * n);
        parts.alloc(sizeof(double) * 3 * (size_t)n * nblk_max);
        parts2.alloc(sizeof(double) * 3 * (size_t)n * nblk_max);
    }
    static size_t bytes_bicg(int prec, int64_t Vh)
    {
        size_t f64 = 12 * 16 * Vh, fl = 12 * elem_bytes(prec) * Vh + (prec == P16 ? 4 * Vh : 0);
        return 7 * f64 + (prec == P64 ? 6 : 7) * fl + 6 * 8 * ((Vh + 63) / 64) + 256;
    }
    static size_t bytes_cgnr(int prec, int64_t Vh)
    {
        size_t fl = 12 * elem_bytes(prec) * Vh + (prec == P16 ? 4 * Vh : 0);
        return 10 * fl + 6 * 8 * ((Vh + 63) / 64) + 256;
    }
};

int parse_poll(const dl_solve_params &prm) { return prm.poll > 0 ? prm.poll : 4; }

int count_host(const DevBuf &flags, int n, hipStream_t s, std::vector<int> &h)
{
    h.resize(n);
    DL_HIP(hipMemcpyAsync(h.data(), flags.p, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    int c = 0;
    for (int v : h) c += v != 0;
    return c;
}

// BiCGStab on the even-site Schur system for w.n right-hand sides whose
// sources are in w.be / w.bo (FP64).  Leaves x_e in w.x64 and x_o in w.xo
// and the per right-hand side state in w.st.  Iterated vectors in w.prec;
// below FP64 the iterate is folded into the FP64 x and the residual
// recomputed in FP64 whenever |r| drops by delta since the last update.
void bicgstab_batch(const Ctx &c, double kappa, const dl_solve_params &prm, SolveWork &w)
{
    const int n = w.n, P = w.prec;
    const bool mixed = P != P64;
    const int64_t Vh = c.g.Vh;
    const int nb = blas_blocks(Vh);
    KState *st = w.st.as<KState>();
    int *act = w.act.as<int>(), *upd = w.upd.as<int>(), *rst = w.restart.as<int>();
    double *parts = w.parts.as<double>(), *parts2 = w.parts2.as<double>();
    const double k2 = kappa * kappa;
    const double delta = mixed ? (prm.delta > 0 ? prm.delta : 0.1) : 0.0;
    Field xit = mixed ? w.xlo.view() : w.x64.view();

    // |b|^2 over both parities; bhat = b_e + kappa D_eo b_o
    k_norm2_parts(P64, w.be.view(), Vh, n, nullptr, parts, c.s);
    k_norm2_parts(P64, w.bo.view(), Vh, n, nullptr, parts2, c.s);
    k_bicg_init(st, act, upd, n, parts, parts2, nb, prm.tol * prm.tol, delta * delta, prm.maxiter, c.s);
    launch_dslash(dcall(c, P64, 0, false, EPI_XPAY, w.bo.view(), w.bhat.view(), w.be.view(), NOF, kappa, n, nullptr,
                        nullptr),
                  c.s);
    k_zero(P64, w.x64.view(), Vh, n, nullptr, c.s);
    if (mixed) k_zero(P, w.xlo.view(), Vh, n, nullptr, c.s);
    k_copy(P, w.r.view(), P64, w.bhat.view(), Vh, n, nullptr, c.s);
    k_copy(P, w.rh.view(), P, w.r.view(), Vh, n, nullptr, c.s);
    k_zero(P, w.p.view(), Vh, n, nullptr, c.s);
    k_zero(P, w.v.view(), Vh, n, nullptr, c.s);
    k_dot_parts(P, w.rh.view(), w.r.view(), Vh, n, nullptr, parts, c.s);
    k_bicg_rho(st, act, upd, nullptr, n, parts, nb, 2, 1, mixed, c.s);

    const int poll = parse_poll(prm);
    std::vector<int> h;
    int it = 0;
    const int cap = prm.maxiter + 8;
    while (it < cap) {
        for (int k = 0; k < poll; ++k, ++it) {
            k_bicg_p(P, w.p.view(), w.r.view(), w.v.view(), st, act, Vh, n, c.s);
            launch_dslash(dcall(c, P, 1, false, EPI_PLAIN, w.p.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, act),
                          c.s);
            int nbd = launch_dslash(dcall(c, P, 0, false, EPI_XPAY_DOT, w.tmpo.view(), w.v.view(), w.p.view(),
                                          w.rh.view(), -k2, n, parts, act),
                                    c.s);
            k_bicg_alpha(st, act, n, parts, nbd, c.s);
            k_bicg_s(P, w.r.view(), w.v.view(), st, act, Vh, n, c.s);
            launch_dslash(dcall(c, P, 1, false, EPI_PLAIN, w.r.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, act),
                          c.s);
            nbd = launch_dslash(dcall(c, P, 0, false, EPI_XPAY_TS, w.tmpo.view(), w.t.view(), w.r.view(), NOF, -k2, n,
                                      parts, act),
                                c.s);
            k_bicg_omega(st, act, n, parts, nbd, c.s);
            k_bicg_xr(P, xit, w.r.view(), w.p.view(), w.t.view(), w.rh.view(), st, act, Vh, n, parts, c.s);
            k_bicg_rho(st, act, upd, nullptr, n, parts, nb, 3, 0, mixed, c.s);
            // reliable update / convergence check for the flagged right-hand sides:
            // fold the iterate, recompute r = bhat - Mhat x in FP64
            if (mixed) k_fold_x(w.x64.view(), P, w.xlo.view(), Vh, n, upd, c.s);
            launch_dslash(
                dcall(c, P64, 1, false, EPI_PLAIN, w.x64.view(), w.tmp64.view(), NOF, NOF, 1.0, n, nullptr, upd), c.s);
            int nb64 = launch_dslash(dcall(c, P64, 0, false, EPI_XMY_NRM, w.tmp64.view(), w.r64.view(), w.bhat.view(),
                                           w.x64.view(), k2, n, parts2, upd),
                                     c.s);
            k_copy(P, w.r.view(), P64, w.r64.view(), Vh, n, upd, c.s);
            k_true_residual(st, act, upd, rst, n, parts2, nullptr, nb64, 0, c.s);
            // restart the recursion where the true residual disagreed with the iterated one
            k_copy(P, w.rh.view(), P, w.r.view(), Vh, n, rst, c.s);
            k_zero(P, w.p.view(), Vh, n, rst, c.s);
            k_zero(P, w.v.view(), Vh, n, rst, c.s);
            k_dot_parts(P, w.rh.view(), w.r.view(), Vh, n, rst, parts, c.s);
            k_bicg_rho(st, act, upd, rst, n, parts, nb, 2, 1, mixed, c.s);
        }
        DL_HIP(hipGetLastError());
        if (count_host(w.act, n, c.s, h) == 0) break;
    }
    // x_o = b_o + kappa D_oe x_e
    launch_dslash(
        dcall(c, P64, 1, false, EPI_XPAY, w.x64.view(), w.xo.view(), w.bo.view(), NOF, kappa, n, nullptr, nullptr),
        c.s);
}

// Full-lattice FP64 true residual |b - M x|^2 per right-hand side into out[n].
void true_residual_full(const Ctx &c, double kappa, SolveWork &w, std::vector<double> &out)
{
    const int n = w.n;
    double *parts = w.parts.as<double>(), *parts2 = w.parts2.as<double>();
    // r_e = b_e - x_e + kappa D_eo x_o ; r_o = b_o - x_o + kappa D_oe x_e
    int nbd = launch_dslash(dcall(c, P64, 0, false, EPI_XMY_NRM, w.xo.view(), w.r64.view(), w.be.view(), w.x64.view(),
                                  kappa, n, parts, nullptr),
                            c.s);
    launch_dslash(dcall(c, P64, 1, false, EPI_XMY_NRM, w.x64.view(), w.tmp64.view(), w.bo.view(), w.xo.view(), kappa,
                        n, parts2, nullptr),
                  c.s);
    DevBuf sums(sizeof(double) * 2 * n);
    k_sum_parts(parts, n, nbd, 1, sums.as<double>(), c.s);
    k_sum_parts(parts2, n, nbd, 1, sums.as<double>() + n, c.s);
    std::vector<double> h(2 * n);
    DL_HIP(hipMemcpyAsync(h.data(), sums.p, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, c.s));
    DL_HIP(hipStreamSynchronize(c.s));
    out.resize(n);
    for (int i = 0; i < n; ++i) out[i] = h[i] + h[n + i];
}

// Truncated CGNR (x0 = 0, exactly `iters` iterations) on the normal equations
// of the even-site Schur system, all in precision w.prec; sources in w.be /
// w.bo (same precision).  x_e -> w.x64 (slot), x_o -> w.xo.
void cgnr_batch(const Ctx &c, double kappa, int iters, SolveWork &w)
{
    const int n = w.n, P = w.prec;
    const int64_t Vh = c.g.Vh;
    const int nb = blas_blocks(Vh);
    KState *st = w.st.as<KState>();
    int *act = w.act.as<int>();
    double *parts = w.parts.as<double>();
    const double k2 = kappa * kappa;
    // bhat = b_e + kappa D_eo b_o ; r = Mhat^+ bhat ; x = 0 ; p = r
    launch_dslash(
        dcall(c, P, 0, false, EPI_XPAY, w.bo.view(), w.bhat.view(), w.be.view(), NOF, kappa, n, nullptr, nullptr),
        c.s);
    launch_dslash(dcall(c, P, 1, true, EPI_PLAIN, w.bhat.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, nullptr),
                  c.s);
    int nbd = launch_dslash(
        dcall(c, P, 0, true, EPI_XPAY_NRM, w.tmpo.view(), w.r.view(), w.bhat.view(), NOF, -k2, n, parts, nullptr), c.s);
    k_cg_init(st, act, n, parts, nbd, iters, c.s);
    k_zero(P, w.x64.view(), Vh, n, nullptr, c.s);
    k_copy(P, w.p.view(), P, w.r.view(), Vh, n, nullptr, c.s);
    for (int it = 0; it < iters; ++it) {
        // t = Mhat p ; q = Mhat^+ t with partial (p, q)
        launch_dslash(dcall(c, P, 1, false, EPI_PLAIN, w.p.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, act),
                      c.s);
        launch_dslash(
            dcall(c, P, 0, false, EPI_XPAY, w.tmpo.view(), w.t.view(), w.p.view(), NOF, -k2, n, nullptr, act), c.s);
        launch_dslash(dcall(c, P, 1, true, EPI_PLAIN, w.t.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, act), c.s);
        nbd = launch_dslash(
            dcall(c, P, 0, true, EPI_XPAY_DOT, w.tmpo.view(), w.v.view(), w.t.view(), w.p.view(), -k2, n, parts, act),
            c.s);
        k_cg_alpha(st, act, n, parts, nbd, c.s);
        k_cg_xr(P, w.x64.view(), w.r.view(), w.p.view(), w.v.view(), st, act, Vh, n, parts, c.s);
        k_cg_beta(st, act, n, parts, nb, c.s);
        k_cg_p(P, w.p.view(), w.r.view(), st, act, Vh, n, c.s);
    }
    launch_dslash(
        dcall(c, P, 1, false, EPI_XPAY, w.x64.view(), w.xo.view(), w.bo.view(), NOF, kappa, n, nullptr, nullptr), c.s);
    DL_HIP(hipGetLastError());
}

void validate_params(const dl_solve_params *prm)
{
    DL_REQUIRE(prm != nullptr, "solve parameters: null pointer");
    DL_REQUIRE(prm->solver == DL_BICGSTAB || prm->solver == DL_CGNR, "solve parameters: unknown solver");
    DL_REQUIRE(prm->prec >= 0 && prm->prec <= 3, "solve parameters: unknown precision");
    if (prm->solver == DL_CGNR) {
        DL_REQUIRE(prm->fixed_iters >= 0, "solve parameters: CGNR needs fixed_iters >= 0");
    } else {
        DL_REQUIRE(prm->fixed_iters == 0, "solve parameters: BiCGStab is tolerance driven (fixed_iters must be 0)");
        DL_REQUIRE(prm->tol > 0 && prm->tol < 1, "solve parameters: tol must be in (0, 1)");
        DL_REQUIRE(prm->maxiter >= 1, "solve parameters: maxiter must be >= 1");
    }
    DL_REQUIRE(prm->delta >= 0 && prm->delta < 1, "solve parameters: delta must be in [0, 1)");
}

size_t workspace_limit()
{
    const char *e = std::getenv("DL_WORKSPACE_GB");
    double gb = e ? std::atof(e) : 160.0;
    if (!(gb > 0)) gb = 160.0;
    return (size_t)(gb * 1e9);
}

int batch_size(size_t per_rhs, int64_t total, int quantum)
{
    int64_t b = (int64_t)(workspace_limit() / std::max<size_t>(per_rhs, 1));
    b = std::min<int64_t>(b, 65535);
    b = std::max<int64_t>(b / quantum * quantum, quantum);
    return (int)std::min<int64_t>(b, total);
}

void fill_stats(const SolveWork &w, const std::vector<double> &res2, dl_solve_stats *out, hipStream_t s,
                bool cgnr)
{
    std::vector<KState> h(w.n);
    DL_HIP(hipMemcpyAsync(h.data(), w.st.p, sizeof(KState) * w.n, hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < w.n; ++i) {
        dl_solve_stats &o = out[i];
        o.iters = h[i].iters;
        o.reliable_updates = h[i].updates;
        o.pad = 0;
        const double b2 = h[i].b2;
        o.true_rel_residual = (i < (int)res2.size() && b2 > 0) ? std::sqrt(res2[i] / b2) : 0.0;
        if (h[i].nonfinite)
            o.status = DL_ENAN;
        else if (cgnr || h[i].done)
            o.status = DL_OK;
        else
            o.status = DL_ENOCONV;
    }
}

}  // namespace

extern "C" int dl_solve(dl_gauge G, double kappa, const dl_solve_params *params, const void *b, void *x, int64_t nrhs,
                        dl_solve_stats *stats, void *stream)
{
    return guarded([&]() {
        DL_REQUIRE(G && b && x, "dl_solve: null pointer");
        DL_REQUIRE(nrhs >= 1, "dl_solve: nrhs must be >= 1");
        DL_REQUIRE(b != x, "dl_solve: b and x must not overlap");
        validate_params(params);
        const dl_solve_params prm = *params;
        check_prec(G, prm.prec);
        if (prm.solver == DL_BICGSTAB) check_prec(G, P64);
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        const int64_t Vh = G->lat.Vh, V = G->lat.V;
        const bool cg = prm.solver == DL_CGNR;
        const size_t per = cg ? SolveWork::bytes_cgnr(prm.prec, Vh) : SolveWork::bytes_bicg(prm.prec, Vh);
        const int B = batch_size(per, nrhs, 1);
        int worst = DL_OK;
        for (int64_t r0 = 0; r0 < nrhs; r0 += B) {
            const int n = (int)std::min<int64_t>(B, nrhs - r0);
            SolveWork w;
            const double *bsrc = static_cast<const double *>(b) + r0 * V * 24;
            double *xdst = static_cast<double *>(x) + r0 * V * 24;
            std::vector<double> res2;
            if (cg) {
                w.alloc_cgnr(prm.prec, n, Vh);
                k_pack(prm.prec, w.be.view(), 0, bsrc, c.g, n, c.s);
                k_pack(prm.prec, w.bo.view(), 1, bsrc, c.g, n, c.s);
                cgnr_batch(c, kappa, prm.fixed_iters, w);
                k_unpack(prm.prec, w.x64.view(), 0, xdst, c.g, n, c.s);
                k_unpack(prm.prec, w.xo.view(), 1, xdst, c.g, n, c.s);
            } else {
                w.alloc_bicg(prm.prec, n, Vh);
                k_pack(P64, w.be.view(), 0, bsrc, c.g, n, c.s);
                k_pack(P64, w.bo.view(), 1, bsrc, c.g, n, c.s);
                bicgstab_batch(c, kappa, prm, w);
                true_residual_full(c, kappa, w, res2);
                k_unpack(P64, w.x64.view(), 0, xdst, c.g, n, c.s);
                k_unpack(P64, w.xo.view(), 1, xdst, c.g, n, c.s);
            }
            DL_HIP(hipGetLastError());
            DL_HIP(hipStreamSynchronize(c.s));
            std::vector<dl_solve_stats> st(n);
            fill_stats(w, res2, st.data(), c.s, cg);
            for (int i = 0; i < n; ++i) {
                if (stats) stats[r0 + i] = st[i];
                if (st[i].status != DL_OK && worst == DL_OK) worst = st[i].status;
            }
        }
        if (worst != DL_OK) g_err = "dl_solve: at least one right-hand side did not converge";
        return worst;
    });
}

// ====================================================================== loops

namespace {

int dilution_classes(int scheme)
{
    return ((scheme & DL_DIL_SPIN_COLOUR) ? 12 : 1) * ((scheme & DL_DIL_CUBIC) ? 8 : 1) *
           ((scheme & DL_DIL_EVEN_ODD) ? 2 : 1);
}

void validate_sources(const dl_lattice_s &lat, const dl_sources *src)
{
    DL_REQUIRE(src != nullptr, "sources: null pointer");
    DL_REQUIRE(src->kind == DL_SRC_Z2 || src->kind == DL_SRC_POINT, "sources: unknown kind");
    if (src->kind == DL_SRC_POINT) {
        DL_REQUIRE(src->n_noise == 1, "sources: point sources need n_noise = 1");
        DL_REQUIRE(src->point_site >= 0 && src->point_site < lat.V, "sources: point_site outside the lattice");
    } else {
        DL_REQUIRE(src->n_noise >= 1, "sources: n_noise must be >= 1");
        DL_REQUIRE(src->first_noise >= 0, "sources: first_noise must be >= 0");
        DL_REQUIRE((src->scheme & ~7) == 0, "sources: unknown dilution bits");
    }
}

int source_classes(const dl_sources *src) { return src->kind == DL_SRC_POINT ? 12 : dilution_classes(src->scheme); }

}  // namespace

extern "C" int64_t dl_sources_count(dl_lattice lat, const dl_sources *src)
{
    int64_t r = DL_EINVAL;
    int rc = guarded([&]() {
        DL_REQUIRE(lat != nullptr, "dl_sources_count: null lattice");
        validate_sources(*lat, src);
        r = (int64_t)src->n_noise * source_classes(src);
        return DL_OK;
    });
    return rc == DL_OK ? r : rc;
}

extern "C" int dl_sources_fill(dl_lattice lat, const dl_sources *src, int64_t first_rhs, int64_t nrhs, void *out,
                               void *stream)
{
    return guarded([&]() {
        DL_REQUIRE(lat && out, "dl_sources_fill: null pointer");
        validate_sources(*lat, src);
        const int ncls = source_classes(src);
        const int64_t total = (int64_t)src->n_noise * ncls;
        DL_REQUIRE(nrhs >= 1 && nrhs <= 65535 && first_rhs >= 0 && first_rhs + nrhs <= total,
                   "dl_sources_fill: right-hand side range outside the description");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom g = lat->geom();
        const int n = (int)nrhs;
        std::vector<int64_t> hnoise(n);
        std::vector<int> hcls(n);
        for (int i = 0; i < n; ++i) {
            hnoise[i] = src->first_noise + (first_rhs + i) / ncls;
            hcls[i] = (int)((first_rhs + i) % ncls);
        }
        DevBuf dnoise(sizeof(int64_t) * n), dcls(sizeof(int) * n);
        DL_HIP(hipMemcpyAsync(dnoise.p, hnoise.data(), dnoise.bytes, hipMemcpyHostToDevice, s));
        DL_HIP(hipMemcpyAsync(dcls.p, hcls.data(), dcls.bytes, hipMemcpyHostToDevice, s));
        SourceSpec ss;
        ss.kind = src->kind;
        ss.scheme = src->kind == DL_SRC_POINT ? 0 : src->scheme;
        ss.seed = src->seed;
        ss.V = lat->V;
        ss.point_site = src->point_site;
        ss.noise = dnoise.as<int64_t>();
        ss.cls = dcls.as<int>();
        HalfField fe, fo;
        fe.alloc(P64, n, lat->Vh);
        fo.alloc(P64, n, lat->Vh);
        k_source(P64, fe.view(), 0, ss, g, n, s);
        k_source(P64, fo.view(), 1, ss, g, n, s);
        k_unpack(P64, fe.view(), 0, static_cast<double *>(out), g, n, s);
        k_unpack(P64, fo.view(), 1, static_cast<double *>(out), g, n, s);
        DL_HIP(hipGetLastError());
        DL_HIP(hipStreamSynchronize(s));
        return DL_OK;
    });
}

extern "C" int dl_loops(dl_gauge G, double kappa, const dl_sources *src, const dl_solve_params *params,
                        const int32_t *gammas, int32_t n_gamma, double *loops, dl_solve_stats *stats, void *stream)
{
    return guarded([&]() {
        DL_REQUIRE(G && loops && gammas, "dl_loops: null pointer");
        validate_sources(G->lat, src);
        validate_params(params);
        DL_REQUIRE(n_gamma >= 1 && n_gamma <= 16, "dl_loops: n_gamma must be in [1, 16]");
        for (int i = 0; i < n_gamma; ++i)
            DL_REQUIRE(gammas[i] >= 0 && gammas[i] <= 15, "dl_loops: gamma index outside [0, 15]");
        const dl_solve_params prm = *params;
        check_prec(G, prm.prec);
        if (prm.solver == DL_BICGSTAB) check_prec(G, P64);
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        const int64_t Vh = G->lat.Vh;
        const int T = c.g.T;
        const int ncls = source_classes(src);
        const bool cg = prm.solver == DL_CGNR;
        const size_t per = (cg ? SolveWork::bytes_cgnr(prm.prec, Vh) : SolveWork::bytes_bicg(prm.prec, Vh)) +
                           (size_t)T * 32 * 8 + 16;
        const int64_t total = (int64_t)src->n_noise * ncls;
        const int B = batch_size(per, total, ncls);  // whole noises per batch
        // gamma table and indices
        std::vector<double> gtab = gamma_table();
        DevBuf dgam(gtab.size() * sizeof(double)), dgidx(sizeof(int) * n_gamma),
            dloops((size_t)src->n_noise * n_gamma * T * 2 * sizeof(double));
        DL_HIP(hipMemcpyAsync(dgam.p, gtab.data(), dgam.bytes, hipMemcpyHostToDevice, c.s));
        DL_HIP(hipMemcpyAsync(dgidx.p, gammas, dgidx.bytes, hipMemcpyHostToDevice, c.s));
        int worst = DL_OK;
        std::vector<int64_t> hnoise;
        std::vector<int> hcls;
        for (int64_t r0 = 0; r0 < total; r0 += B) {
            const int n = (int)std::min<int64_t>(B, total - r0);
            const int nn = n / ncls;
            hnoise.resize(n);
            hcls.resize(n);
            for (int i = 0; i < n; ++i) {
                hnoise[i] = src->first_noise + (r0 + i) / ncls;
                hcls[i] = (int)((r0 + i) % ncls);
            }
            DevBuf dnoise(sizeof(int64_t) * n), dcls(sizeof(int) * n), dC((size_t)n * T * 32 * sizeof(double));
            DL_HIP(hipMemcpyAsync(dnoise.p, hnoise.data(), dnoise.bytes, hipMemcpyHostToDevice, c.s));
            DL_HIP(hipMemcpyAsync(dcls.p, hcls.data(), dcls.bytes, hipMemcpyHostToDevice, c.s));
            SourceSpec ss;
            ss.kind = src->kind;
            ss.scheme = src->kind == DL_SRC_POINT ? 0 : src->scheme;
            ss.seed = src->seed;
            ss.V = G->lat.V;
            ss.point_site = src->point_site;
            ss.noise = dnoise.as<int64_t>();
            ss.cls = dcls.as<int>();
            SolveWork w;
            std::vector<double> res2;
            int sol_prec;
            if (cg) {
                w.alloc_cgnr(prm.prec, n, Vh);
                k_source(prm.prec, w.be.view(), 0, ss, c.g, n, c.s);
                k_source(prm.prec, w.bo.view(), 1, ss, c.g, n, c.s);
                cgnr_batch(c, kappa, prm.fixed_iters, w);
                sol_prec = prm.prec;
            } else {
                w.alloc_bicg(prm.prec, n, Vh);
                k_source(P64, w.be.view(), 0, ss, c.g, n, c.s);
                k_source(P64, w.bo.view(), 1, ss, c.g, n, c.s);
                bicgstab_batch(c, kappa, prm, w);
                if (stats) true_residual_full(c, kappa, w, res2);
                sol_prec = P64;
            }
            k_trace(sol_prec, w.x64.view(), w.xo.view(), ss, c.g, n, dC.as<double>(), c.s);
            k_gamma_contract(dC.as<double>(), nn, ncls, T, dgam.as<double>(), dgidx.as<int>(), n_gamma,
                             dloops.as<double>() + (r0 / ncls) * n_gamma * T * 2, c.s);
            DL_HIP(hipGetLastError());
            DL_HIP(hipStreamSynchronize(c.s));
            std::vector<dl_solve_stats> st(n);
            fill_stats(w, res2, st.data(), c.s, cg);
            for (int i = 0; i < n; ++i) {
                if (stats) stats[r0 + i] = st[i];
                if (st[i].status != DL_OK && worst == DL_OK) worst = st[i].status;
            }
        }
        DL_HIP(hipMemcpyAsync(loops, dloops.p, dloops.bytes, hipMemcpyDeviceToHost, c.s));
        DL_HIP(hipStreamSynchronize(c.s));
        if (worst != DL_OK) g_err = "dl_loops: at least one solve did not converge";
        return worst;
    });
}

// ====================================================================== profiling API

extern "C" int dl_profile_enable(int32_t on)
{
    prof_drain();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    for (int k = 0; k < PROF_NKIND; ++k) {
        g_prof_ms[k] = 0;
        g_prof_bytes[k] = 0;
        g_prof_n[k] = 0;
    }
    return DL_OK;
}

extern "C" int64_t dl_profile_read(int32_t kind, double *ms, double *bytes)
{
    if (kind < 0 || kind >= PROF_NKIND) return DL_EINVAL;
    prof_drain();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (ms) *ms = g_prof_ms[kind];
    if (bytes) *bytes = g_prof_bytes[kind];
    return g_prof_n[kind];
}
