// dl_fields.hip -- layout conversion (canonical <-> even-odd SoA, and the
// chiral spin basis <-> the stored basis of dl_common.hpp), noise and point
// sources with dilution masks, the timeslice trace reduction and the gamma
// contraction of the loops, and link-format conversion.
#include "dl_dslash.hpp"

namespace dl {

namespace {

constexpr int BS = 256;

__device__ __forceinline__ int64_t lex_index(const Geom &g, const Site &s)
{
    return s.x + (int64_t)g.X * (s.y + (int64_t)g.Y * (s.z + (int64_t)g.Z * s.t));
}

// ---------------------------------------------------------------- noise

// SplitMix64 (Steele, Lea and Flood, 2014): the stream seeded with `seed`
// adds the odd constant 0x9e3779b97f4a7c15 to its state before every output
// and returns the state passed through a two-round xor-shift-multiply
// finaliser.  Output number n (from 0) therefore only needs the state
// seed + (n + 1) * constant, which makes every noise entry independent.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// class of entry (site, spin, colour) under the dilution bits
__device__ __forceinline__ int dil_class(int scheme, const Site &s, int spin, int col)
{
    int d = 0;
    if (scheme & DL_DIL_SPIN_COLOUR) d = d * 12 + 3 * spin + col;
    if (scheme & DL_DIL_SPIN) d = d * 4 + spin;
    if (scheme & DL_DIL_SPIN_EVEN_ODD) d = d * 2 + (spin & 1);
    if (scheme & DL_DIL_COLOUR) d = d * 3 + col;
    if (scheme & DL_DIL_CUBIC) d = d * 8 + (s.x & 1) + 2 * (s.y & 1) + 4 * (s.z & 1);
    if (scheme & DL_DIL_EVEN_ODD) d = d * 2 + ((s.x + s.y + s.z + s.t) & 1);
    return d;
}

// source entries of one site for one right-hand side
__device__ __forceinline__ void source_site(const SourceSpec &src, int rhs, const Site &st, int64_t lex,
                                            cx<double> eta[12])
{
    const int cls = src.cls[rhs];
    if (src.kind == DL_SRC_POINT) {
#pragma unroll
        for (int e = 0; e < 12; ++e) eta[e] = {(lex == src.point_site && e == cls) ? 1.0 : 0.0, 0.0};
        return;
    }
    const double amp = 0.70710678118654752440;  // 1/sqrt(2)
    if ((src.scheme & DL_DIL_TIME) && st.t != (int)(src.noise[rhs] % src.T)) {
#pragma unroll
        for (int e = 0; e < 12; ++e) eta[e] = {0.0, 0.0};
        return;
    }
    const uint64_t base = ((uint64_t)src.noise[rhs] * (uint64_t)src.V + (uint64_t)lex) * 12ull;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int e = 3 * sp + c;
            if (src.scheme != 0 && dil_class(src.scheme, st, sp, c) != cls) {
                eta[e] = {0.0, 0.0};
                continue;
            }
            const uint64_t r = splitmix64_at(src.seed, base + (uint64_t)e);
            eta[e] = {(r & 1ull) ? -amp : amp, (r & 2ull) ? -amp : amp};
        }
}

// ---------------------------------------------------------------- kernels

template <typename S>
__global__ __launch_bounds__(BS) void pack_kernel(Field dst, int parity, const double *canon, Geom g)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    const int cb = blockIdx.x * BS + threadIdx.x;
    if (cb >= g.Vh) return;
    const Site s = decode(g, cb, parity);
    const int64_t V = 2 * (int64_t)g.Vh;
    const double2 *src = reinterpret_cast<const double2 *>(canon) + ((int64_t)rhs * V + lex_index(g, s)) * 12;
    cx<double> z[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) z[e] = {src[e].x, src[e].y};
    to_internal(z);
    cx<R> v[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) v[e] = {R(z[e].re), R(z[e].im)};
    store_spinor<S>(dst, g.Vh, rhs, cb, v);
}

template <typename S>
__global__ __launch_bounds__(BS) void unpack_kernel(Field src, int parity, double *canon, Geom g)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    const int cb = blockIdx.x * BS + threadIdx.x;
    if (cb >= g.Vh) return;
    const Site s = decode(g, cb, parity);
    const int64_t V = 2 * (int64_t)g.Vh;
    double2 *dst = reinterpret_cast<double2 *>(canon) + ((int64_t)rhs * V + lex_index(g, s)) * 12;
    cx<R> v[12];
    load_spinor<S>(src, g.Vh, rhs, cb, v);
    cx<double> z[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) z[e] = {(double)v[e].re, (double)v[e].im};
    to_canonical(z);
#pragma unroll
    for (int e = 0; e < 12; ++e) dst[e] = make_double2(z[e].re, z[e].im);
}

template <typename S>
__global__ __launch_bounds__(BS) void source_kernel(Field dst, int parity, SourceSpec src, Geom g)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    const int cb = blockIdx.x * BS + threadIdx.x;
    if (cb >= g.Vh) return;
    const Site s = decode(g, cb, parity);
    cx<double> eta[12];
    source_site(src, rhs, s, lex_index(g, s), eta);
    to_internal(eta);
    cx<R> v[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) v[e] = {R(eta[e].re), R(eta[e].im)};
    store_spinor<S>(dst, g.Vh, rhs, cb, v);
}

// One block per (timeslice, right-hand side); threads stride over the
// timeslice's sites of both parities and accumulate the 4x4 colour-traced
// spin matrix C[a][b] = sum_c conj(eta_{a c}) s_{b c} in FP64.
template <typename S>
__global__ __launch_bounds__(BS) void trace_kernel(Field se, Field so, SourceSpec src, Geom g, double *C)
{
    using R = typename Fmt<S>::R;
    __shared__ double red[32 * (BS / 64)];
    const int t = blockIdx.x, rhs = blockIdx.y;
    const int per = g.sT;  // checkerboard sites per timeslice and parity
    double acc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] = 0;
    for (int j = threadIdx.x; j < 2 * per; j += BS) {
        const int par = j >= per ? 1 : 0;
        const int cb = t * per + (j - par * per);
        const Site s = decode(g, cb, par);
        cx<double> eta[12];
        if (src.kind == SRC_STORED) {
            load_spinor<double>(par ? src.xo : src.xe, g.Vh, rhs, cb, eta);
            to_canonical(eta);
        } else {
            source_site(src, rhs, s, lex_index(g, s), eta);
        }
        cx<R> sl[12];
        load_spinor<S>(par ? so : se, g.Vh, rhs, cb, sl);
        cx<double> sv[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) sv[e] = {(double)sl[e].re, (double)sl[e].im};
        to_canonical(sv);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double re = 0, im = 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const cx<double> e = eta[3 * a + c];
                    const double vr = sv[3 * b + c].re, vi = sv[3 * b + c].im;
                    re += e.re * vr + e.im * vi;
                    im += e.re * vi - e.im * vr;
                }
                acc[2 * (4 * a + b)] += re;
                acc[2 * (4 * a + b) + 1] += im;
            }
    }
    block_sum<32>(acc, red);
    if (threadIdx.x == 0) {
        double *out = C + ((int64_t)rhs * g.T + t) * 32;
#pragma unroll
        for (int k = 0; k < 32; ++k) out[k] = acc[k];
    }
}

// loops[n][g][t] = sum_d sum_{ab} Gamma_g[a][b] C[n*ncls + d][t][a][b]
__global__ void gamma_contract_kernel(const double *C, int ncls, int T, const double *gam, const int *gidx,
                                      int n_gamma, double *loops)
{
    const int n = blockIdx.x;
    for (int k = threadIdx.x; k < n_gamma * T; k += blockDim.x) {
        const int gi = k / T, t = k - gi * T;
        const double *G = gam + gidx[gi] * 32;
        double re = 0, im = 0;
        for (int d = 0; d < ncls; ++d) {
            const double *c = C + (((int64_t)n * ncls + d) * T + t) * 32;
            for (int ab = 0; ab < 16; ++ab) {
                const double gr = G[2 * ab], gi2 = G[2 * ab + 1];
                re += gr * c[2 * ab] - gi2 * c[2 * ab + 1];
                im += gr * c[2 * ab + 1] + gi2 * c[2 * ab];
            }
        }
        loops[(((int64_t)n * n_gamma + gi) * T + t) * 2] = re;
        loops[(((int64_t)n * n_gamma + gi) * T + t) * 2 + 1] = im;
    }
}


// Gauge-covariant Gaussian smearing of quark fields (Section 2), one step on
// the output parity p:
//   out(x) = [ in(x) + alpha sum_{i=x,y,z} ( U_i(x) in(x+i) + U_i(x-i)^+ in(x-i) ) ] / (1 + 6 alpha),
// spin-diagonal (the same colour multiply on all four spins), no boundary
// sign (space is periodic).  FP64 fields and links.
// One workgroup per (block of BS sites, right-hand side).  Workgroup b runs on
// XCD b mod 8; each XCD takes a contiguous eighth of the (site block, RHS)
// items with the RHS running fastest, so the right-hand sides of a site block
// run together on one XCD and its links are fetched into that L2 once.
template <int NE>
__global__ __launch_bounds__(BS) void smear_kernel(const void *links, Field in_same, Field in_other, Field out,
                                                   int parity, Geom g, double alpha, double norm, int nrhs)
{
    const int64_t total = (int64_t)gridDim.x;
    const int xcd = blockIdx.x % 8;
    const int64_t item = xcd * (total / 8) + min<int64_t>(xcd, total % 8) + blockIdx.x / 8;
    const int rhs = (int)(item % nrhs);
    const int cb = (int)(item / nrhs) * BS + threadIdx.x;
    if (cb >= g.Vh) return;
    const int p = parity, q = 1 - p;
    const Site s = decode(g, cb, p);
    int nb[8];
    neighbours(g, cb, s, nb);
    cx<double> acc[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[e] = {0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int mu = d >> 1;
        const bool fwd = (d & 1) == 0;
        cx<double> u[9];
        load_link<double, NE>(links, g.Vh, mu, fwd ? p : q, fwd ? cb : nb[d], u);
        cx<double> v[12];
        load_spinor<double>(in_other, g.Vh, rhs, nb[d], v);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (fwd)
                        cmac(acc[3 * sp + i], u[3 * i + j], v[3 * sp + j]);
                    else
                        cmac_conj(acc[3 * sp + i], u[3 * j + i], v[3 * sp + j]);
                }
            }
    }
    cx<double> x[12];
    load_spinor<double>(in_same, g.Vh, rhs, cb, x);
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        x[e].re = norm * fma(alpha, acc[e].re, x[e].re);
        x[e].im = norm * fma(alpha, acc[e].im, x[e].im);
    }
    store_spinor<double>(out, g.Vh, rhs, cb, x);
}

// Disconnected two-loop correlator (Section 3, Eq. 2) from per-noise loops
// l[n][T] complex (re, im interleaved).  noise_sum_kernel: sum[t] = sum_n l[n][t]
// (one thread per t, n in order).  corr_kernel, block dt: the ordered pairs of
// distinct noises, as all pairs minus the same-noise ones,
//     S = sum_t sb[t] sa[t + dt] - sum_n sum_t lb[n][t] la[n][t + dt]   (t + dt mod T),
// and out[dt] = -norm * S.  Fixed summation order: deterministic.
__global__ void noise_sum_kernel(const double *l, int n, int T, double *sum)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double re = 0, im = 0;
    for (int k = 0; k < n; ++k) {
        re += l[((int64_t)k * T + t) * 2];
        im += l[((int64_t)k * T + t) * 2 + 1];
    }
    sum[2 * t] = re;
    sum[2 * t + 1] = im;
}

__global__ __launch_bounds__(256) void corr_kernel(const double *lb, const double *la, const double *sb,
                                                   const double *sa, int n, int T, double norm, double *out)
{
    __shared__ double red[2 * 4];
    const int dt = blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        for (int t = 0; t < T; ++t) {
            const int u = t + dt < T ? t + dt : t + dt - T;
            const double br = lb[((int64_t)k * T + t) * 2], bi = lb[((int64_t)k * T + t) * 2 + 1];
            const double ar = la[((int64_t)k * T + u) * 2], ai = la[((int64_t)k * T + u) * 2 + 1];
            v[0] += br * ar - bi * ai;
            v[1] += br * ai + bi * ar;
        }
    block_sum<2>(v, red);
    if (threadIdx.x != 0) return;
    double cr = 0, ci = 0;
    for (int t = 0; t < T; ++t) {
        const int u = t + dt < T ? t + dt : t + dt - T;
        cr += sb[2 * t] * sa[2 * u] - sb[2 * t + 1] * sa[2 * u + 1];
        ci += sb[2 * t] * sa[2 * u + 1] + sb[2 * t + 1] * sa[2 * u];
    }
    out[2 * dt] = -norm * (cr - v[0]);
    out[2 * dt + 1] = -norm * (ci - v[1]);
}

// dst(x) = A_{n,t(x)} eta(x): the source gamma5 sum_g W[n][g][t] Gamma_g^+ eta of
// the adjoint solve of noise n, with A as [noise][T][4][4] complex (row a, column b)
__global__ __launch_bounds__(BS) void adjoint_source_kernel(Field dst, int parity, SourceSpec src, Geom g,
                                                            const double *A, int64_t first_noise)
{
    const int rhs = blockIdx.y;
    const int cb = blockIdx.x * BS + threadIdx.x;
    if (cb >= g.Vh) return;
    const Site s = decode(g, cb, parity);
    cx<double> eta[12];
    source_site(src, rhs, s, lex_index(g, s), eta);
    const double *At = A + ((src.noise[rhs] - first_noise) * g.T + s.t) * 32;
    cx<double> v[12];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int b = 0; b < 4; ++b) cmac(acc, cx<double>{At[2 * (4 * a + b)], At[2 * (4 * a + b) + 1]}, eta[3 * b + c]);
            v[3 * a + c] = acc;
        }
    to_internal(v);
    store_spinor<double>(dst, g.Vh, rhs, cb, v);
}

// a stored FP64 spinor in the chiral basis
__device__ __forceinline__ void load_chiral(const Field &f, int64_t Vh, int rhs, int64_t cb, cx<double> v[12])
{
    load_spinor<double>(f, Vh, rhs, cb, v);
    to_canonical(v);
}

// load a full spinor (chiral basis) and apply gamma5 = diag(1, 1, -1, -1) when g5 is set
__device__ __forceinline__ void load_g5(const Field &f, int64_t Vh, int rhs, int64_t cb, bool g5, cx<double> v[12])
{
    load_chiral(f, Vh, rhs, cb, v);
    if (g5)
#pragma unroll
        for (int e = 6; e < 12; ++e) v[e] = -v[e];
}

// one direction of the link gradient at site x with forward neighbour y = x + mu:
//   X_ac = sum_alpha conj(a_{alpha a}(x)) [(1 - g_mu) s(y)]_{alpha c}
//        = sum over the two projected spins of conj(P- a(x)) P- s(y),
//   Y_ac = sum_alpha conj(a_{alpha a}(y)) [(1 + g_mu) s(x)]_{alpha c}
//        = sum over the two projected spins of conj(P+ a(y)) P+ s(x),
//   acc_ac += conj(X_ac) + Y_ca      (dF = Re(conj(grad) dU) convention)
template <int MU>
__device__ __forceinline__ void grad_dir(const Field &se, const Field &so, const Field &ae, const Field &ao,
                                         const Geom &g, int par, int64_t cbx, int64_t cby, int nrhs,
                                         cx<double> acc[9])
{
    const Field &sx = par ? so : se, &ax = par ? ao : ae;
    const Field &sy = par ? se : so, &ay = par ? ae : ao;
    for (int r = 0; r < nrhs; ++r) {
        cx<double> v[12], h[6], ah[6];
        load_chiral(sy, g.Vh, r, cby, v);
        project<double, MU, -1>(v, h);
        load_g5(ax, g.Vh, r, cbx, true, v);
        project<double, MU, -1>(v, ah);
        cx<double> X[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cx<double> t = {0.0, 0.0};
                cmac_conj(t, ah[a], h[c]);
                cmac_conj(t, ah[3 + a], h[3 + c]);
                X[3 * a + c] = t;
            }
        load_chiral(sx, g.Vh, r, cbx, v);
        project<double, MU, +1>(v, h);
        load_g5(ay, g.Vh, r, cby, true, v);
        project<double, MU, +1>(v, ah);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cx<double> y = {0.0, 0.0};  // Y_{c a}
                cmac_conj(y, ah[c], h[a]);
                cmac_conj(y, ah[3 + c], h[3 + a]);
                acc[3 * a + c] = acc[3 * a + c] + conj(X[3 * a + c]) + y;
            }
    }
}

// grad[mu][x] += kappa b_mu(x) sum_rhs (conj X + Y^T).  A workgroup takes 64
// sites of one parity and its four wavefronts the four directions (wavefront
// mu owns the entries (mu, x) of those sites), so the four walk the
// right-hand sides together and read each site's own spinors at about the
// same time: one fetch from memory serves all four instead of one pass over
// every right-hand side per direction.
__global__ __launch_bounds__(256) void link_grad_kernel(Field se, Field so, Field ae, Field ao, Geom g, int nrhs,
                                                        double kappa, double *grad)
{
    const int par = blockIdx.y;
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cb = blockIdx.x * 64 + (threadIdx.x & 63);
    if (cb >= g.Vh) return;
    const Site s = decode(g, cb, par);
    const int64_t lex = lex_index(g, s);
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t base_x = cb - (s.x >> 1);
    cx<double> acc[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[e] = {0.0, 0.0};
    int64_t cby;
    double b = 1.0;
    if (mu == 0) {
        const int xf = s.x + 1 == g.X ? 0 : s.x + 1;
        cby = base_x + (xf >> 1);
        grad_dir<0>(se, so, ae, ao, g, par, cb, cby, nrhs, acc);
    } else if (mu == 1) {
        cby = s.y + 1 == g.Y ? cb - (int64_t)(g.Y - 1) * g.sY : cb + g.sY;
        grad_dir<1>(se, so, ae, ao, g, par, cb, cby, nrhs, acc);
    } else if (mu == 2) {
        cby = s.z + 1 == g.Z ? cb - (int64_t)(g.Z - 1) * g.sZ : cb + g.sZ;
        grad_dir<2>(se, so, ae, ao, g, par, cb, cby, nrhs, acc);
    } else {
        cby = s.t + 1 == g.T ? cb - (int64_t)(g.T - 1) * g.sT : cb + g.sT;
        if (g.tap && s.t + 1 == g.T) b = -1.0;
        grad_dir<3>(se, so, ae, ao, g, par, cb, cby, nrhs, acc);
    }
    double2 *dst = reinterpret_cast<double2 *>(grad) + ((int64_t)mu * V + lex) * 9;
    const double f = kappa * b;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        double2 o = dst[e];
        dst[e] = make_double2(o.x + f * acc[e].re, o.y + f * acc[e].im);
    }
}

template <typename S>
__global__ __launch_bounds__(BS) void links_convert_kernel(void *dst, int ne, const double *src64, int64_t Vh)
{
    using F = Fmt<S>;
    using R = typename F::R;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    const int mp = blockIdx.y;  // mu * 2 + parity
    if (cb >= Vh) return;
    const double2 *s = reinterpret_cast<const double2 *>(src64) + (int64_t)mp * 9 * Vh;
    typename F::E *d = static_cast<typename F::E *>(dst) + (int64_t)mp * ne * Vh;
    for (int e = 0; e < ne; ++e) {
        double2 z = s[e * Vh + cb];
        F::st(d, e * Vh + cb, cx<R>{R(z.x), R(z.y)});
    }
}

// canonical links [4][V][9] complex128 (site i = x + X (y + Y (z + Z t))) ->
// [4][2][9][Vh] complex128, U_mu(x) of a site of parity p at [mu][p][.][i >> 1]
__global__ __launch_bounds__(BS) void links_reorder_kernel(const double2 *src, double2 *dst, Geom g, int64_t V)
{
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const int mu = blockIdx.y;
    if (i >= V) return;
    int64_t r = i;
    const int x = (int)(r % g.X);
    r /= g.X;
    const int y = (int)(r % g.Y);
    r /= g.Y;
    const int z = (int)(r % g.Z);
    const int t = (int)(r / g.Z);
    const int par = (x + y + z + t) & 1;
    const int64_t Vh = V / 2, cb = i >> 1;
    const double2 *a = src + ((int64_t)mu * V + i) * 9;
    double2 *b = dst + ((int64_t)(mu * 2 + par) * 9) * Vh + cb;
#pragma unroll
    for (int e = 0; e < 9; ++e) b[e * Vh] = a[e];
}

#define DL_DISPATCH(prec, NAME, ...)                                                                    \
    do {                                                                                                \
        switch (prec) {                                                                                 \
        case P64: hipLaunchKernelGGL(NAME<double>, __VA_ARGS__); break;                                 \
        case P32: hipLaunchKernelGGL(NAME<float>, __VA_ARGS__); break;                                  \
        case P16: hipLaunchKernelGGL(NAME<__half>, __VA_ARGS__); break;                                 \
        default: hipLaunchKernelGGL(NAME<__hip_bfloat16>, __VA_ARGS__); break;                          \
        }                                                                                               \
    } while (0)

double field_bytes(int prec, int64_t Vh, int nrhs)
{
    return ((double)Vh * 12 * elem_bytes(prec) + (prec == P16 ? 4.0 * Vh : 0.0)) * nrhs;
}

}  // namespace

void k_pack(int prec, Field dst, int parity, const double *canon, const Geom &g, int nrhs, hipStream_t s)
{
    dim3 grid((g.Vh + BS - 1) / BS, nrhs);
    DL_DISPATCH(prec, pack_kernel, grid, dim3(BS), 0, s, dst, parity, canon, g);
}

void k_unpack(int prec, Field src, int parity, double *canon, const Geom &g, int nrhs, hipStream_t s)
{
    dim3 grid((g.Vh + BS - 1) / BS, nrhs);
    DL_DISPATCH(prec, unpack_kernel, grid, dim3(BS), 0, s, src, parity, canon, g);
}

void k_source(int prec, Field dst, int parity, const SourceSpec &src, const Geom &g, int nrhs, hipStream_t s)
{
    ProfScope ps(PROF_TRACE, field_bytes(prec, g.Vh, nrhs), s);
    dim3 grid((g.Vh + BS - 1) / BS, nrhs);
    DL_DISPATCH(prec, source_kernel, grid, dim3(BS), 0, s, dst, parity, src, g);
}

void k_trace(int prec, Field se, Field so, const SourceSpec &src, const Geom &g, int nrhs, double *C, hipStream_t s)
{
    ProfScope ps(PROF_TRACE, 2 * field_bytes(prec, g.Vh, nrhs), s);
    dim3 grid(g.T, nrhs);
    DL_DISPATCH(prec, trace_kernel, grid, dim3(BS), 0, s, se, so, src, g, C);
}

void k_gamma_contract(const double *C, int n_noise, int ncls, int T, const double *gam, const int *gidx,
                      int n_gamma, double *loops, hipStream_t s)
{
    hipLaunchKernelGGL(gamma_contract_kernel, dim3(n_noise), dim3(128), 0, s, C, ncls, T, gam, gidx, n_gamma, loops);
}

void k_smear(const void *links, int recon, Field ine, Field ino, Field oute, Field outo, const Geom &g, int nrhs,
             double alpha, hipStream_t s)
{
    // per step: both parities read once as the centre and once as neighbours' source, written once;
    // links of the three spatial directions, both parities, once
    ProfScope ps(PROF_SMEAR, 6 * field_bytes(P64, g.Vh, nrhs) + 2.0 * 3 * g.Vh * (recon == 12 ? 6 : 9) * 16, s);
    const double norm = 1.0 / (1.0 + 6.0 * alpha);
    // one workgroup per (site block, RHS), the kernel maps them to XCDs; the
    // right-hand sides go in chunks that keep the grid below 2^31 workgroups
    const int64_t nblk = (g.Vh + BS - 1) / BS;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nrhs, 0x7fffffff / nblk));
    for (int r0 = 0; r0 < nrhs; r0 += chunk) {
        const int n = std::min(chunk, nrhs - r0);
        auto sub = [&](Field f) {  // FP64 fields: [rhs][12][Vh] complex (and the gap), no scales
            f.d = static_cast<char *>(f.d) + (size_t)r0 * rhs_stride_bytes(g.Vh, 16);
            return f;
        };
        const dim3 grid((unsigned)(nblk * n));
        if (recon == 12) {
            hipLaunchKernelGGL(smear_kernel<6>, grid, dim3(BS), 0, s, links, sub(ine), sub(ino), sub(oute), 0, g,
                               alpha, norm, n);
            hipLaunchKernelGGL(smear_kernel<6>, grid, dim3(BS), 0, s, links, sub(ino), sub(ine), sub(outo), 1, g,
                               alpha, norm, n);
        } else {
            hipLaunchKernelGGL(smear_kernel<9>, grid, dim3(BS), 0, s, links, sub(ine), sub(ino), sub(oute), 0, g,
                               alpha, norm, n);
            hipLaunchKernelGGL(smear_kernel<9>, grid, dim3(BS), 0, s, links, sub(ino), sub(ine), sub(outo), 1, g,
                               alpha, norm, n);
        }
    }
}

void k_correlator(const double *lb, const double *la, double *sb, double *sa, int n, int T, double norm, double *out,
                  hipStream_t s)
{
    hipLaunchKernelGGL(noise_sum_kernel, dim3((T + 63) / 64), dim3(64), 0, s, lb, n, T, sb);
    hipLaunchKernelGGL(noise_sum_kernel, dim3((T + 63) / 64), dim3(64), 0, s, la, n, T, sa);
    hipLaunchKernelGGL(corr_kernel, dim3(T), dim3(256), 0, s, lb, la, sb, sa, n, T, norm, out);
}

void k_adjoint_source(Field dst, int parity, const SourceSpec &src, const Geom &g, int nrhs, const double *A,
                      int64_t first_noise, hipStream_t s)
{
    ProfScope ps(PROF_TRACE, field_bytes(P64, g.Vh, nrhs), s);
    dim3 grid((g.Vh + BS - 1) / BS, nrhs);
    hipLaunchKernelGGL(adjoint_source_kernel, grid, dim3(BS), 0, s, dst, parity, src, g, A, first_noise);
}

void k_link_grad(Field se, Field so, Field ae, Field ao, const Geom &g, int nrhs, double kappa, double *grad,
                 hipStream_t s)
{
    ProfScope ps(PROF_TRACE, 4 * field_bytes(P64, g.Vh, nrhs) + 2.0 * 2 * g.Vh * 4 * 9 * 16, s);
    // 64 sites and four directions (one wavefront each) per workgroup
    dim3 grid((g.Vh + 63) / 64, 2);
    hipLaunchKernelGGL(link_grad_kernel, grid, dim3(256), 0, s, se, so, ae, ao, g, nrhs, kappa, grad);
}

void k_links_reorder(const double *canon, double *dst, const Geom &g, hipStream_t s)
{
    const int64_t V = (int64_t)g.X * g.Y * g.Z * g.T;
    dim3 grid((unsigned)((V + BS - 1) / BS), 4);
    hipLaunchKernelGGL(links_reorder_kernel, grid, dim3(BS), 0, s, reinterpret_cast<const double2 *>(canon),
                       reinterpret_cast<double2 *>(dst), g, V);
}

void k_links_convert(int prec, void *dst, int ne, const double *src64, int64_t Vh, hipStream_t s)
{
    dim3 grid((Vh + BS - 1) / BS, 8);
    DL_DISPATCH(prec, links_convert_kernel, grid, dim3(BS), 0, s, dst, ne, src64, Vh);
}

}  // namespace dl
