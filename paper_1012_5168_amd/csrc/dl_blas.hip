// dl_blas.hip -- Krylov vector kernels: fused BiCGStab / CGNR updates with
// their reductions, the per-right-hand-side scalar updates, and generic field
// kernels (copy/convert, norms, dots, reliable-update folding).
//
// Every launch covers a batch of segments (one per lattice); a work item is
// one (right-hand side, site block) of a segment, or one right-hand side for
// the scalar kernels.  Reductions are deterministic: each site block writes
// one partial per right-hand side, and a one-wave-per-right-hand-side kernel
// sums the partials in a fixed order.  Items whose mask flag is clear return
// at once.
#include <algorithm>

#include "dl_internal.hpp"

namespace dl {

namespace {

constexpr int BS = 256;
constexpr int PERSIST = 8 * 32 * 16;  // grid cap of the streaming kernels (multiple of 8)

template <typename R>
__device__ __forceinline__ cx<R> ld_c(const double *p) { return {R(p[0]), R(p[1])}; }

__device__ __forceinline__ bool masked_off(const int *mask, int rhs) { return mask != nullptr && !mask[rhs]; }

// profiling: the first block of a live right-hand side counts it once
__device__ __forceinline__ void count_live(unsigned *live, int blk)
{
    if (live != nullptr && blk == 0 && threadIdx.x == 0) atomicAdd(live, 1u);
}

// ---------------------------------------------------------------- scalar kernels (one wave per rhs)

// sum of partials [rhs][nblk][np] component k, fixed order
__device__ double sum_parts(const double *parts, int rhs, int nblk, int np, int k)
{
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += parts[((int64_t)rhs * nblk + b) * np + k];
    return wave_sum(s);
}

__device__ __forceinline__ void cdiv(const double a[2], const double b[2], double out[2])
{
    double d = b[0] * b[0] + b[1] * b[1];
    double re = (a[0] * b[0] + a[1] * b[1]) / d, im = (a[1] * b[0] - a[0] * b[1]) / d;
    out[0] = re;
    out[1] = im;
}
__device__ __forceinline__ void cmul(const double a[2], const double b[2], double out[2])
{
    double re = a[0] * b[0] - a[1] * b[1], im = a[0] * b[1] + a[1] * b[0];
    out[0] = re;
    out[1] = im;
}

__device__ void bicg_init(const SSeg &a, const SParams &p, int rhs)
{
    double b2 = sum_parts(a.parts, rhs, a.nblk, 1, 0);
    if (a.parts2) b2 += sum_parts(a.parts2, rhs, a.nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = {};
    s.rho[0] = s.alpha[0] = s.omega[0] = 1.0;
    s.b2 = b2;
    s.stop2 = p.tol2 * b2;
    s.delta2 = p.delta2;
    s.maxiter = p.maxiter;
    s.done = b2 > 0 ? 0 : 1;
    a.st[rhs] = s;
    a.act[rhs] = b2 > 0 ? 1 : 0;
    a.upd[rhs] = 0;
}

// (Re)start of the recursion: rho = (rhat, r) from partials [.., 2] (with
// rhat = r, so |r|^2 is its real part), alpha = omega = 1.
__device__ void bicg_rho(const SSeg &a, const SParams &p, int rhs)
{
    if (masked_off(a.mask, rhs)) return;
    double rn[2] = {sum_parts(a.parts, rhs, a.nblk, 2, 0), sum_parts(a.parts, rhs, a.nblk, 2, 1)};
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    s.rho[0] = rn[0];
    s.rho[1] = rn[1];
    s.alpha[0] = s.omega[0] = 1.0;
    s.alpha[1] = s.omega[1] = 0.0;
    s.beta[0] = s.beta[1] = 0.0;
    s.rr = rn[0];
    s.maxrr = rn[0];
    if (!isfinite(rn[0]) || !isfinite(rn[1])) {
        s.nonfinite = 1;
        a.act[rhs] = 0;
        a.upd[rhs] = 0;
    }
    a.st[rhs] = s;
}

// After the x / r / p update of an iteration: |r|^2 from partials [.., 1];
// counts the iteration and flags convergence (or the iteration cap, or a
// breakdown: rho = 0 or omega = 0) for the FP64 true-residual check, and a
// reliable update when |r| fell by delta since the last one.
__device__ void bicg_check(const SSeg &a, const SParams &p, int rhs)
{
    if (!a.act[rhs]) return;
    const double rr = sum_parts(a.parts, rhs, a.nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    s.iters += 1;
    s.rr = rr;
    if (!isfinite(rr) || !isfinite(s.beta[0]) || !isfinite(s.beta[1])) {
        s.nonfinite = 1;
        a.act[rhs] = 0;
        a.upd[rhs] = 0;
    } else {
        if (rr <= s.stop2 || s.iters >= s.maxiter || (s.rho[0] == 0 && s.rho[1] == 0) ||
            (s.omega[0] == 0 && s.omega[1] == 0)) {
            // converged (or out of iterations, or breakdown): check the FP64 true residual
            a.act[rhs] = 0;
            a.upd[rhs] = 1;
        } else if (p.mixed && rr < s.delta2 * s.maxrr) {
            a.upd[rhs] = 1;
        }
        if (rr > s.maxrr) s.maxrr = rr;
    }
    a.st[rhs] = s;
}

__device__ void bicg_alpha(const SSeg &a, int rhs)
{
    if (!a.act[rhs]) return;
    double rv[2] = {sum_parts(a.parts, rhs, a.nblk, 2, 0), sum_parts(a.parts, rhs, a.nblk, 2, 1)};
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    cdiv(s.rho, rv, s.alpha);
    if (!isfinite(s.alpha[0]) || !isfinite(s.alpha[1])) s.alpha[0] = s.alpha[1] = 0.0;
    a.st[rhs] = s;
}

// omega = (t, s) / |t|^2 from the partials of the hop that made t ([.., 5]:
// (t, s), |t|^2, (rhat, t)); the next rho by linearity of r = s - omega t,
// rho' = (rhat, s) - omega (rhat, t), with (rhat, s) from parts2 [.., 2] (the
// s update); beta = (rho' / rho) (alpha / omega).  Each dot is taken directly
// from the vectors of this iteration: nothing accumulates across iterations.
// omega = 0 (t = 0, e.g. s = 0 after an exact half step) ends the recursion:
// beta is set to 0, and the check sends the right-hand side to the FP64 true
// residual, which either confirms convergence or restarts from it.
__device__ void bicg_omega(const SSeg &a, int rhs)
{
    if (!a.act[rhs]) return;
    const int nb2 = a.nblk2 > 0 ? a.nblk2 : a.nblk;
    double ts[2] = {sum_parts(a.parts, rhs, a.nblk, 5, 0), sum_parts(a.parts, rhs, a.nblk, 5, 1)};
    double tt = sum_parts(a.parts, rhs, a.nblk, 5, 2);
    double rt[2] = {sum_parts(a.parts, rhs, a.nblk, 5, 3), sum_parts(a.parts, rhs, a.nblk, 5, 4)};
    double rs[2] = {sum_parts(a.parts2, rhs, nb2, 2, 0), sum_parts(a.parts2, rhs, nb2, 2, 1)};
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    if (tt > 0) {
        s.omega[0] = ts[0] / tt;
        s.omega[1] = ts[1] / tt;
    } else {
        s.omega[0] = s.omega[1] = 0.0;
    }
    double wrt[2], rn[2], q[2], ao[2];
    cmul(s.omega, rt, wrt);
    rn[0] = rs[0] - wrt[0];
    rn[1] = rs[1] - wrt[1];
    if (s.omega[0] == 0 && s.omega[1] == 0) {
        s.beta[0] = s.beta[1] = 0.0;
    } else {
        cdiv(rn, s.rho, q);
        cdiv(s.alpha, s.omega, ao);
        cmul(q, ao, s.beta);
    }
    s.rho[0] = rn[0];
    s.rho[1] = rn[1];
    a.st[rhs] = s;
}

// After a reliable update replaced r by the FP64 residual (partials [.., 2]:
// (rhat, r) of the replaced r): rho takes that value, so that the next alpha
// matches the r it multiplies; alpha, omega and beta stay.
__device__ void bicg_resync(const SSeg &a, int rhs)
{
    if (masked_off(a.mask, rhs)) return;
    double rn[2] = {sum_parts(a.parts, rhs, a.nblk, 2, 0), sum_parts(a.parts, rhs, a.nblk, 2, 1)};
    if (threadIdx.x != 0) return;
    a.st[rhs].rho[0] = rn[0];
    a.st[rhs].rho[1] = rn[1];
}

// after an FP64 residual recomputation (parts: |r_e|^2 [, parts2: |r_o|^2])
__device__ void true_residual(const SSeg &a, const SParams &p, int rhs)
{
    if (!a.upd[rhs]) {
        if (threadIdx.x == 0) a.restart[rhs] = 0;
        return;
    }
    double r2 = sum_parts(a.parts, rhs, a.nblk, 1, 0);
    if (a.parts2) r2 += sum_parts(a.parts2, rhs, a.nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    s.true2 = r2;
    s.updates += 1;
    a.restart[rhs] = 0;
    if (!isfinite(r2)) {
        s.nonfinite = 1;
        a.act[rhs] = 0;
    } else if (r2 <= s.stop2) {
        s.done = 1;
        a.act[rhs] = 0;
    } else if (!a.act[rhs] && !p.final_check && s.iters < s.maxiter) {
        // the iterated residual claimed convergence but the true one disagrees:
        // restart the recursion from the true residual
        a.act[rhs] = 1;
        a.restart[rhs] = 1;
    }
    s.maxrr = r2;
    s.rr = r2;
    a.st[rhs] = s;
    a.upd[rhs] = 0;
}

__device__ void cg_init(const SSeg &a, const SParams &p, int rhs)
{
    double rr = sum_parts(a.parts, rhs, a.nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = {};
    s.rr = rr;
    s.maxiter = p.maxiter;
    a.st[rhs] = s;
    a.act[rhs] = (rr > 0 && p.maxiter > 0) ? 1 : 0;
}

// alpha = |r|^2 / |Mhat p|^2 (= (p, Mhat^+ Mhat p)), partials [.., 1]
__device__ void cg_alpha(const SSeg &a, int rhs)
{
    if (!a.act[rhs]) return;
    if (a.act[rhs] == 2) {  // finished last iteration (its x update is done): now inactive
        if (threadIdx.x == 0) a.act[rhs] = 0;
        return;
    }
    double pq = sum_parts(a.parts, rhs, a.nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    if (pq > 0) {
        s.alpha[0] = s.rr / pq;
    } else {  // exact convergence: nothing left to do
        s.alpha[0] = 0;
        a.act[rhs] = 0;
    }
    s.alpha[1] = 0;
    a.st[rhs] = s;
}

__device__ void cg_beta(const SSeg &a, int rhs)
{
    if (!a.act[rhs]) return;
    double rr = sum_parts(a.parts, rhs, a.nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = a.st[rhs];
    s.beta[0] = s.rr > 0 ? rr / s.rr : 0;
    s.beta[1] = 0;
    s.rr = rr;
    s.iters += 1;
    // finished: 2 keeps it live for this iteration's x update (V_CG_P)
    if (s.iters >= s.maxiter || !(rr > 0)) a.act[rhs] = 2;
    a.st[rhs] = s;
}

__device__ void sum_out(const SSeg &a, const SParams &p, int rhs)
{
    for (int k = 0; k < p.np; ++k) {
        double v = sum_parts(a.parts, rhs, a.nblk, p.np, k);
        if (threadIdx.x == 0) a.out[rhs * p.np + k] = v;
    }
}

template <int OP>
__global__ __launch_bounds__(64) void scalar_kernel(Segs<SSeg> B, SParams p)
{
    for_each_item(B, [&](const SSeg &a, int rhs) {
        if constexpr (OP == S_BICG_INIT) bicg_init(a, p, rhs);
        else if constexpr (OP == S_BICG_RHO) bicg_rho(a, p, rhs);
        else if constexpr (OP == S_BICG_ALPHA) bicg_alpha(a, rhs);
        else if constexpr (OP == S_BICG_OMEGA) bicg_omega(a, rhs);
        else if constexpr (OP == S_BICG_CHECK) bicg_check(a, p, rhs);
        else if constexpr (OP == S_BICG_RESYNC) bicg_resync(a, rhs);
        else if constexpr (OP == S_TRUE_RES) true_residual(a, p, rhs);
        else if constexpr (OP == S_CG_INIT) cg_init(a, p, rhs);
        else if constexpr (OP == S_CG_ALPHA) cg_alpha(a, rhs);
        else if constexpr (OP == S_CG_BETA) cg_beta(a, rhs);
        else sum_out(a, p, rhs);
    });
}

// ---------------------------------------------------------------- vector kernels

template <int NP>
__device__ __forceinline__ void write_parts(double v[NP], double *red, double *parts, int rhs, int nb, int blk)
{
    block_sum<NP>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NP; ++k) parts[((int64_t)rhs * nb + blk) * NP + k] = v[k];
    __syncthreads();
}

// f[0..4] by operation:
//   V_BICG_S   s = r - alpha v (in r's storage); parts (rhat, s)                   f: r, v, rhat
//   V_BICG_XRP x += alpha p + omega s; r = s - omega t; p = r + beta (p - omega v);
//              parts |r|^2                                                          f: x, r(s), p, t, v
//   V_CG_XR    r -= alpha q; parts |r|^2                                            f: r, q
//   V_CG_P     x += alpha p; p = r + beta p                                         f: p, r, x
//   V_ZERO     f0 = 0
//   V_NORM2    parts |f0|^2
//   V_DOT      parts (f0, f1)
template <typename S, int OP>
__device__ __forceinline__ void vec_item(const VSeg &a, int item, double *red)
{
    using R = typename Fmt<S>::R;
    const int nb = (int)((a.Vh + BS - 1) / BS);
    const int rhs = item / nb, blk = item - rhs * nb;
    if (masked_off(a.mask, rhs)) return;
    count_live(a.live, blk);
    const int64_t Vh = a.Vh;
    const int64_t cb = (int64_t)blk * BS + threadIdx.x;
    const bool valid = cb < Vh;
    if constexpr (OP == V_BICG_S) {
        double part[2] = {0, 0};
        if (valid) {
            const cx<R> alpha = ld_c<R>(a.st[rhs].alpha);
            cx<R> rv[12], vv[12], hv[12];
            load_spinor<S, true>(a.f[0], Vh, rhs, cb, rv);
            load_spinor<S, true>(a.f[1], Vh, rhs, cb, vv);
            load_spinor<S, true>(a.f[2], Vh, rhs, cb, hv);
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                rv[e] = rv[e] - alpha * vv[e];
                part[0] += (double)hv[e].re * rv[e].re + (double)hv[e].im * rv[e].im;
                part[1] += (double)hv[e].re * rv[e].im - (double)hv[e].im * rv[e].re;
            }
            store_spinor<S, true>(a.f[0], Vh, rhs, cb, rv);
        }
        write_parts<2>(part, red, a.parts, rhs, nb, blk);
    } else if constexpr (OP == V_BICG_XRP) {
        double part[1] = {0};
        if (valid) {
            const KState &k = a.st[rhs];
            const cx<R> alpha = ld_c<R>(k.alpha), omega = ld_c<R>(k.omega), beta = ld_c<R>(k.beta);
            cx<R> xv[12], sv[12], pv[12], tv[12], vv[12];
            load_spinor<S, true>(a.f[0], Vh, rhs, cb, xv);
            load_spinor<S, true>(a.f[1], Vh, rhs, cb, sv);
            load_spinor<S, true>(a.f[2], Vh, rhs, cb, pv);
            load_spinor<S, true>(a.f[3], Vh, rhs, cb, tv);
            load_spinor<S, true>(a.f[4], Vh, rhs, cb, vv);
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                xv[e] = xv[e] + alpha * pv[e] + omega * sv[e];
                sv[e] = sv[e] - omega * tv[e];
                pv[e] = sv[e] + beta * (pv[e] - omega * vv[e]);
                part[0] += (double)sv[e].re * sv[e].re + (double)sv[e].im * sv[e].im;
            }
            store_spinor<S, true>(a.f[0], Vh, rhs, cb, xv);
            store_spinor<S, true>(a.f[1], Vh, rhs, cb, sv);
            store_spinor<S, true>(a.f[2], Vh, rhs, cb, pv);
        }
        write_parts<1>(part, red, a.parts, rhs, nb, blk);
    } else if constexpr (OP == V_CG_XR) {
        double part[1] = {0};
        if (valid) {
            const R alpha = R(a.st[rhs].alpha[0]);
            cx<R> rv[12], qv[12];
            load_spinor<S, true>(a.f[0], Vh, rhs, cb, rv);
            load_spinor<S, true>(a.f[1], Vh, rhs, cb, qv);
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                rv[e] = rv[e] - alpha * qv[e];
                part[0] += (double)rv[e].re * rv[e].re + (double)rv[e].im * rv[e].im;
            }
            store_spinor<S, true>(a.f[0], Vh, rhs, cb, rv);
        }
        write_parts<1>(part, red, a.parts, rhs, nb, blk);
    } else if constexpr (OP == V_CG_P) {
        if (!valid) return;
        const R alpha = R(a.st[rhs].alpha[0]), beta = R(a.st[rhs].beta[0]);
        cx<R> pv[12], rv[12], xv[12];
        load_spinor<S, true>(a.f[0], Vh, rhs, cb, pv);
        load_spinor<S, true>(a.f[1], Vh, rhs, cb, rv);
        load_spinor<S, true>(a.f[2], Vh, rhs, cb, xv);
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            xv[e] = xv[e] + alpha * pv[e];
            pv[e] = rv[e] + beta * pv[e];
        }
        store_spinor<S, true>(a.f[2], Vh, rhs, cb, xv);
        store_spinor<S, true>(a.f[0], Vh, rhs, cb, pv);
    } else if constexpr (OP == V_ZERO) {
        if (!valid) return;
        cx<R> v[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) v[e] = {R(0), R(0)};
        store_spinor<S, true>(a.f[0], Vh, rhs, cb, v);
    } else if constexpr (OP == V_NORM2) {
        double part[1] = {0};
        if (valid) {
            cx<R> v[12];
            load_spinor<S, true>(a.f[0], Vh, rhs, cb, v);
#pragma unroll
            for (int e = 0; e < 12; ++e) part[0] += (double)v[e].re * v[e].re + (double)v[e].im * v[e].im;
        }
        write_parts<1>(part, red, a.parts, rhs, nb, blk);
    } else if constexpr (OP == V_DOT) {
        double part[2] = {0, 0};
        if (valid) {
            cx<R> av[12], bv[12];
            load_spinor<S, true>(a.f[0], Vh, rhs, cb, av);
            load_spinor<S, true>(a.f[1], Vh, rhs, cb, bv);
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                part[0] += (double)av[e].re * bv[e].re + (double)av[e].im * bv[e].im;
                part[1] += (double)av[e].re * bv[e].im - (double)av[e].im * bv[e].re;
            }
        }
        write_parts<2>(part, red, a.parts, rhs, nb, blk);
    }
}

template <typename S, int OP>
__global__ __launch_bounds__(BS) void vec_kernel(Segs<VSeg> B)
{
    __shared__ double red[3 * (BS / 64)];
    for_each_item(B, [&](const VSeg &a, int item) { vec_item<S, OP>(a, item, red); });
}

// dst (f0, precision SD) = src (f1, precision SS)
template <typename SD, typename SS>
__global__ __launch_bounds__(BS) void copy_kernel(Segs<VSeg> B)
{
    using RD = typename Fmt<SD>::R;
    using RS = typename Fmt<SS>::R;
    for_each_item(B, [&](const VSeg &a, int item) {
        const int nb = (int)((a.Vh + BS - 1) / BS);
        const int rhs = item / nb, blk = item - rhs * nb;
        if (masked_off(a.mask, rhs)) return;
        count_live(a.live, blk);
        const int64_t cb = (int64_t)blk * BS + threadIdx.x;
        if (cb >= a.Vh) return;
        cx<RS> v[12];
        cx<RD> w[12];
        load_spinor<SS>(a.f[1], a.Vh, rhs, cb, v);
#pragma unroll
        for (int e = 0; e < 12; ++e) w[e] = {RD(v[e].re), RD(v[e].im)};
        store_spinor<SD, true>(a.f[0], a.Vh, rhs, cb, w);
    });
}

// f0 (FP64) += f1 (precision S); f1 = 0      (reliable update of x)
template <typename S>
__global__ __launch_bounds__(BS) void fold_kernel(Segs<VSeg> B)
{
    using R = typename Fmt<S>::R;
    for_each_item(B, [&](const VSeg &a, int item) {
        const int nb = (int)((a.Vh + BS - 1) / BS);
        const int rhs = item / nb, blk = item - rhs * nb;
        if (masked_off(a.mask, rhs)) return;
        count_live(a.live, blk);
        const int64_t cb = (int64_t)blk * BS + threadIdx.x;
        if (cb >= a.Vh) return;
        cx<double> xv[12];
        cx<R> lv[12];
        load_spinor<double>(a.f[0], a.Vh, rhs, cb, xv);
        load_spinor<S>(a.f[1], a.Vh, rhs, cb, lv);
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            xv[e].re += (double)lv[e].re;
            xv[e].im += (double)lv[e].im;
            lv[e] = {R(0), R(0)};
        }
        store_spinor<double, true>(a.f[0], a.Vh, rhs, cb, xv);
        store_spinor<S, true>(a.f[1], a.Vh, rhs, cb, lv);
    });
}

// f0 (r, precision S) = f1 (the FP64 residual); f2 (p, precision S) += f1 - old f0
template <typename S>
__global__ __launch_bounds__(BS) void replace_kernel(Segs<VSeg> B)
{
    using R = typename Fmt<S>::R;
    __shared__ double red[2 * (BS / 64)];
    for_each_item(B, [&](const VSeg &a, int item) {
        const int nb = (int)((a.Vh + BS - 1) / BS);
        const int rhs = item / nb, blk = item - rhs * nb;
        if (masked_off(a.mask, rhs)) return;
        count_live(a.live, blk);
        const int64_t cb = (int64_t)blk * BS + threadIdx.x;
        double part[2] = {0, 0};
        if (cb < a.Vh) {
            cx<R> rv[12], pv[12], hv[12];
            cx<double> nv[12];
            load_spinor<S>(a.f[0], a.Vh, rhs, cb, rv);
            load_spinor<double>(a.f[1], a.Vh, rhs, cb, nv);
            load_spinor<S>(a.f[2], a.Vh, rhs, cb, pv);
            load_spinor<S>(a.f[3], a.Vh, rhs, cb, hv);
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                const cx<R> n = {R(nv[e].re), R(nv[e].im)};
                pv[e] = pv[e] + (n - rv[e]);
                rv[e] = n;
                part[0] += (double)hv[e].re * rv[e].re + (double)hv[e].im * rv[e].im;
                part[1] += (double)hv[e].re * rv[e].im - (double)hv[e].im * rv[e].re;
            }
            store_spinor<S, true>(a.f[0], a.Vh, rhs, cb, rv);
            store_spinor<S, true>(a.f[2], a.Vh, rhs, cb, pv);
        }
        write_parts<2>(part, red, a.parts, rhs, nb, blk);
    });
}

// f0 = f1 - f2 (FP64)
__global__ __launch_bounds__(BS) void sub_kernel(Segs<VSeg> B)
{
    for_each_item(B, [&](const VSeg &a, int item) {
        const int nb = (int)((a.Vh + BS - 1) / BS);
        const int rhs = item / nb, blk = item - rhs * nb;
        if (masked_off(a.mask, rhs)) return;
        count_live(a.live, blk);
        const int64_t cb = (int64_t)blk * BS + threadIdx.x;
        if (cb >= a.Vh) return;
        cx<double> av[12], bv[12];
        load_spinor<double>(a.f[1], a.Vh, rhs, cb, av);
        load_spinor<double>(a.f[2], a.Vh, rhs, cb, bv);
#pragma unroll
        for (int e = 0; e < 12; ++e) av[e] = av[e] - bv[e];
        store_spinor<double, true>(a.f[0], a.Vh, rhs, cb, av);
    });
}

template <typename A>
Segs<A> make_segs(const std::vector<A> &v, int (*items)(const A &))
{
    Segs<A> B;
    if (v.empty() || v.size() > (size_t)MAXSEG) throw Error{DL_EINVAL, "internal: segment count out of range"};
    B.n = (int)v.size();
    B.prefix[0] = 0;
    for (int k = 0; k < B.n; ++k) {
        B.a[k] = v[k];
        B.prefix[k + 1] = B.prefix[k] + items(v[k]);
    }
    return B;
}

int vec_items(const VSeg &a) { return (int)((a.Vh + BS - 1) / BS) * a.nrhs; }
int scalar_items(const SSeg &a) { return a.nrhs; }

int grid_for(int total, int cap) { return total > cap ? cap : total; }

double field_rhs_bytes(int prec, int64_t Vh) { return (double)Vh * 12 * elem_bytes(prec) + (prec == P16 ? 4.0 * Vh : 0.0); }

double vec_bytes(int prec, const std::vector<VSeg> &segs, int nvec)
{
    double b = 0;
    for (const VSeg &a : segs) b += field_rhs_bytes(prec, a.Vh) * a.nrhs;
    return b * nvec;
}

// Profiled launches count the right-hand sides they process (masked ones
// move no bytes): per_rhs(Vh) bytes for each counted one.
template <typename F>
std::vector<VSeg> counted_segs(const std::vector<VSeg> &segs, ProfScope &ps, hipStream_t s, F per_rhs)
{
    std::vector<VSeg> v = segs;
    if (!prof_on() || capturing(s)) return v;
    for (VSeg &a : v) {
        a.live = prof_counter();
        if (a.live) ps.parts.push_back({a.live, per_rhs(a.Vh), 0.0, 1.0});
    }
    return v;
}

template <int OP>
void vec_dispatch(int prec, const Segs<VSeg> &B, int grid, hipStream_t s)
{
    switch (prec) {
    case P64: hipLaunchKernelGGL((vec_kernel<double, OP>), dim3(grid), dim3(BS), 0, s, B); break;
    case P32: hipLaunchKernelGGL((vec_kernel<float, OP>), dim3(grid), dim3(BS), 0, s, B); break;
    case P16: hipLaunchKernelGGL((vec_kernel<__half, OP>), dim3(grid), dim3(BS), 0, s, B); break;
    default: hipLaunchKernelGGL((vec_kernel<__hip_bfloat16, OP>), dim3(grid), dim3(BS), 0, s, B); break;
    }
}

template <typename SD>
void copy_from(int prec_src, const Segs<VSeg> &B, int grid, hipStream_t s)
{
    switch (prec_src) {
    case P64: hipLaunchKernelGGL((copy_kernel<SD, double>), dim3(grid), dim3(BS), 0, s, B); break;
    case P32: hipLaunchKernelGGL((copy_kernel<SD, float>), dim3(grid), dim3(BS), 0, s, B); break;
    case P16: hipLaunchKernelGGL((copy_kernel<SD, __half>), dim3(grid), dim3(BS), 0, s, B); break;
    default: hipLaunchKernelGGL((copy_kernel<SD, __hip_bfloat16>), dim3(grid), dim3(BS), 0, s, B); break;
    }
}

}  // namespace

int blas_blocks(int64_t Vh) { return (int)((Vh + BS - 1) / BS); }

void scalar_launch(int op, const std::vector<SSeg> &segs, const SParams &p, hipStream_t s)
{
    Segs<SSeg> B = make_segs(segs, scalar_items);
    const int grid = grid_for(B.prefix[B.n], PERSIST);
    switch (op) {
    case S_BICG_INIT: hipLaunchKernelGGL(scalar_kernel<S_BICG_INIT>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_BICG_RHO: hipLaunchKernelGGL(scalar_kernel<S_BICG_RHO>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_BICG_ALPHA: hipLaunchKernelGGL(scalar_kernel<S_BICG_ALPHA>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_BICG_OMEGA: hipLaunchKernelGGL(scalar_kernel<S_BICG_OMEGA>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_BICG_CHECK: hipLaunchKernelGGL(scalar_kernel<S_BICG_CHECK>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_BICG_RESYNC: hipLaunchKernelGGL(scalar_kernel<S_BICG_RESYNC>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_TRUE_RES: hipLaunchKernelGGL(scalar_kernel<S_TRUE_RES>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_CG_INIT: hipLaunchKernelGGL(scalar_kernel<S_CG_INIT>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_CG_ALPHA: hipLaunchKernelGGL(scalar_kernel<S_CG_ALPHA>, dim3(grid), dim3(64), 0, s, B, p); break;
    case S_CG_BETA: hipLaunchKernelGGL(scalar_kernel<S_CG_BETA>, dim3(grid), dim3(64), 0, s, B, p); break;
    default: hipLaunchKernelGGL(scalar_kernel<S_SUM>, dim3(grid), dim3(64), 0, s, B, p); break;
    }
}

void vec_launch(int op, int prec, const std::vector<VSeg> &segs, hipStream_t s)
{
    static const int nvec[] = {4, 8, 3, 5, 1, 1, 2};
    ProfScope ps(PROF_BLAS, vec_bytes(prec, segs, nvec[op]), s);
    const std::vector<VSeg> sg =
        counted_segs(segs, ps, s, [&](int64_t Vh) { return nvec[op] * field_rhs_bytes(prec, Vh); });
    Segs<VSeg> B = make_segs(sg, vec_items);
    const int grid = grid_for(B.prefix[B.n], PERSIST);
    switch (op) {
    case V_BICG_S: vec_dispatch<V_BICG_S>(prec, B, grid, s); break;
    case V_BICG_XRP: vec_dispatch<V_BICG_XRP>(prec, B, grid, s); break;
    case V_CG_XR: vec_dispatch<V_CG_XR>(prec, B, grid, s); break;
    case V_CG_P: vec_dispatch<V_CG_P>(prec, B, grid, s); break;
    case V_ZERO: vec_dispatch<V_ZERO>(prec, B, grid, s); break;
    case V_NORM2: vec_dispatch<V_NORM2>(prec, B, grid, s); break;
    default: vec_dispatch<V_DOT>(prec, B, grid, s); break;
    }
}

void copy_launch(int prec_dst, int prec_src, const std::vector<VSeg> &segs, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec_dst, segs, 1) + vec_bytes(prec_src, segs, 1), s);
    const std::vector<VSeg> sg = counted_segs(
        segs, ps, s, [&](int64_t Vh) { return field_rhs_bytes(prec_dst, Vh) + field_rhs_bytes(prec_src, Vh); });
    Segs<VSeg> B = make_segs(sg, vec_items);
    const int grid = grid_for(B.prefix[B.n], PERSIST);
    switch (prec_dst) {
    case P64: copy_from<double>(prec_src, B, grid, s); break;
    case P32: copy_from<float>(prec_src, B, grid, s); break;
    case P16: copy_from<__half>(prec_src, B, grid, s); break;
    default: copy_from<__hip_bfloat16>(prec_src, B, grid, s); break;
    }
}

void fold_launch(int prec, const std::vector<VSeg> &segs, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(P64, segs, 2) + vec_bytes(prec, segs, 2), s);
    const std::vector<VSeg> sg = counted_segs(
        segs, ps, s, [&](int64_t Vh) { return 2 * field_rhs_bytes(P64, Vh) + 2 * field_rhs_bytes(prec, Vh); });
    Segs<VSeg> B = make_segs(sg, vec_items);
    const int grid = grid_for(B.prefix[B.n], PERSIST);
    switch (prec) {
    case P64: hipLaunchKernelGGL(fold_kernel<double>, dim3(grid), dim3(BS), 0, s, B); break;
    case P32: hipLaunchKernelGGL(fold_kernel<float>, dim3(grid), dim3(BS), 0, s, B); break;
    case P16: hipLaunchKernelGGL(fold_kernel<__half>, dim3(grid), dim3(BS), 0, s, B); break;
    default: hipLaunchKernelGGL(fold_kernel<__hip_bfloat16>, dim3(grid), dim3(BS), 0, s, B); break;
    }
}

void replace_launch(int prec, const std::vector<VSeg> &segs, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(P64, segs, 1) + vec_bytes(prec, segs, 5), s);
    const std::vector<VSeg> sg = counted_segs(
        segs, ps, s, [&](int64_t Vh) { return field_rhs_bytes(P64, Vh) + 5 * field_rhs_bytes(prec, Vh); });
    Segs<VSeg> B = make_segs(sg, vec_items);
    const int grid = grid_for(B.prefix[B.n], PERSIST);
    switch (prec) {
    case P64: hipLaunchKernelGGL(replace_kernel<double>, dim3(grid), dim3(BS), 0, s, B); break;
    case P32: hipLaunchKernelGGL(replace_kernel<float>, dim3(grid), dim3(BS), 0, s, B); break;
    case P16: hipLaunchKernelGGL(replace_kernel<__half>, dim3(grid), dim3(BS), 0, s, B); break;
    default: hipLaunchKernelGGL(replace_kernel<__hip_bfloat16>, dim3(grid), dim3(BS), 0, s, B); break;
    }
}

using U4v = unsigned __attribute__((ext_vector_type(4)));

// Streaming probe (measurement only): MODE 0 copies n 16-byte words from src
// to dst, MODE 1 reads them (the XOR of a thread's words reaches dst only if
// it equals a fixed value, so the loads stay live).  A workgroup takes tiles
// of STREAM_U x 256 contiguous words, thread t the words t, t + 256, ...: the
// STREAM_U non-temporal loads of a thread are in flight together and each
// instruction of a wavefront covers 1 KiB, the access of the field kernels
// (one 16-byte word per site and component plane).  Spreading a thread's
// loads over the whole buffer instead (grid stride) was slower: 4.7 against
// 5.5 TB/s for a copy.  Words after the last whole tile take a grid-stride
// tail.
constexpr int STREAM_U = 8;
constexpr int STREAM_GRID = 8192;

template <int MODE>
__global__ __launch_bounds__(256) void stream_kernel(const U4v *src, U4v *dst, int64_t n)
{
    const int64_t ntiles = n / (256 * STREAM_U);
    U4v acc = {0u, 0u, 0u, 0u};
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * (256 * STREAM_U) + threadIdx.x;
        U4v v[STREAM_U];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) v[u] = __builtin_nontemporal_load(src + base + u * 256);
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) {
            if constexpr (MODE == 0)
                __builtin_nontemporal_store(v[u], dst + base + u * 256);
            else
                acc ^= v[u];
        }
    }
    for (int64_t i = ntiles * (256 * STREAM_U) + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const U4v v = __builtin_nontemporal_load(src + i);
        if constexpr (MODE == 0)
            __builtin_nontemporal_store(v, dst + i);
        else
            acc ^= v;
    }
    if constexpr (MODE == 1)
        if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xbf58476du && acc.w == 0x94d049bbu)
            dst[blockIdx.x] = acc;
}

// nwords 16-byte words of zeros from p on (flat buffers that are no packed
// field, such as the link gradient)
__global__ __launch_bounds__(256) void fill_zero_kernel(U4v *p, int64_t n)
{
    const U4v z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = z;
}

void zero_launch(void *p, int64_t nwords, hipStream_t s)
{
    if (nwords <= 0) return;
    const int grid = (int)std::min<int64_t>((nwords + 255) / 256, PERSIST);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, s, static_cast<U4v *>(p), nwords);
}

// Read mode writes at most one word per workgroup: dst needs STREAM_GRID x 16
// bytes (128 KiB).
void stream_launch(int mode, const void *src, void *dst, int64_t nwords, hipStream_t s)
{
    const int64_t want = (nwords + 256 * STREAM_U - 1) / (256 * STREAM_U);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, STREAM_GRID));
    const U4v *a = static_cast<const U4v *>(src);
    U4v *b = static_cast<U4v *>(dst);
    if (mode == 0)
        hipLaunchKernelGGL(stream_kernel<0>, dim3(grid), dim3(256), 0, s, a, b, nwords);
    else
        hipLaunchKernelGGL(stream_kernel<1>, dim3(grid), dim3(256), 0, s, a, b, nwords);
}

void sub_launch(const std::vector<VSeg> &segs, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(P64, segs, 3), s);
    const std::vector<VSeg> sg = counted_segs(segs, ps, s, [&](int64_t Vh) { return 3 * field_rhs_bytes(P64, Vh); });
    Segs<VSeg> B = make_segs(sg, vec_items);
    hipLaunchKernelGGL(sub_kernel, dim3(grid_for(B.prefix[B.n], PERSIST)), dim3(BS), 0, s, B);
}

}  // namespace dl
