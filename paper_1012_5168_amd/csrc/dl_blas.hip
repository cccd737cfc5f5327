// dl_blas.hip -- Krylov vector kernels: fused BiCGStab / CGNR updates with
// their reductions, the per-right-hand-side scalar updates, and generic field
// kernels (copy/convert, norms, dots, reliable-update folding).
//
// Reductions are deterministic: each block writes one partial per
// right-hand side, and a one-wave-per-right-hand-side kernel sums the
// partials in a fixed order.  Vector kernels run one thread per site with the
// right-hand side on grid.y and return early for right-hand sides whose mask
// flag is clear.
#include "dl_internal.hpp"

namespace dl {

namespace {

constexpr int BS = 256;

template <typename R>
__device__ __forceinline__ cx<R> ld_c(const double *p) { return {R(p[0]), R(p[1])}; }

__device__ __forceinline__ bool masked_off(const int *mask, int rhs) { return mask != nullptr && !mask[rhs]; }

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

__global__ void bicg_init_kernel(KState *st, int *act, int *upd, const double *b2_parts_e, const double *b2_parts_o,
                                 int nblk, double tol2, double delta2, int maxiter)
{
    const int rhs = blockIdx.x;
    double b2 = sum_parts(b2_parts_e, rhs, nblk, 1, 0);
    if (b2_parts_o) b2 += sum_parts(b2_parts_o, rhs, nblk, 1, 0);
    if (threadIdx.x == 0) {
        KState s = {};
        s.rho[0] = s.alpha[0] = s.omega[0] = 1.0;
        s.b2 = b2;
        s.stop2 = tol2 * b2;
        s.delta2 = delta2;
        s.maxiter = maxiter;
        st[rhs] = s;
        act[rhs] = b2 > 0 ? 1 : 0;
        st[rhs].done = b2 > 0 ? 0 : 1;
        upd[rhs] = 0;
    }
}

// rho_new = (rhat, r) from parts[2] (+ |r|^2 in parts[2] of a 3-part layout when np = 3)
__global__ void bicg_rho_kernel(KState *st, int *act, int *upd, const int *mask, const double *parts, int nblk,
                                int np, int first, int mixed)
{
    const int rhs = blockIdx.x;
    if (masked_off(mask, rhs)) return;
    if (!first && !act[rhs]) return;
    double rn[2] = {sum_parts(parts, rhs, nblk, np, 0), sum_parts(parts, rhs, nblk, np, 1)};
    double rr = np == 3 ? sum_parts(parts, rhs, nblk, np, 2) : rn[0];
    if (threadIdx.x != 0) return;
    KState s = st[rhs];
    if (first) {
        // restart: rho = alpha = omega = 1, p = v = 0, so beta = rho_new
        s.rho[0] = s.alpha[0] = s.omega[0] = 1.0;
        s.rho[1] = s.alpha[1] = s.omega[1] = 0.0;
        s.maxrr = rr;
    } else {
        s.iters += 1;
    }
    double q[2], ao[2];
    cdiv(rn, s.rho, q);
    cdiv(s.alpha, s.omega, ao);
    cmul(q, ao, s.beta);
    s.rho[0] = rn[0];
    s.rho[1] = rn[1];
    s.rr = rr;
    if (!isfinite(rr) || !isfinite(s.beta[0]) || !isfinite(s.beta[1])) {
        s.nonfinite = 1;
        act[rhs] = 0;
        upd[rhs] = 0;
    } else if (!first) {
        if (rr <= s.stop2 || s.iters >= s.maxiter || (rn[0] == 0 && rn[1] == 0)) {
            // converged (or out of iterations, or breakdown): check the FP64 true residual
            act[rhs] = 0;
            upd[rhs] = 1;
        } else if (mixed && rr < s.delta2 * s.maxrr) {
            upd[rhs] = 1;
        }
        if (rr > s.maxrr) s.maxrr = rr;
    }
    st[rhs] = s;
}

__global__ void bicg_alpha_kernel(KState *st, const int *act, const double *parts, int nblk)
{
    const int rhs = blockIdx.x;
    if (!act[rhs]) return;
    double rv[2] = {sum_parts(parts, rhs, nblk, 2, 0), sum_parts(parts, rhs, nblk, 2, 1)};
    if (threadIdx.x != 0) return;
    KState s = st[rhs];
    cdiv(s.rho, rv, s.alpha);
    if (!isfinite(s.alpha[0]) || !isfinite(s.alpha[1])) s.alpha[0] = s.alpha[1] = 0.0;
    st[rhs] = s;
}

__global__ void bicg_omega_kernel(KState *st, const int *act, const double *parts, int nblk)
{
    const int rhs = blockIdx.x;
    if (!act[rhs]) return;
    double ts[2] = {sum_parts(parts, rhs, nblk, 3, 0), sum_parts(parts, rhs, nblk, 3, 1)};
    double tt = sum_parts(parts, rhs, nblk, 3, 2);
    if (threadIdx.x != 0) return;
    KState s = st[rhs];
    if (tt > 0) {
        s.omega[0] = ts[0] / tt;
        s.omega[1] = ts[1] / tt;
    } else {
        s.omega[0] = s.omega[1] = 0.0;
    }
    st[rhs] = s;
}

// after an FP64 residual recomputation (parts: |r_e|^2 [, |r_o|^2])
__global__ void true_residual_kernel(KState *st, int *act, int *upd, int *restart, const double *parts_e,
                                     const double *parts_o, int nblk, int final_check)
{
    const int rhs = blockIdx.x;
    if (!upd[rhs]) {
        if (threadIdx.x == 0) restart[rhs] = 0;
        return;
    }
    double r2 = sum_parts(parts_e, rhs, nblk, 1, 0);
    if (parts_o) r2 += sum_parts(parts_o, rhs, nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = st[rhs];
    s.true2 = r2;
    s.updates += 1;
    restart[rhs] = 0;
    if (!isfinite(r2)) {
        s.nonfinite = 1;
        act[rhs] = 0;
    } else if (r2 <= s.stop2) {
        s.done = 1;
        act[rhs] = 0;
    } else if (!act[rhs] && !final_check && s.iters < s.maxiter) {
        // the iterated residual claimed convergence but the true one disagrees:
        // restart the recursion from the true residual
        act[rhs] = 1;
        restart[rhs] = 1;
    }
    s.maxrr = r2;
    s.rr = r2;
    st[rhs] = s;
    upd[rhs] = 0;
}

__global__ void cg_init_kernel(KState *st, int *act, const double *parts, int nblk, int iters)
{
    const int rhs = blockIdx.x;
    double rr = sum_parts(parts, rhs, nblk, 1, 0);
    if (threadIdx.x == 0) {
        KState s = {};
        s.rr = rr;
        s.maxiter = iters;
        st[rhs] = s;
        act[rhs] = (rr > 0 && iters > 0) ? 1 : 0;
    }
}

// alpha = rr / Re(p, q)
__global__ void cg_alpha_kernel(KState *st, int *act, const double *parts, int nblk)
{
    const int rhs = blockIdx.x;
    if (!act[rhs]) return;
    double pq = sum_parts(parts, rhs, nblk, 2, 0);
    if (threadIdx.x != 0) return;
    KState s = st[rhs];
    if (pq > 0) {
        s.alpha[0] = s.rr / pq;
    } else {  // exact convergence: nothing left to do
        s.alpha[0] = 0;
        act[rhs] = 0;
    }
    s.alpha[1] = 0;
    st[rhs] = s;
}

__global__ void cg_beta_kernel(KState *st, int *act, const double *parts, int nblk)
{
    const int rhs = blockIdx.x;
    if (!act[rhs]) return;
    double rr = sum_parts(parts, rhs, nblk, 1, 0);
    if (threadIdx.x != 0) return;
    KState s = st[rhs];
    s.beta[0] = s.rr > 0 ? rr / s.rr : 0;
    s.beta[1] = 0;
    s.rr = rr;
    s.iters += 1;
    if (s.iters >= s.maxiter || !(rr > 0)) act[rhs] = 0;
    st[rhs] = s;
}

__global__ void sum_parts_kernel(const double *parts, int nblk, int np, double *out)
{
    const int rhs = blockIdx.x;
    for (int k = 0; k < np; ++k) {
        double v = sum_parts(parts, rhs, nblk, np, k);
        if (threadIdx.x == 0) out[rhs * np + k] = v;
    }
}

// ---------------------------------------------------------------- vector kernels

template <int NP>
__device__ __forceinline__ void write_parts(double v[NP], double *parts, int rhs)
{
    __shared__ double red[NP * (BS / 64)];
    block_sum<NP>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NP; ++k) parts[((int64_t)rhs * gridDim.x + blockIdx.x) * NP + k] = v[k];
}

// p = r + beta (p - omega v)
template <typename S>
__global__ __launch_bounds__(BS) void bicg_p_kernel(Field p, Field r, Field v, const KState *st, const int *act,
                                                    int64_t Vh)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (!act[rhs]) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    const cx<R> beta = ld_c<R>(st[rhs].beta), omega = ld_c<R>(st[rhs].omega);
    cx<R> pv[12], rv[12], vv[12];
    load_spinor<S>(p, Vh, rhs, cb, pv);
    load_spinor<S>(r, Vh, rhs, cb, rv);
    load_spinor<S>(v, Vh, rhs, cb, vv);
#pragma unroll
    for (int e = 0; e < 12; ++e) pv[e] = rv[e] + beta * (pv[e] - omega * vv[e]);
    store_spinor<S>(p, Vh, rhs, cb, pv);
}

// r = r - alpha v   (r becomes s)
template <typename S>
__global__ __launch_bounds__(BS) void bicg_s_kernel(Field r, Field v, const KState *st, const int *act, int64_t Vh)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (!act[rhs]) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    const cx<R> alpha = ld_c<R>(st[rhs].alpha);
    cx<R> rv[12], vv[12];
    load_spinor<S>(r, Vh, rhs, cb, rv);
    load_spinor<S>(v, Vh, rhs, cb, vv);
#pragma unroll
    for (int e = 0; e < 12; ++e) rv[e] = rv[e] - alpha * vv[e];
    store_spinor<S>(r, Vh, rhs, cb, rv);
}

// x += alpha p + omega s;  r = s - omega t;  partials (rhat, r), |r|^2
template <typename S>
__global__ __launch_bounds__(BS) void bicg_xr_kernel(Field x, Field r, Field p, Field t, Field rh, const KState *st,
                                                     const int *act, int64_t Vh, double *parts)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (!act[rhs]) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    double part[3] = {0, 0, 0};
    if (cb < Vh) {
        const cx<R> alpha = ld_c<R>(st[rhs].alpha), omega = ld_c<R>(st[rhs].omega);
        cx<R> xv[12], sv[12], pv[12], tv[12], hv[12];
        load_spinor<S>(x, Vh, rhs, cb, xv);
        load_spinor<S>(r, Vh, rhs, cb, sv);
        load_spinor<S>(p, Vh, rhs, cb, pv);
        load_spinor<S>(t, Vh, rhs, cb, tv);
        load_spinor<S>(rh, Vh, rhs, cb, hv);
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            xv[e] = xv[e] + alpha * pv[e] + omega * sv[e];
            sv[e] = sv[e] - omega * tv[e];
            part[0] += (double)hv[e].re * sv[e].re + (double)hv[e].im * sv[e].im;
            part[1] += (double)hv[e].re * sv[e].im - (double)hv[e].im * sv[e].re;
            part[2] += (double)sv[e].re * sv[e].re + (double)sv[e].im * sv[e].im;
        }
        store_spinor<S>(x, Vh, rhs, cb, xv);
        store_spinor<S>(r, Vh, rhs, cb, sv);
    }
    write_parts<3>(part, parts, rhs);
}

// x += alpha p;  r -= alpha q;  partial |r|^2
template <typename S>
__global__ __launch_bounds__(BS) void cg_xr_kernel(Field x, Field r, Field p, Field q, const KState *st,
                                                   const int *act, int64_t Vh, double *parts)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (!act[rhs]) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    double part[1] = {0};
    if (cb < Vh) {
        const R alpha = R(st[rhs].alpha[0]);
        cx<R> xv[12], rv[12], pv[12], qv[12];
        load_spinor<S>(x, Vh, rhs, cb, xv);
        load_spinor<S>(r, Vh, rhs, cb, rv);
        load_spinor<S>(p, Vh, rhs, cb, pv);
        load_spinor<S>(q, Vh, rhs, cb, qv);
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            xv[e] = xv[e] + alpha * pv[e];
            rv[e] = rv[e] - alpha * qv[e];
            part[0] += (double)rv[e].re * rv[e].re + (double)rv[e].im * rv[e].im;
        }
        store_spinor<S>(x, Vh, rhs, cb, xv);
        store_spinor<S>(r, Vh, rhs, cb, rv);
    }
    write_parts<1>(part, parts, rhs);
}

// p = r + beta p
template <typename S>
__global__ __launch_bounds__(BS) void cg_p_kernel(Field p, Field r, const KState *st, const int *act, int64_t Vh)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (!act[rhs]) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    const R beta = R(st[rhs].beta[0]);
    cx<R> pv[12], rv[12];
    load_spinor<S>(p, Vh, rhs, cb, pv);
    load_spinor<S>(r, Vh, rhs, cb, rv);
#pragma unroll
    for (int e = 0; e < 12; ++e) pv[e] = rv[e] + beta * pv[e];
    store_spinor<S>(p, Vh, rhs, cb, pv);
}

template <typename SD, typename SS>
__global__ __launch_bounds__(BS) void copy_kernel(Field dst, Field src, const int *mask, int64_t Vh)
{
    using RD = typename Fmt<SD>::R;
    using RS = typename Fmt<SS>::R;
    const int rhs = blockIdx.y;
    if (masked_off(mask, rhs)) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    cx<RS> v[12];
    cx<RD> w[12];
    load_spinor<SS>(src, Vh, rhs, cb, v);
#pragma unroll
    for (int e = 0; e < 12; ++e) w[e] = {RD(v[e].re), RD(v[e].im)};
    store_spinor<SD>(dst, Vh, rhs, cb, w);
}

template <typename S>
__global__ __launch_bounds__(BS) void zero_kernel(Field f, const int *mask, int64_t Vh)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (masked_off(mask, rhs)) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    cx<R> v[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) v[e] = {R(0), R(0)};
    store_spinor<S>(f, Vh, rhs, cb, v);
}

// x64 += xlo; xlo = 0   (masked by the update flags)
template <typename S>
__global__ __launch_bounds__(BS) void fold_kernel(Field x64, Field xlo, const int *mask, int64_t Vh)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (masked_off(mask, rhs)) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    cx<double> xv[12];
    cx<R> lv[12];
    load_spinor<double>(x64, Vh, rhs, cb, xv);
    load_spinor<S>(xlo, Vh, rhs, cb, lv);
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        xv[e].re += (double)lv[e].re;
        xv[e].im += (double)lv[e].im;
        lv[e] = {R(0), R(0)};
    }
    store_spinor<double>(x64, Vh, rhs, cb, xv);
    store_spinor<S>(xlo, Vh, rhs, cb, lv);
}

template <typename S>
__global__ __launch_bounds__(BS) void norm2_kernel(Field f, const int *mask, int64_t Vh, double *parts)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (masked_off(mask, rhs)) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    double part[1] = {0};
    if (cb < Vh) {
        cx<R> v[12];
        load_spinor<S>(f, Vh, rhs, cb, v);
#pragma unroll
        for (int e = 0; e < 12; ++e) part[0] += (double)v[e].re * v[e].re + (double)v[e].im * v[e].im;
    }
    write_parts<1>(part, parts, rhs);
}

template <typename S>
__global__ __launch_bounds__(BS) void dot_kernel(Field a, Field b, const int *mask, int64_t Vh, double *parts)
{
    using R = typename Fmt<S>::R;
    const int rhs = blockIdx.y;
    if (masked_off(mask, rhs)) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    double part[2] = {0, 0};
    if (cb < Vh) {
        cx<R> av[12], bv[12];
        load_spinor<S>(a, Vh, rhs, cb, av);
        load_spinor<S>(b, Vh, rhs, cb, bv);
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            part[0] += (double)av[e].re * bv[e].re + (double)av[e].im * bv[e].im;
            part[1] += (double)av[e].re * bv[e].im - (double)av[e].im * bv[e].re;
        }
    }
    write_parts<2>(part, parts, rhs);
}

__global__ __launch_bounds__(BS) void sub_kernel(Field dst, Field a, Field b, const int *mask, int64_t Vh)
{
    const int rhs = blockIdx.y;
    if (masked_off(mask, rhs)) return;
    const int64_t cb = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (cb >= Vh) return;
    cx<double> av[12], bv[12];
    load_spinor<double>(a, Vh, rhs, cb, av);
    load_spinor<double>(b, Vh, rhs, cb, bv);
#pragma unroll
    for (int e = 0; e < 12; ++e) av[e] = av[e] - bv[e];
    store_spinor<double>(dst, Vh, rhs, cb, av);
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

double vec_bytes(int prec, int64_t Vh, int nrhs, int nvec)
{
    double per = (double)Vh * 12 * elem_bytes(prec) + (prec == P16 ? 4.0 * Vh : 0.0);
    return per * nrhs * nvec;
}

}  // namespace

int blas_blocks(int64_t Vh) { return (int)((Vh + BS - 1) / BS); }

static dim3 vgrid(int64_t Vh, int nrhs) { return dim3(blas_blocks(Vh), nrhs); }

// ---------------------------------------------------------------- scalar launches

void k_bicg_init(KState *st, int *act, int *upd, int nrhs, const double *b2_parts_e, const double *b2_parts_o,
                 int nblk, double tol2, double delta2, int maxiter, hipStream_t s)
{
    hipLaunchKernelGGL(bicg_init_kernel, dim3(nrhs), dim3(64), 0, s, st, act, upd, b2_parts_e, b2_parts_o, nblk, tol2,
                       delta2, maxiter);
}
void k_bicg_rho(KState *st, int *act, int *upd, const int *mask, int nrhs, const double *parts, int nblk, int np,
                int first, int mixed, hipStream_t s)
{
    hipLaunchKernelGGL(bicg_rho_kernel, dim3(nrhs), dim3(64), 0, s, st, act, upd, mask, parts, nblk, np, first, mixed);
}
void k_bicg_alpha(KState *st, const int *act, int nrhs, const double *parts, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(bicg_alpha_kernel, dim3(nrhs), dim3(64), 0, s, st, act, parts, nblk);
}
void k_bicg_omega(KState *st, const int *act, int nrhs, const double *parts, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(bicg_omega_kernel, dim3(nrhs), dim3(64), 0, s, st, act, parts, nblk);
}
void k_true_residual(KState *st, int *act, int *upd, int *restart, int nrhs, const double *parts_e,
                     const double *parts_o, int nblk, int final_check, hipStream_t s)
{
    hipLaunchKernelGGL(true_residual_kernel, dim3(nrhs), dim3(64), 0, s, st, act, upd, restart, parts_e, parts_o,
                       nblk, final_check);
}
void k_cg_init(KState *st, int *act, int nrhs, const double *parts, int nblk, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(cg_init_kernel, dim3(nrhs), dim3(64), 0, s, st, act, parts, nblk, iters);
}
void k_cg_alpha(KState *st, int *act, int nrhs, const double *parts, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(nrhs), dim3(64), 0, s, st, act, parts, nblk);
}
void k_cg_beta(KState *st, int *act, int nrhs, const double *parts, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(cg_beta_kernel, dim3(nrhs), dim3(64), 0, s, st, act, parts, nblk);
}
void k_sum_parts(const double *parts, int nrhs, int nblk, int nparts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_parts_kernel, dim3(nrhs), dim3(64), 0, s, parts, nblk, nparts, out);
}

// ---------------------------------------------------------------- vector launches

void k_bicg_p(int prec, Field p, Field r, Field v, const KState *st, const int *act, int64_t Vh, int nrhs,
              hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 4), s);
    DL_DISPATCH(prec, bicg_p_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, p, r, v, st, act, Vh);
}
void k_bicg_s(int prec, Field r, Field v, const KState *st, const int *act, int64_t Vh, int nrhs, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 3), s);
    DL_DISPATCH(prec, bicg_s_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, r, v, st, act, Vh);
}
void k_bicg_xr(int prec, Field x, Field r, Field p, Field t, Field rh, const KState *st, const int *act, int64_t Vh,
               int nrhs, double *parts, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 7), s);
    DL_DISPATCH(prec, bicg_xr_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, x, r, p, t, rh, st, act, Vh, parts);
}
void k_cg_xr(int prec, Field x, Field r, Field p, Field q, const KState *st, const int *act, int64_t Vh, int nrhs,
             double *parts, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 6), s);
    DL_DISPATCH(prec, cg_xr_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, x, r, p, q, st, act, Vh, parts);
}
void k_cg_p(int prec, Field p, Field r, const KState *st, const int *act, int64_t Vh, int nrhs, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 3), s);
    DL_DISPATCH(prec, cg_p_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, p, r, st, act, Vh);
}

template <typename SD>
static void copy_from(int prec_src, Field dst, Field src, const int *mask, int64_t Vh, int nrhs, hipStream_t s)
{
    dim3 g = vgrid(Vh, nrhs);
    switch (prec_src) {
    case P64: hipLaunchKernelGGL((copy_kernel<SD, double>), g, dim3(BS), 0, s, dst, src, mask, Vh); break;
    case P32: hipLaunchKernelGGL((copy_kernel<SD, float>), g, dim3(BS), 0, s, dst, src, mask, Vh); break;
    case P16: hipLaunchKernelGGL((copy_kernel<SD, __half>), g, dim3(BS), 0, s, dst, src, mask, Vh); break;
    default: hipLaunchKernelGGL((copy_kernel<SD, __hip_bfloat16>), g, dim3(BS), 0, s, dst, src, mask, Vh); break;
    }
}

void k_copy(int prec_dst, Field dst, int prec_src, Field src, int64_t Vh, int nrhs, const int *mask, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec_dst, Vh, nrhs, 1) + vec_bytes(prec_src, Vh, nrhs, 1), s);
    switch (prec_dst) {
    case P64: copy_from<double>(prec_src, dst, src, mask, Vh, nrhs, s); break;
    case P32: copy_from<float>(prec_src, dst, src, mask, Vh, nrhs, s); break;
    case P16: copy_from<__half>(prec_src, dst, src, mask, Vh, nrhs, s); break;
    default: copy_from<__hip_bfloat16>(prec_src, dst, src, mask, Vh, nrhs, s); break;
    }
}

void k_zero(int prec, Field f, int64_t Vh, int nrhs, const int *mask, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 1), s);
    DL_DISPATCH(prec, zero_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, f, mask, Vh);
}

void k_fold_x(Field x64, int prec, Field xlo, int64_t Vh, int nrhs, const int *mask, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(P64, Vh, nrhs, 2) + vec_bytes(prec, Vh, nrhs, 2), s);
    DL_DISPATCH(prec, fold_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, x64, xlo, mask, Vh);
}

void k_norm2_parts(int prec, Field f, int64_t Vh, int nrhs, const int *mask, double *parts, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 1), s);
    DL_DISPATCH(prec, norm2_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, f, mask, Vh, parts);
}

void k_dot_parts(int prec, Field a, Field b, int64_t Vh, int nrhs, const int *mask, double *parts, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(prec, Vh, nrhs, 2), s);
    DL_DISPATCH(prec, dot_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, a, b, mask, Vh, parts);
}

void k_sub(Field dst, Field a, Field b, int64_t Vh, int nrhs, const int *mask, hipStream_t s)
{
    ProfScope ps(PROF_BLAS, vec_bytes(P64, Vh, nrhs, 3), s);
    hipLaunchKernelGGL(sub_kernel, vgrid(Vh, nrhs), dim3(BS), 0, s, dst, a, b, mask, Vh);
}

}  // namespace dl
