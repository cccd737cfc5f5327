// dl_dslash.hpp -- the even-odd Wilson hopping kernel (one parity out, the
// other parity in) with fused epilogues.
//
// (D psi)(x) = sum_mu (1 - g_mu) b U_mu(x) psi(x+mu) + (1 + g_mu) b U_mu(x-mu)^+ psi(x-mu)
// (D^+ flips both projector signs).  Each neighbour spinor is projected to a
// half spinor (two spin components) before the colour multiply, using the
// block form g_mu = [[0, A_mu], [A_mu^+, 0]] of the chiral basis
// (A_k = -i sigma_k, A_4 = 1):
//     (1 + s g_mu) psi = [h ; s A_mu^+ h],   h = psi_up + s A_mu psi_down,
// so a hop costs two SU(3) matrix-vector products instead of four.
#pragma once

#include "dl_internal.hpp"

namespace dl {

struct DKArgs {
    Geom g;
    int parity;
    Field in, out, x, y;
    const void *links;
    double a;
    int nrhs;
    int nblk;  // site blocks per right-hand-side group
    double *partials;
    const int *active;
    unsigned *live_count;
};

// h = psi_up + s A_mu psi_down (two spin components x three colours)
template <typename R, int MU, int SG>
__device__ __forceinline__ void project(const cx<R> p[12], cx<R> h[6])
{
    const R s = R(SG);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MU == 0) {  // A = -i sigma_1: A psi_d = -i (psi3, psi2)
            h[c] = p[c] - s * times_i(p[9 + c]);
            h[3 + c] = p[3 + c] - s * times_i(p[6 + c]);
        } else if constexpr (MU == 1) {  // A = -i sigma_2: A psi_d = (-psi3, psi2)
            h[c] = p[c] - s * p[9 + c];
            h[3 + c] = p[3 + c] + s * p[6 + c];
        } else if constexpr (MU == 2) {  // A = -i sigma_3: A psi_d = (-i psi2, i psi3)
            h[c] = p[c] - s * times_i(p[6 + c]);
            h[3 + c] = p[3 + c] + s * times_i(p[9 + c]);
        } else {  // A = 1
            h[c] = p[c] + s * p[6 + c];
            h[3 + c] = p[3 + c] + s * p[9 + c];
        }
    }
}

// acc += [g ; s A_mu^+ g]
template <typename R, int MU, int SG>
__device__ __forceinline__ void reconstruct(cx<R> acc[12], const cx<R> g[6])
{
    const R s = R(SG);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = acc[c] + g[c];
        acc[3 + c] = acc[3 + c] + g[3 + c];
        if constexpr (MU == 0) {  // A^+ = i sigma_1: A^+ g = i (g1, g0)
            acc[6 + c] = acc[6 + c] + s * times_i(g[3 + c]);
            acc[9 + c] = acc[9 + c] + s * times_i(g[c]);
        } else if constexpr (MU == 1) {  // A^+ = i sigma_2: A^+ g = (g1, -g0)
            acc[6 + c] = acc[6 + c] + s * g[3 + c];
            acc[9 + c] = acc[9 + c] - s * g[c];
        } else if constexpr (MU == 2) {  // A^+ = i sigma_3: A^+ g = (i g0, -i g1)
            acc[6 + c] = acc[6 + c] + s * times_i(g[c]);
            acc[9 + c] = acc[9 + c] - s * times_i(g[3 + c]);
        } else {
            acc[6 + c] = acc[6 + c] + s * g[c];
            acc[9 + c] = acc[9 + c] + s * g[3 + c];
        }
    }
}

// one hop: neighbour spinor at checkerboard index nb (other parity), link at
// (lpar, lcb); forward hops multiply by U, backward hops by U^+
template <typename S, int NE, int MU, int SG, bool FWD, int NR>
__device__ __forceinline__ void hop(const DKArgs &a, int64_t nb, int lpar, int64_t lcb, typename Fmt<S>::R bsign,
                                    const int rhs[NR], cx<typename Fmt<S>::R> acc[NR][12])
{
    using R = typename Fmt<S>::R;
    const int64_t Vh = a.g.Vh;
    cx<R> u[9];
    load_link<S, NE>(a.links, Vh, MU, lpar, lcb, u);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        cx<R> psi[12];
        load_spinor<S>(a.in, Vh, rhs[r], nb, psi);
        cx<R> h[6];
        project<R, MU, SG>(psi, h);
        if constexpr (MU == 3) {
#pragma unroll
            for (int e = 0; e < 6; ++e) h[e] = bsign * h[e];
        }
        cx<R> gg[6];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                cx<R> t = {R(0), R(0)};
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if constexpr (FWD)
                        cmac(t, u[3 * i + j], h[3 * sp + j]);
                    else
                        cmac_conj(t, u[3 * j + i], h[3 * sp + j]);
                }
                gg[3 * sp + i] = t;
            }
        reconstruct<R, MU, SG>(acc[r], gg);
    }
    // Pin the accumulators here: this forces the hop's arithmetic to finish
    // before the next hop's loads issue.  Without it the compiler issues all
    // eight neighbours' loads first and runs out of registers.
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int e = 0; e < 12; ++e) asm volatile("" : "+v"(acc[r][e].re), "+v"(acc[r][e].im));
}

template <int EPI>
constexpr int nparts_c()
{
    return EPI == EPI_XPAY_DOT ? 2 : EPI == EPI_XPAY_TS ? 3 : (EPI == EPI_XPAY_NRM || EPI == EPI_XMY_NRM) ? 1 : 0;
}

// One work item: site block sb of right-hand-side group grp, item L = grp * nblk + sb.
template <typename S, int NE, bool DAG, int EPI, int NR>
__device__ __forceinline__ void dslash_item(const DKArgs &a, int L, double *red)
{
    using R = typename Fmt<S>::R;
    constexpr int NP = nparts_c<EPI>();

    const Geom &g = a.g;
    const int grp = L / a.nblk, sb = L - grp * a.nblk;
    int rhs[NR];
    bool live[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        int q = grp * NR + r;
        live[r] = q < a.nrhs && (a.active == nullptr || a.active[q]);
        rhs[r] = q < a.nrhs ? q : grp * NR;
        any = any || live[r];
    }
    if (!any) return;  // uniform across the block
    if (a.live_count != nullptr && threadIdx.x == 0) {
        unsigned nl = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) nl += live[r] ? 1u : 0u;
        atomicAdd(a.live_count, nl);
    }

    const int cb = sb * blockDim.x + threadIdx.x;
    const bool valid = cb < g.Vh;
    cx<R> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int e = 0; e < 12; ++e) acc[r][e] = {R(0), R(0)};

    if (valid) {
        const int p = a.parity, q = 1 - p;
        const Site s = decode(g, cb, p);
        const int64_t base_x = cb - (s.x >> 1);
        constexpr int SF = DAG ? +1 : -1;  // forward projector 1 + SF g
        constexpr int SB = -SF;            // backward projector
        const R one = R(1);
        // x
        {
            int xf = s.x + 1 == g.X ? 0 : s.x + 1;
            int xb = s.x == 0 ? g.X - 1 : s.x - 1;
            hop<S, NE, 0, SF, true, NR>(a, base_x + (xf >> 1), p, cb, one, rhs, acc);
            int64_t nbb = base_x + (xb >> 1);
            hop<S, NE, 0, SB, false, NR>(a, nbb, q, nbb, one, rhs, acc);
        }
        // y
        {
            int64_t nf = s.y + 1 == g.Y ? cb - (int64_t)(g.Y - 1) * g.sY : cb + g.sY;
            int64_t nbb = s.y == 0 ? cb + (int64_t)(g.Y - 1) * g.sY : cb - g.sY;
            hop<S, NE, 1, SF, true, NR>(a, nf, p, cb, one, rhs, acc);
            hop<S, NE, 1, SB, false, NR>(a, nbb, q, nbb, one, rhs, acc);
        }
        // z
        {
            int64_t nf = s.z + 1 == g.Z ? cb - (int64_t)(g.Z - 1) * g.sZ : cb + g.sZ;
            int64_t nbb = s.z == 0 ? cb + (int64_t)(g.Z - 1) * g.sZ : cb - g.sZ;
            hop<S, NE, 2, SF, true, NR>(a, nf, p, cb, one, rhs, acc);
            hop<S, NE, 2, SB, false, NR>(a, nbb, q, nbb, one, rhs, acc);
        }
        // t, with the boundary sign on the wrapping hops
        {
            const bool lastt = s.t + 1 == g.T, firstt = s.t == 0;
            int64_t nf = lastt ? cb - (int64_t)(g.T - 1) * g.sT : cb + g.sT;
            int64_t nbb = firstt ? cb + (int64_t)(g.T - 1) * g.sT : cb - g.sT;
            R bf = (g.tap && lastt) ? R(-1) : R(1);
            R bb = (g.tap && firstt) ? R(-1) : R(1);
            hop<S, NE, 3, SF, true, NR>(a, nf, p, cb, bf, rhs, acc);
            hop<S, NE, 3, SB, false, NR>(a, nbb, q, nbb, bb, rhs, acc);
        }
    }

    const R coef = R(a.a);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double part[NP > 0 ? NP : 1];
#pragma unroll
        for (int k = 0; k < (NP > 0 ? NP : 1); ++k) part[k] = 0.0;
        if (valid && live[r]) {
            cx<R> o[12];
            if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
                for (int e = 0; e < 12; ++e) o[e] = coef * acc[r][e];
            } else {
                cx<R> xv[12];
                load_spinor<S>(a.x, g.Vh, rhs[r], cb, xv);
                if constexpr (EPI == EPI_XMY_NRM) {
                    cx<R> yv[12];
                    load_spinor<S>(a.y, g.Vh, rhs[r], cb, yv);
#pragma unroll
                    for (int e = 0; e < 12; ++e) xv[e] = xv[e] - yv[e];
                }
#pragma unroll
                for (int e = 0; e < 12; ++e) {
                    o[e].re = fma(coef, acc[r][e].re, xv[e].re);
                    o[e].im = fma(coef, acc[r][e].im, xv[e].im);
                }
                if constexpr (EPI == EPI_XPAY_DOT) {
                    cx<R> yv[12];
                    load_spinor<S>(a.y, g.Vh, rhs[r], cb, yv);
#pragma unroll
                    for (int e = 0; e < 12; ++e) {
                        part[0] += (double)yv[e].re * o[e].re + (double)yv[e].im * o[e].im;
                        part[1] += (double)yv[e].re * o[e].im - (double)yv[e].im * o[e].re;
                    }
                } else if constexpr (EPI == EPI_XPAY_TS) {
#pragma unroll
                    for (int e = 0; e < 12; ++e) {
                        part[0] += (double)o[e].re * xv[e].re + (double)o[e].im * xv[e].im;
                        part[1] += (double)o[e].re * xv[e].im - (double)o[e].im * xv[e].re;
                        part[2] += (double)o[e].re * o[e].re + (double)o[e].im * o[e].im;
                    }
                }
            }
            if constexpr (EPI == EPI_XPAY_NRM || EPI == EPI_XMY_NRM) {
#pragma unroll
                for (int e = 0; e < 12; ++e) part[0] += (double)o[e].re * o[e].re + (double)o[e].im * o[e].im;
            }
            store_spinor<S>(a.out, g.Vh, rhs[r], cb, o);
        }
        if constexpr (NP > 0) {
            block_sum<NP>(part, red);
            if (threadIdx.x == 0 && live[r]) {
                double *dst = a.partials + ((int64_t)rhs[r] * a.nblk + sb) * NP;
#pragma unroll
                for (int k = 0; k < NP; ++k) dst[k] = part[k];
            }
            __syncthreads();
        }
    }
}

// A launch covers the work items of every segment (lattice) of the batch.
template <typename S, int NE, bool DAG, int EPI, int NR>
__global__ __launch_bounds__(256) void dslash_kernel(Segs<DKArgs> B)
{
    constexpr int NP = nparts_c<EPI>();
    __shared__ double red[(NP > 0 ? NP : 1) * 4];
    for_each_item(B, [&](const DKArgs &a, int L) { dslash_item<S, NE, DAG, EPI, NR>(a, L, red); });
}

template <typename S>
void launch_dslash_t(const DslashCall *c, int nseg, int nr, int bs, int persistent, hipStream_t s);

}  // namespace dl
