// dl_dslash.hpp -- the even-odd Wilson hopping kernel (one parity out, the
// other parity in) with fused epilogues.
//
// (D psi)(x) = sum_mu (1 - g_mu) b U_mu(x) psi(x+mu) + (1 + g_mu) b U_mu(x-mu)^+ psi(x-mu)
// (D^+ flips both projector signs).  Each neighbour spinor is projected to a
// half spinor (two spin components) before the colour multiply, so a hop costs
// two SU(3) matrix-vector products instead of four.  The fields are stored in
// the spin basis of dl_common.hpp (T = [[1, 1], [1, -1]] applied to the chiral
// basis).  There the spatial gammas keep the block form g_k = [[0, A_k],
// [A_k^+, 0]] with A_k = +i sigma_k (the chiral -i sigma_k with its sign
// flipped):
//     (1 + s g_k) psi = [h ; s A_k^+ h],   h = psi_up + s A_k psi_down,
// and g_4 = diag(1, 1, -1, -1): (1 + g_4) psi = [2 psi_up ; 0] and
// (1 - g_4) psi = [0 ; 2 psi_down], so a temporal hop reads one spin pair of
// its neighbour, half the bytes of a spatial one.
#pragma once

#include <type_traits>

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
    const KState *st;
};

// h = psi_up + s A_mu psi_down (two spin components x three colours) with the
// chiral A_mu (A_k = -i sigma_k, A_4 = 1); the stored basis uses it with s
// negated for the spatial directions
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

// gg = U h (forward) or U^+ h (backward) for both spin rows of a half spinor
template <typename R, bool FWD>
__device__ __forceinline__ void colour_mul(const cx<R> u[9], const cx<R> h[6], cx<R> gg[6])
{
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
}

// One spatial hop (MU < 3) on a loaded neighbour spinor in the stored basis:
// project with the projector (1 + SG g_MU), colour-multiply by U (forward)
// or U^+ (backward), reconstruct into the accumulator.
template <typename R, int MU, int SG, bool FWD>
__device__ __forceinline__ void hop_mul(const cx<R> u[9], const cx<R> psi[12], cx<R> acc[12])
{
    static_assert(MU < 3, "temporal hops take one spin pair (hop_mul_t)");
    cx<R> h[6], gg[6];
    project<R, MU, -SG>(psi, h);
    colour_mul<R, FWD>(u, h, gg);
    reconstruct<R, MU, -SG>(acc, gg);
}

// The spin pair a temporal projector (1 + SG g_4) keeps: 0 = upper, 1 = lower.
template <int SG>
constexpr int t_half() { return SG > 0 ? 0 : 1; }

// One temporal hop: `half` is the spin pair t_half<SG>() of the neighbour and
// coef = 2 b (the projector's 2 times the time-boundary sign).
template <typename R, int SG, bool FWD>
__device__ __forceinline__ void hop_mul_t(const cx<R> u[9], const cx<R> half[6], R coef, cx<R> acc[12])
{
    cx<R> h[6], gg[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) h[e] = coef * half[e];
    colour_mul<R, FWD>(u, h, gg);
    constexpr int o = 6 * t_half<SG>();
#pragma unroll
    for (int e = 0; e < 6; ++e) acc[o + e] = acc[o + e] + gg[e];
}

// Pin the accumulators: this forces a hop's arithmetic to finish before the
// next hop's loads issue.  Without it the compiler issues all eight
// neighbours' loads first and runs out of registers.
template <typename R>
__device__ __forceinline__ void pin_acc(cx<R> acc[12])
{
#pragma unroll
    for (int e = 0; e < 12; ++e) asm volatile("" : "+v"(acc[e].re), "+v"(acc[e].im));
}

// one hop of the item kernel: neighbour spinor at checkerboard index nb
// (other parity), link at (lpar, lcb) read from global memory
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
        if constexpr (MU == 3) {
            cx<R> half[6];
            load_half<S, t_half<SG>()>(a.in, Vh, rhs[r], nb, half);
            hop_mul_t<R, SG, FWD>(u, half, R(2) * bsign, acc[r]);
        } else {
            cx<R> psi[12];
            load_spinor<S>(a.in, Vh, rhs[r], nb, psi);
            hop_mul<R, MU, SG, FWD>(u, psi, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) pin_acc<R>(acc[r]);
}

template <int EPI>
constexpr int nparts_c()
{
    return EPI == EPI_XPAY_DOT ? 2
           : EPI == EPI_XPAY_TS ? 5
           : (EPI == EPI_XPAY_NRM || EPI == EPI_XMY_NRM || EPI == EPI_CG_R) ? 1
                                                                           : 0;
}

// Epilogue for one right-hand side at one site: out = a * acc (PLAIN) or
// x + a * acc (the XPAY family, with x - y in place of x for XMY), plus this
// site's share of the epilogue's reductions in part[].
// BUF: read x and y through buffer resources (the LDS-link kernel, whose
// launcher checks that a right-hand side's field fits one), non-temporal.
// NT: store the output non-temporal (it is not read again by the launch).
template <typename S, bool BUF>
__device__ __forceinline__ void load_site(const Field &f, int Vh, int rhs, int64_t cb, cx<typename Fmt<S>::R> v[12])
{
    if constexpr (BUF)
        load_spinor_rsrc<S, 2>(spinor_rsrc<S>(f, Vh, rhs), f, Vh, rhs, (int)cb, v);
    else
        load_spinor<S>(f, Vh, rhs, cb, v);
}

// The operands an epilogue reads at its own site: x for the XPAY family, y
// where it takes a dot product with y, subtracts it or updates it.
template <int EPI>
constexpr bool epi_reads_x()
{
    return EPI != EPI_PLAIN;
}
template <int EPI>
constexpr bool epi_reads_y()
{
    return EPI == EPI_XPAY_DOT || EPI == EPI_XPAY_TS || EPI == EPI_XMY_NRM || EPI == EPI_CG_R;
}
template <typename R, int EPI>
struct EpiOps {
    cx<R> x[epi_reads_x<EPI>() ? 12 : 1], y[epi_reads_y<EPI>() ? 12 : 1];
};

// the epilogue's operand loads (issued ahead of its arithmetic by the
// LDS-link kernel's walk)
template <typename S, int EPI, bool BUF>
__device__ __forceinline__ void epilogue_load(const DKArgs &a, int rhs, int64_t cb,
                                              EpiOps<typename Fmt<S>::R, EPI> &ops)
{
    if constexpr (epi_reads_x<EPI>()) load_site<S, BUF>(a.x, a.g.Vh, rhs, cb, ops.x);
    if constexpr (epi_reads_y<EPI>()) load_site<S, BUF>(a.y, a.g.Vh, rhs, cb, ops.y);
}

template <typename S, int EPI, bool NT>
__device__ __forceinline__ void epilogue_apply(const DKArgs &a, int rhs, int64_t cb,
                                               const cx<typename Fmt<S>::R> acc[12],
                                               const EpiOps<typename Fmt<S>::R, EPI> &ops, double part[], bool valid)
{
    using R = typename Fmt<S>::R;
    const R coef = R(a.a);
    cx<R> o[12];
    if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
        for (int e = 0; e < 12; ++e) o[e] = coef * acc[e];
    } else {
        cx<R> xv[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) xv[e] = ops.x[e];
        if constexpr (EPI == EPI_XMY_NRM) {
#pragma unroll
            for (int e = 0; e < 12; ++e) xv[e] = xv[e] - ops.y[e];
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            o[e].re = fma(coef, acc[e].re, xv[e].re);
            o[e].im = fma(coef, acc[e].im, xv[e].im);
        }
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;
        if constexpr (EPI == EPI_XPAY_DOT) {
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                p0 += (double)ops.y[e].re * o[e].re + (double)ops.y[e].im * o[e].im;
                p1 += (double)ops.y[e].re * o[e].im - (double)ops.y[e].im * o[e].re;
            }
        } else if constexpr (EPI == EPI_XPAY_TS) {
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                p0 += (double)o[e].re * xv[e].re + (double)o[e].im * xv[e].im;
                p1 += (double)o[e].re * xv[e].im - (double)o[e].im * xv[e].re;
                p2 += (double)o[e].re * o[e].re + (double)o[e].im * o[e].im;
                p3 += (double)ops.y[e].re * o[e].re + (double)ops.y[e].im * o[e].im;
                p4 += (double)ops.y[e].re * o[e].im - (double)ops.y[e].im * o[e].re;
            }
        }
        if constexpr (EPI == EPI_CG_R) {
            // the residual update of the normal equations' CG: r -= alpha q
            const R al = R(a.st[rhs].alpha[0]);
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                o[e].re = fma(-al, o[e].re, ops.y[e].re);
                o[e].im = fma(-al, o[e].im, ops.y[e].im);
            }
        }
        if (valid) {
            if constexpr (EPI == EPI_XPAY_DOT) {
                part[0] += p0;
                part[1] += p1;
            } else if constexpr (EPI == EPI_XPAY_TS) {
                part[0] += p0;
                part[1] += p1;
                part[2] += p2;
                part[3] += p3;
                part[4] += p4;
            }
        }
    }
    if constexpr (EPI == EPI_XPAY_NRM || EPI == EPI_XMY_NRM || EPI == EPI_CG_R) {
        double p0 = 0.0;
#pragma unroll
        for (int e = 0; e < 12; ++e) p0 += (double)o[e].re * o[e].re + (double)o[e].im * o[e].im;
        if (valid) part[0] += p0;
    }
    if (valid) store_spinor<S, NT>(a.out, a.g.Vh, rhs, cb, o);
}

template <typename S, int EPI, bool BUF = false, bool NT = false>
__device__ __forceinline__ void epilogue(const DKArgs &a, int rhs, int64_t cb, const cx<typename Fmt<S>::R> acc[12],
                                         double part[], bool valid = true)
{
    EpiOps<typename Fmt<S>::R, EPI> ops;
    epilogue_load<S, EPI, BUF>(a, rhs, cb, ops);
    epilogue_apply<S, EPI, NT>(a, rhs, cb, acc, ops, part, valid);
}

// neighbour checkerboard indices (x+, x-, y+, y-, z+, z-, t+, t-) of site
// cb of parity p
__device__ __forceinline__ void neighbours(const Geom &g, int cb, const Site &s, int nb[8])
{
    const int bx = cb - (s.x >> 1);
    const int xf = s.x + 1 == g.X ? 0 : s.x + 1, xb = s.x == 0 ? g.X - 1 : s.x - 1;
    nb[0] = bx + (xf >> 1);
    nb[1] = bx + (xb >> 1);
    nb[2] = s.y + 1 == g.Y ? cb - (g.Y - 1) * g.sY : cb + g.sY;
    nb[3] = s.y == 0 ? cb + (g.Y - 1) * g.sY : cb - g.sY;
    nb[4] = s.z + 1 == g.Z ? cb - (g.Z - 1) * g.sZ : cb + g.sZ;
    nb[5] = s.z == 0 ? cb + (g.Z - 1) * g.sZ : cb - g.sZ;
    nb[6] = s.t + 1 == g.T ? cb - (g.T - 1) * g.sT : cb + g.sT;
    nb[7] = s.t == 0 ? cb + (g.T - 1) * g.sT : cb - g.sT;
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
    // profiling: live right-hand-side blocks, counted once per group by its
    // first site block (the mask is the same for every block of the group;
    // one atomic per block would contend on the counter)
    if (a.live_count != nullptr && threadIdx.x == 0 && sb == 0) {
        unsigned nl = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) nl += live[r] ? 1u : 0u;
        atomicAdd(a.live_count, nl * (unsigned)a.nblk);
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
        int nb[8];
        neighbours(g, cb, s, nb);
        constexpr int SF = DAG ? +1 : -1;  // forward projector 1 + SF g
        constexpr int SB = -SF;            // backward projector
        const R one = R(1);
        const R bf = (g.tap && s.t + 1 == g.T) ? R(-1) : R(1);
        const R bb = (g.tap && s.t == 0) ? R(-1) : R(1);
        hop<S, NE, 0, SF, true, NR>(a, nb[0], p, cb, one, rhs, acc);
        hop<S, NE, 0, SB, false, NR>(a, nb[1], q, nb[1], one, rhs, acc);
        hop<S, NE, 1, SF, true, NR>(a, nb[2], p, cb, one, rhs, acc);
        hop<S, NE, 1, SB, false, NR>(a, nb[3], q, nb[3], one, rhs, acc);
        hop<S, NE, 2, SF, true, NR>(a, nb[4], p, cb, one, rhs, acc);
        hop<S, NE, 2, SB, false, NR>(a, nb[5], q, nb[5], one, rhs, acc);
        hop<S, NE, 3, SF, true, NR>(a, nb[6], p, cb, bf, rhs, acc);
        hop<S, NE, 3, SB, false, NR>(a, nb[7], q, nb[7], bb, rhs, acc);
    }

#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double part[NP > 0 ? NP : 1];
#pragma unroll
        for (int k = 0; k < (NP > 0 ? NP : 1); ++k) part[k] = 0.0;
        if (valid && live[r]) epilogue<S, EPI, false, true>(a, rhs[r], cb, acc[r], part);
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

// ---------------------------------------------------------------- LDS-link kernel
//
// A workgroup owns 64 consecutive checkerboard sites (one wavefront wide) and
// keeps their 8 link matrices in LDS, expanded to all three rows in the
// arithmetic precision (converted and rebuilt once per block, not once per
// right-hand side and hop; FP64 keeps the six spatial ones as stored and the
// two temporal ones in registers, see lds_tregs); its LANES wavefronts then walk the
// right-hand sides (wavefront w takes w, w + LANES, ...), so every link is
// read from memory once per launch instead of once per right-hand side.
// Site blocks are grouped into regions of rb consecutive blocks; region i
// runs on XCD i mod 8, and the grid is sized so that a region's blocks are
// resident together and advance through the right-hand sides in step: the
// neighbour spinors they share are then fetched into that XCD's L2 once.
// The partial sums of a reducing epilogue are per wavefront, i.e. per
// (right-hand side, 64-site block).
constexpr int LDS_SITES = 64;

// Whether the LDS holds the links expanded (9 complex numbers per link in the
// arithmetic precision) or as stored (NE entries in the storage format,
// converted and completed per use).
// LDS_TLINK_REGS (FP64): the LDS holds only the six spatial links, as stored,
// and every wavefront keeps its site's two temporal links expanded in
// registers, so that four blocks fit per CU (36 KiB each with 12-parameter
// links) and an XCD's whole share of a 16^3 x 32 lattice (four timeslices,
// 128 blocks) is resident at once: a region then reads a quarter more input
// than its own (the two neighbouring timeslices' spin pairs) instead of a
// half.  Measured on the all-live plain launch of 288 right-hand sides with
// one wavefront per block and regions of 128 blocks: 1.48x instead of 1.65x
// the input and links fetched, 1688-1714 against 1736-1761 us with the
// expanded links in LDS (two blocks per CU, regions of 64).
template <typename S>
constexpr bool lds_tregs()
{
    return LDS_TLINK_REGS && std::is_same<S, double>::value;
}

template <typename S, int NE>
constexpr bool lds_expanded()
{
    return !LDS_COMPACT_LINKS && !lds_tregs<S>();
}

template <typename S, int NE>
constexpr int lds_link_bytes()
{
    return lds_tregs<S>()           ? 6 * NE * LDS_SITES * (int)sizeof(typename Fmt<S>::E)
           : lds_expanded<S, NE>() ? 8 * 9 * LDS_SITES * (int)sizeof(cx<typename Fmt<S>::R>)
                                   : 8 * NE * LDS_SITES * (int)sizeof(typename Fmt<S>::E);
}

// Reserve registers so that at most OCC wavefronts share a SIMD (0: the
// occupancy the kernel compiles to).  The register file of a SIMD lane holds
// 512 registers (VGPRs and AGPRs together): claiming v255 and a31 leaves room
// for one wavefront, claiming v191 for two.  The FP64 LDS-link kernel runs
// best at one wavefront per SIMD (measured at 288 right-hand sides with all
// links in LDS: 9 GB fetched per launch instead of 13-14 GB, a third faster);
// capping the blocks per CU through LDS instead, at the same wavefronts per
// CU, does not do it.  With its temporal links in registers it compiles to
// one wavefront per SIMD by itself.
template <int OCC>
__device__ __forceinline__ void reserve_waves()
{
    if constexpr (OCC == 1)
        asm volatile("" ::: "v255", "a31");
    else if constexpr (OCC == 2)
        asm volatile("" ::: "v191");
}

// Whether the LDS-link kernel prefetches its neighbour loads (pipelined walk)
// or walks one hop at a time.  Measured on 288 right-hand sides at 16^3 x 32:
// FP64 (one wavefront per SIMD, registers to spare) and BF16 gained 4-8%.
// FP32 lost 5% while its links were staged as stored (its occupancy was then
// set by registers); with expanded links the LDS caps it first, and the
// pipelined walk takes the plain FP32 launch from 974 to 906 us (the tuner
// then picks one wavefront per block) and the FP32 hopping time of a
// mixed-precision step from 146 to 142 ms.  LDS_PIPELINE_F32=0 builds FP32
// with the serial walk.
#ifndef LDS_PIPELINE_F32
#define LDS_PIPELINE_F32 1
#endif
template <typename S>
constexpr bool lds_pipelined()
{
    return !std::is_same<S, float>::value || LDS_PIPELINE_F32;
}

// How many hops ahead the pipelined walk issues its neighbour loads (1 or 2;
// it keeps 2 x that many neighbour buffers).  Measured at 288 right-hand
// sides on 16^3 x 32: two hops ahead speed the plain FP64 launch up from 1868
// to 1842 us and the plain BF16 one from 636 to 627 us; FP16 is unchanged,
// and the FP64 epilogue variants slow down (x + a D in with a dot product
// 2624 -> 3006 us: 250 registers instead of 220), so of FP64 and BF16 only
// the plain launches take two.  FP32, whose occupancy the LDS sets, takes
// two in every variant (its epilogue variants hold 150-218 registers without
// spills; FP32 hopping time of a mixed-precision 288-RHS step 142 -> 138 ms).
// LDS_PREFETCH=1 builds the plain launches with one, LDS_PREFETCH_EPI_F32=1
// the FP32 epilogue variants.
#ifndef LDS_PREFETCH
#define LDS_PREFETCH 2
#endif
#ifndef LDS_PREFETCH_EPI_F32
#define LDS_PREFETCH_EPI_F32 2
#endif
template <typename S, int EPI>
constexpr int lds_prefetch()
{
    if constexpr (EPI != EPI_PLAIN && std::is_same<S, float>::value) return LDS_PREFETCH_EPI_F32;
    return (EPI == EPI_PLAIN && !std::is_same<S, __half>::value) ? LDS_PREFETCH : 1;
}

// The hop during which the walk issues the epilogue's own-site operand loads
// (x, y) of the current right-hand side, so that they are in flight while the
// last hops compute; 8 issues them after the last hop.  Measured on whole
// solves at 16^3 x 32 (hopping time per 288-RHS step): issued during hop 6,
// FP64 242 -> 233 ms and FP32 (mixed precision) 145 -> 143 ms; the 16-bit
// formats slow down (FP16 CGNR on 416 RHS 122 -> 130 ms) and keep 8.
// LDS_EPI_PREFETCH overrides the choice for every format.
template <typename S>
constexpr int lds_epi_prefetch()
{
#ifdef LDS_EPI_PREFETCH
    return LDS_EPI_PREFETCH;
#else
    return Fmt<S>::VEC < 4 ? 6 : 8;
#endif
}

// a neighbour spinor converted to the arithmetic precision
template <typename R>
struct CxSpinor {
    cx<R> v[12];
};

// the per-(right-hand side, site block) partial sums of a reducing epilogue,
// summed over the wavefront and written by its first lane
template <int NP>
__device__ __forceinline__ void write_block_partials(const DKArgs &a, int r, int sb, int sl, double part[])
{
    if constexpr (NP > 0) {
#pragma unroll
        for (int k = 0; k < NP; ++k) part[k] = wave_sum(part[k]);
        if (sl == 0) {
            double *dst = a.partials + ((int64_t)r * a.nblk + sb) * NP;
#pragma unroll
            for (int k = 0; k < NP; ++k) dst[k] = part[k];
        }
    }
}

template <typename S, int NE, bool DAG, int EPI, int LANES, int OCC>
__global__ __launch_bounds__(LDS_SITES *LANES) void dslash_lds_kernel(Segs<DKArgs> B, int rb)
{
    using R = typename Fmt<S>::R;
    using E = typename Fmt<S>::E;
    constexpr int NP = nparts_c<EPI>();
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    constexpr int EPF = epi_reads_x<EPI>() ? lds_epi_prefetch<S>() : 8;
    __shared__ __align__(16) unsigned char lds[lds_link_bytes<S, NE>()];
    E *const lk = reinterpret_cast<E *>(lds);           // links as stored
    cx<R> *const lx = reinterpret_cast<cx<R> *>(lds);   // links expanded
    reserve_waves<OCC>();
    cx<R> ut[2][9];  // the temporal links in registers (lds_tregs)
    // the link of hop d at this lane's site, all three rows
    auto load_u = [&](int d, int sl_, cx<R> u[9]) {
        if constexpr (lds_tregs<S>()) {
            if (d >= 6) {
#pragma unroll
                for (int e = 0; e < 9; ++e) u[e] = ut[d - 6][e];
                return;
            }
        }
        if constexpr (lds_expanded<S, NE>()) {
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = lx[(d * 9 + e) * LDS_SITES + sl_];
        } else {
#pragma unroll
            for (int e = 0; e < NE; ++e) u[e] = Fmt<S>::ld(lk, (d * NE + e) * LDS_SITES + sl_);
            if constexpr (NE == 6) {
                u[6] = conj(u[1] * u[5] - u[2] * u[4]);
                u[7] = conj(u[2] * u[3] - u[0] * u[5]);
                u[8] = conj(u[0] * u[4] - u[1] * u[3]);
            }
        }
    };

    // w is the wavefront's index, uniform across it: said so explicitly, the
    // per-right-hand-side buffer resources below stay in scalar registers
    const int sl = threadIdx.x & (LDS_SITES - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / LDS_SITES);
    const int total = B.prefix[B.n];
    const int nreg = (total + rb - 1) / rb;
    const int xcd = blockIdx.x % 8, j = blockIdx.x / 8;
    const int nbx = gridDim.x / 8 + (xcd < (int)(gridDim.x % 8) ? 1 : 0);
    const int myreg = nreg / 8 + (xcd < nreg % 8 ? 1 : 0);
    const int cnt = myreg * rb;
    for (int it = j; it < cnt; it += nbx) {
        const int ri = it / rb;
        const int item = (xcd + 8 * ri) * rb + (it - ri * rb);
        if (item >= total) continue;  // uniform across the block
        int sg = 0;
        while (sg + 1 < B.n && item >= B.prefix[sg + 1]) ++sg;
        const DKArgs &a = B.a[sg];
        const Geom &g = a.g;
        const int sb = item - B.prefix[sg];
        // lanes past the last site mirror it: their loads stay in bounds and
        // the epilogue stores nothing and adds nothing for them
        const int cb0 = sb * LDS_SITES + sl;
        const bool valid = cb0 < g.Vh;
        const int cb = valid ? cb0 : g.Vh - 1;
        const int p = a.parity, q = 1 - p;
        const Site s = decode(g, cb, p);
        int nb[8];
        neighbours(g, cb, s, nb);
        __syncthreads();  // the previous item's links are no longer read
        for (int d = w; d < 8; d += LANES) {
            if (lds_tregs<S>() && d >= 6) continue;
            const int mu = d >> 1, bwd = d & 1;
            const int lcb = bwd ? nb[d] : cb;
            const E *src = static_cast<const E *>(a.links) + ((int64_t)(mu * 2 + (bwd ? q : p)) * NE) * g.Vh + lcb;
            if constexpr (lds_expanded<S, NE>()) {
                cx<R> u[9];
                load_link<S, NE>(a.links, g.Vh, mu, bwd ? q : p, lcb, u);
#pragma unroll
                for (int e = 0; e < 9; ++e) lx[(d * 9 + e) * LDS_SITES + sl] = u[e];
            } else {
#pragma unroll
                for (int e = 0; e < NE; ++e) lk[(d * NE + e) * LDS_SITES + sl] = src[(int64_t)e * g.Vh];
            }
        }
        if constexpr (lds_tregs<S>()) {
            load_link<S, NE>(a.links, g.Vh, 3, p, cb, ut[0]);
            load_link<S, NE>(a.links, g.Vh, 3, q, nb[7], ut[1]);
        }
        __syncthreads();

        const R bf = (g.tap && s.t + 1 == g.T) ? R(-1) : R(1);
        const R bb = (g.tap && s.t == 0) ? R(-1) : R(1);
        // hop d's neighbour of right-hand side rr (resource rs) into dst
        auto load_hop = [&](__amdgpu_buffer_rsrc_t rs, int rr, int d, CxSpinor<R> &dst) {
            if (d < 6)
                load_spinor_rsrc<S>(rs, a.in, g.Vh, rr, nb[d], dst.v);
            else if (d == 6)
                load_half_rsrc<S, t_half<SF>()>(rs, a.in, g.Vh, rr, nb[6], dst.v);
            else
                load_half_rsrc<S, t_half<SB>()>(rs, a.in, g.Vh, rr, nb[7], dst.v);
        };
        // hop d on a loaded neighbour, with its link from LDS
        auto apply_hop = [&](int d, const CxSpinor<R> &src, cx<R> acc[12]) {
            cx<R> u[9];
            load_u(d, sl, u);
            switch (d) {
            case 0: hop_mul<R, 0, SF, true>(u, src.v, acc); break;
            case 1: hop_mul<R, 0, SB, false>(u, src.v, acc); break;
            case 2: hop_mul<R, 1, SF, true>(u, src.v, acc); break;
            case 3: hop_mul<R, 1, SB, false>(u, src.v, acc); break;
            case 4: hop_mul<R, 2, SF, true>(u, src.v, acc); break;
            case 5: hop_mul<R, 2, SB, false>(u, src.v, acc); break;
            case 6: hop_mul_t<R, SF, true>(u, src.v, R(2) * bf, acc); break;
            default: hop_mul_t<R, SB, false>(u, src.v, R(2) * bb, acc); break;
            }
        };
        unsigned nlive = 0;
        // Wavefront w takes right-hand sides w, w + LANES, ...  The flags of its
        // next 64 are read once, one per lane, into a wave-uniform mask, so the
        // walk itself reads no flag: a flag load inside it would wait for the
        // previous right-hand side's stores.
        for (int r0 = w; r0 < a.nrhs; r0 += 64 * LANES) {
            const int rl = r0 + sl * LANES;
            const bool on = rl < a.nrhs && (a.active == nullptr || a.active[rl] != 0);
            uint64_t m = __ballot(on);
            nlive += (unsigned)__popcll(m);
            if constexpr (lds_pipelined<S>()) {
                // Neighbour spinors prefetched PF hops ahead: hop d + PF's
                // loads are in flight while hop d computes, and the next
                // right-hand side's first hops while the last hops and the
                // epilogue of this one run.  The empty asm statements fence
                // memory operations: the one after a hop's loads keeps them
                // ahead of the previous hop's arithmetic, the accumulator pin
                // after that arithmetic keeps the following loads behind it
                // (without the fences the compiler issues all eight hops'
                // loads at once and spills).
                if (m == 0) continue;
                int r = r0 + __builtin_ctzll(m) * LANES;
                m &= m - 1;
                __amdgpu_buffer_rsrc_t rin = spinor_rsrc<S>(a.in, g.Vh, r);
                // hop k's neighbour goes to buf[k % NBUF]: NBUF divides 8, so
                // the assignment is the same for every right-hand side
                constexpr int PF = lds_prefetch<S, EPI>(), NBUF = 2 * PF;
                CxSpinor<R> buf[NBUF];
#pragma unroll
                for (int k = 0; k < PF; ++k) load_hop(rin, r, k, buf[k]);
                while (true) {
                    const bool more = m != 0;
                    const int rn = more ? r0 + __builtin_ctzll(m) * LANES : r;
                    m &= m - 1;
                    const __amdgpu_buffer_rsrc_t rin_n = spinor_rsrc<S>(a.in, g.Vh, rn);
                    double part[NP > 0 ? NP : 1];
#pragma unroll
                    for (int k = 0; k < (NP > 0 ? NP : 1); ++k) part[k] = 0.0;
                    cx<R> acc[12];
#pragma unroll
                    for (int e = 0; e < 12; ++e) acc[e] = {R(0), R(0)};
                    EpiOps<R, EPI> ops;
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        // hop d + PF's loads (the next right-hand side's first
                        // hops near the end; after the last right-hand side
                        // rn = r: the redundant loads keep the issue
                        // unconditional, so the compiler need not wait for
                        // them before this hop's arithmetic)
                        const int t = d + PF;
                        if (t < 8)
                            load_hop(rin, r, t, buf[t % NBUF]);
                        else
                            load_hop(rin_n, rn, t - 8, buf[t % NBUF]);
                        if (d == EPF) epilogue_load<S, EPI, true>(a, r, cb, ops);
                        asm volatile("" ::: "memory");
                        apply_hop(d, buf[d % NBUF], acc);
                        pin_acc<R>(acc);
                    }
                    if constexpr (EPF >= 8) epilogue_load<S, EPI, true>(a, r, cb, ops);
                    epilogue_apply<S, EPI, true>(a, r, cb, acc, ops, part, valid);
                    write_block_partials<NP>(a, r, sb, sl, part);
                    if (!more) break;
                    r = rn;
                    rin = rin_n;
                }
            } else {
                while (m != 0) {
                    const int r = r0 + __builtin_ctzll(m) * LANES;
                    m &= m - 1;
                    const __amdgpu_buffer_rsrc_t rin = spinor_rsrc<S>(a.in, g.Vh, r);
                    double part[NP > 0 ? NP : 1];
#pragma unroll
                    for (int k = 0; k < (NP > 0 ? NP : 1); ++k) part[k] = 0.0;
                    cx<R> acc[12];
#pragma unroll
                    for (int e = 0; e < 12; ++e) acc[e] = {R(0), R(0)};
                    EpiOps<R, EPI> ops;
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        CxSpinor<R> cur;
                        load_hop(rin, r, d, cur);
                        if (d == EPF) epilogue_load<S, EPI, true>(a, r, cb, ops);
                        apply_hop(d, cur, acc);
                        pin_acc<R>(acc);
                    }
                    if constexpr (EPF >= 8) epilogue_load<S, EPI, true>(a, r, cb, ops);
                    epilogue_apply<S, EPI, true>(a, r, cb, acc, ops, part, valid);
                    write_block_partials<NP>(a, r, sb, sl, part);
                }
            }
        }
        if (a.live_count != nullptr && sl == 0 && nlive > 0) atomicAdd(a.live_count, nlive);
    }
}

template <typename S>
void launch_dslash_t(const DslashCall *c, int nseg, int kind, int nr, int bs, int persistent, hipStream_t s);

}  // namespace dl
