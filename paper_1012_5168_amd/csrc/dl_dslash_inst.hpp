// dl_dslash_inst.hpp -- instantiation of the hopping kernel for one storage
// precision (included once per precision so the variants compile in parallel).
#pragma once

#include <algorithm>

#include "dl_dslash.hpp"

namespace dl {

template <typename S, int NE, bool DAG, int EPI, int LANES>
static void dslash_go_lds(const Segs<DKArgs> &B, int occ, int grid, int rb, hipStream_t s)
{
    if (occ == 1)
        hipLaunchKernelGGL((dslash_lds_kernel<S, NE, DAG, EPI, LANES, 1>), dim3(grid), dim3(LANES * LDS_SITES), 0, s, B, rb);
    else if (occ == 2)
        hipLaunchKernelGGL((dslash_lds_kernel<S, NE, DAG, EPI, LANES, 2>), dim3(grid), dim3(LANES * LDS_SITES), 0, s, B, rb);
    else
        hipLaunchKernelGGL((dslash_lds_kernel<S, NE, DAG, EPI, LANES, 0>), dim3(grid), dim3(LANES * LDS_SITES), 0, s, B, rb);
}

// kind 1 (LDS-link kernel): nr wavefronts per block, `occ` wavefronts per SIMD
// at most (0: as compiled), regions of rb blocks; kind 0 (item kernel): nr
// right-hand sides per thread, bs sites per block
template <typename S, int NE, bool DAG, int EPI>
static void dslash_go_nr(const Segs<DKArgs> &B, int kind, int nr, int grid, int bs, int rb, hipStream_t s)
{
    if constexpr (lds_link_bytes<S, NE>() <= LDS_WORKGROUP_BYTES) {
        if (kind == 1) {
            if (nr == 4)
                dslash_go_lds<S, NE, DAG, EPI, 4>(B, bs, grid, rb, s);
            else if (nr == 2)
                dslash_go_lds<S, NE, DAG, EPI, 2>(B, bs, grid, rb, s);
            else
                dslash_go_lds<S, NE, DAG, EPI, 1>(B, bs, grid, rb, s);
            return;
        }
    }
    if (nr == 2)
        hipLaunchKernelGGL((dslash_kernel<S, NE, DAG, EPI, 2>), dim3(grid), dim3(bs), 0, s, B);
    else
        hipLaunchKernelGGL((dslash_kernel<S, NE, DAG, EPI, 1>), dim3(grid), dim3(bs), 0, s, B);
}

template <typename S, int NE, bool DAG>
static void dslash_go_epi(const Segs<DKArgs> &B, int epi, int kind, int nr, int grid, int bs, int rb, hipStream_t s)
{
    switch (epi) {
    case EPI_PLAIN: dslash_go_nr<S, NE, DAG, EPI_PLAIN>(B, kind, nr, grid, bs, rb, s); break;
    case EPI_XPAY: dslash_go_nr<S, NE, DAG, EPI_XPAY>(B, kind, nr, grid, bs, rb, s); break;
    case EPI_XPAY_DOT: dslash_go_nr<S, NE, DAG, EPI_XPAY_DOT>(B, kind, nr, grid, bs, rb, s); break;
    case EPI_XPAY_TS: dslash_go_nr<S, NE, DAG, EPI_XPAY_TS>(B, kind, nr, grid, bs, rb, s); break;
    case EPI_XPAY_NRM: dslash_go_nr<S, NE, DAG, EPI_XPAY_NRM>(B, kind, nr, grid, bs, rb, s); break;
    case EPI_XMY_NRM: dslash_go_nr<S, NE, DAG, EPI_XMY_NRM>(B, kind, nr, grid, bs, rb, s); break;
    case EPI_CG_R:  // only the adjoint hop of the normal equations uses it
        if constexpr (DAG) dslash_go_nr<S, NE, DAG, EPI_CG_R>(B, kind, nr, grid, bs, rb, s);
        break;
    default: break;
    }
}

// whether the LDS-link kernel exists for this storage precision and link format
template <typename S>
bool dslash_lds_ok_t(int recon)
{
    return recon == 12 ? lds_link_bytes<S, 6>() <= LDS_WORKGROUP_BYTES : lds_link_bytes<S, 9>() <= LDS_WORKGROUP_BYTES;
}

// c[0..nseg): calls with the same precision, link format, adjoint flag and
// epilogue.  kind 0: the item kernel with nr right-hand sides per thread and
// bs sites per workgroup; persistent > 0 caps its grid at that many blocks (a
// multiple of 8).  kind 1: the LDS-link kernel with nr wavefronts per
// workgroup, at most bs wavefronts per SIMD (0: as compiled) and regions of
// `persistent` site blocks.
// whether every segment's per-right-hand-side field fits the 32-bit offsets of
// the LDS-link kernel's buffer loads
template <typename S>
bool dslash_lds_fits(const DslashCall *c, int nseg)
{
    for (int k = 0; k < nseg; ++k)
        if (12LL * plane_stride(c[k].g.Vh) * (long long)sizeof(typename Fmt<S>::E) >= (1LL << 31)) return false;
    return true;
}

template <typename S>
void launch_dslash_t(const DslashCall *c, int nseg, int kind, int nr, int bs, int persistent, hipStream_t s)
{
    if (kind == 1 && (!dslash_lds_ok_t<S>(c[0].recon) || !dslash_lds_fits<S>(c, nseg))) {
        kind = 0;
        nr = 1;
        bs = 256;
        persistent = 0;
    }
    // the LDS-link kernel's blocks hold LDS_SITES sites; its bs selects the occupancy
    const int blk = kind == 1 ? LDS_SITES : bs;
    Segs<DKArgs> B;
    B.n = nseg;
    B.prefix[0] = 0;
    for (int k = 0; k < nseg; ++k) {
        DKArgs &a = B.a[k];
        a.g = c[k].g;
        a.parity = c[k].parity;
        a.in = c[k].in;
        a.out = c[k].out;
        a.x = c[k].x;
        a.y = c[k].y;
        a.links = c[k].links;
        a.a = c[k].a;
        a.nrhs = c[k].nrhs;
        a.nblk = (c[k].g.Vh + blk - 1) / blk;
        a.partials = c[k].partials;
        a.active = c[k].active;
        a.live_count = c[k].live_count;
        a.st = c[k].st;
        const int groups = kind == 1 ? 1 : (c[k].nrhs + nr - 1) / nr;
        B.prefix[k + 1] = B.prefix[k] + a.nblk * groups;
    }
    const int total = B.prefix[nseg];
    int grid, rb = 0;
    if (kind == 1) {
        rb = persistent > 0 ? persistent : 64;
        // a region is at most an XCD's share, so that every XCD gets work on
        // lattices of fewer than 8 rb site blocks
        rb = std::max(1, std::min(rb, (total + 7) / 8));
        const int nreg = (total + rb - 1) / rb;
        grid = 8 * ((nreg + 7) / 8) * rb;
    } else {
        grid = (persistent > 0 && total > persistent) ? persistent : total;
    }
    const DslashCall &c0 = c[0];
    if (c0.recon == 12) {
        if (c0.dag)
            dslash_go_epi<S, 6, true>(B, c0.epi, kind, nr, grid, bs, rb, s);
        else
            dslash_go_epi<S, 6, false>(B, c0.epi, kind, nr, grid, bs, rb, s);
    } else {
        if (c0.dag)
            dslash_go_epi<S, 9, true>(B, c0.epi, kind, nr, grid, bs, rb, s);
        else
            dslash_go_epi<S, 9, false>(B, c0.epi, kind, nr, grid, bs, rb, s);
    }
}

}  // namespace dl
