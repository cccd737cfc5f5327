// dl_dslash_inst.hpp -- instantiation of the hopping kernel for one storage
// precision (included once per precision so the variants compile in parallel).
#pragma once

#include "dl_dslash.hpp"

namespace dl {

template <typename S, int NE, bool DAG, int EPI>
static void dslash_go_nr(const Segs<DKArgs> &B, int nr, int grid, int bs, hipStream_t s)
{
    if (nr == 2)
        hipLaunchKernelGGL((dslash_kernel<S, NE, DAG, EPI, 2>), dim3(grid), dim3(bs), 0, s, B);
    else
        hipLaunchKernelGGL((dslash_kernel<S, NE, DAG, EPI, 1>), dim3(grid), dim3(bs), 0, s, B);
}

template <typename S, int NE, bool DAG>
static void dslash_go_epi(const Segs<DKArgs> &B, int epi, int nr, int grid, int bs, hipStream_t s)
{
    switch (epi) {
    case EPI_PLAIN: dslash_go_nr<S, NE, DAG, EPI_PLAIN>(B, nr, grid, bs, s); break;
    case EPI_XPAY: dslash_go_nr<S, NE, DAG, EPI_XPAY>(B, nr, grid, bs, s); break;
    case EPI_XPAY_DOT: dslash_go_nr<S, NE, DAG, EPI_XPAY_DOT>(B, nr, grid, bs, s); break;
    case EPI_XPAY_TS: dslash_go_nr<S, NE, DAG, EPI_XPAY_TS>(B, nr, grid, bs, s); break;
    case EPI_XPAY_NRM: dslash_go_nr<S, NE, DAG, EPI_XPAY_NRM>(B, nr, grid, bs, s); break;
    case EPI_XMY_NRM: dslash_go_nr<S, NE, DAG, EPI_XMY_NRM>(B, nr, grid, bs, s); break;
    default: break;
    }
}

// c[0..nseg): calls with the same precision, link format, adjoint flag and
// epilogue; persistent > 0 caps the grid at that many blocks (a multiple of 8)
template <typename S>
void launch_dslash_t(const DslashCall *c, int nseg, int nr, int bs, int persistent, hipStream_t s)
{
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
        a.nblk = (c[k].g.Vh + bs - 1) / bs;
        a.partials = c[k].partials;
        a.active = c[k].active;
        a.live_count = c[k].live_count;
        B.prefix[k + 1] = B.prefix[k] + a.nblk * ((c[k].nrhs + nr - 1) / nr);
    }
    const int total = B.prefix[nseg];
    const int grid = (persistent > 0 && total > persistent) ? persistent : total;
    const DslashCall &c0 = c[0];
    if (c0.recon == 12) {
        if (c0.dag)
            dslash_go_epi<S, 6, true>(B, c0.epi, nr, grid, bs, s);
        else
            dslash_go_epi<S, 6, false>(B, c0.epi, nr, grid, bs, s);
    } else {
        if (c0.dag)
            dslash_go_epi<S, 9, true>(B, c0.epi, nr, grid, bs, s);
        else
            dslash_go_epi<S, 9, false>(B, c0.epi, nr, grid, bs, s);
    }
}

}  // namespace dl
