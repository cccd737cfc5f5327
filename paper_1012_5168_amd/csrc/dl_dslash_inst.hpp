// dl_dslash_inst.hpp -- instantiation of the hopping kernel for one storage
// precision (included once per precision so the variants compile in parallel).
#pragma once

#include "dl_dslash.hpp"

namespace dl {

template <typename S, int NE, bool DAG, int EPI>
static void dslash_go_nr(const DKArgs &a, int nr, int grid, int bs, hipStream_t s)
{
    if (nr == 2)
        hipLaunchKernelGGL((dslash_kernel<S, NE, DAG, EPI, 2>), dim3(grid), dim3(bs), 0, s, a);
    else
        hipLaunchKernelGGL((dslash_kernel<S, NE, DAG, EPI, 1>), dim3(grid), dim3(bs), 0, s, a);
}

template <typename S, int NE, bool DAG>
static void dslash_go_epi(const DKArgs &a, int epi, int nr, int grid, int bs, hipStream_t s)
{
    switch (epi) {
    case EPI_PLAIN: dslash_go_nr<S, NE, DAG, EPI_PLAIN>(a, nr, grid, bs, s); break;
    case EPI_XPAY: dslash_go_nr<S, NE, DAG, EPI_XPAY>(a, nr, grid, bs, s); break;
    case EPI_XPAY_DOT: dslash_go_nr<S, NE, DAG, EPI_XPAY_DOT>(a, nr, grid, bs, s); break;
    case EPI_XPAY_TS: dslash_go_nr<S, NE, DAG, EPI_XPAY_TS>(a, nr, grid, bs, s); break;
    case EPI_XPAY_NRM: dslash_go_nr<S, NE, DAG, EPI_XPAY_NRM>(a, nr, grid, bs, s); break;
    case EPI_XMY_NRM: dslash_go_nr<S, NE, DAG, EPI_XMY_NRM>(a, nr, grid, bs, s); break;
    default: break;
    }
}

template <typename S>
void launch_dslash_t(const DslashCall &c, int nr, int bs, hipStream_t s)
{
    DKArgs a;
    a.g = c.g;
    a.parity = c.parity;
    a.in = c.in;
    a.out = c.out;
    a.x = c.x;
    a.y = c.y;
    a.links = c.links;
    a.a = c.a;
    a.nrhs = c.nrhs;
    a.nblk = (c.g.Vh + bs - 1) / bs;
    a.partials = c.partials;
    a.active = c.active;
    a.live_count = c.live_count;
    const int groups = (c.nrhs + nr - 1) / nr;
    const int grid = a.nblk * groups;
    if (c.recon == 12) {
        if (c.dag)
            dslash_go_epi<S, 6, true>(a, c.epi, nr, grid, bs, s);
        else
            dslash_go_epi<S, 6, false>(a, c.epi, nr, grid, bs, s);
    } else {
        if (c.dag)
            dslash_go_epi<S, 9, true>(a, c.epi, nr, grid, bs, s);
        else
            dslash_go_epi<S, 9, false>(a, c.epi, nr, grid, bs, s);
    }
}

}  // namespace dl
