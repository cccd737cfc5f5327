"""The entry point that allocates nothing (dl_apply_noalloc), through the C ABI, against dl_apply.

Two calls in a row, the second with a smaller input, each compared with dl_apply on the same input:
the two entry points launch the same kernels on the same packed fields (only where those fields live
differs), so the results agree within the FP64 operator bar of 1e-13 relative (bit-identical when the
launch configurations coincide).  A request larger than the scratch is refused before any device work.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def check(dl, G, kappa, op, prec, x):
    n = x.shape[0]
    ref = torch.empty_like(x)
    got = torch.full_like(x, float("nan"))
    dl.dl_apply(G.h, kappa, op, prec, x, ref, n)
    dl.dl_apply_noalloc(G.h, kappa, op, prec, x, got, n)
    torch.cuda.synchronize()
    r, g = ref.cpu().numpy(), got.cpu().numpy()
    err = np.max(np.abs(g - r))
    assert np.all(np.isfinite(g)), (op, prec)
    assert err <= 1e-13 * np.max(np.abs(r)), (op, prec, err)


def test_noalloc_matches_dl_apply_twice_second_smaller(dl, dev):
    w = synth.WORKLOADS["plain_16x16x16x32"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64,))
    x = torch.from_numpy(synth.random_spinor(dims, 1, seed=801)).to(dev)
    # first call: the largest FP64 request at 16^3 x 32 (five packed fields of one right-hand side)
    check(dl, G, kappa, dl.DL_OP_MHAT, dl.DL_F64, x)
    # second call, smaller: three right-hand sides on 4^3 x 8, every operator
    dims2 = (4, 4, 4, 8)
    U2 = synth.gauge_field(dims2, 0.5, seed=802)
    G2 = dl.Gauge(dl.Lattice(dims2, 1), U2, precs=(dl.DL_F64, dl.DL_F16))
    x2 = torch.from_numpy(synth.random_spinor(dims2, 3, seed=803)).to(dev)
    for op in (dl.DL_OP_DHOP, dl.DL_OP_DHOPDAG, dl.DL_OP_M, dl.DL_OP_MDAG, dl.DL_OP_MHAT, dl.DL_OP_MHATDAG):
        check(dl, G2, 0.13, op, dl.DL_F64, x2)
    # another storage precision, and back to the large lattice on its plain operator
    check(dl, G2, 0.13, dl.DL_OP_M, dl.DL_F16, x2)
    check(dl, G, kappa, dl.DL_OP_M, dl.DL_F64, x)


def test_noalloc_refuses_more_than_the_scratch(dl, dev):
    dims = (16, 16, 16, 32)
    U = synth.gauge_field(dims, 0.35, seed=804)
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64,))
    x = torch.zeros((2, 16 * 16 * 16 * 32, 4, 3), dtype=torch.complex128, device=dev)
    out = torch.empty_like(x)
    with pytest.raises(dl.DLError) as e:
        dl.dl_apply_noalloc(G.h, 0.15, dl.DL_OP_M, dl.DL_F64, x, out, 2)
    assert e.value.code == dl.DL_EINVAL and "scratch" in str(e.value)
