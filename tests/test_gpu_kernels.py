"""Both hopping kernels (the item kernel and the LDS-link kernel, the latter
at several wavefront counts, occupancy limits and region sizes, regions
larger than a lattice's share of an XCD included; FP64 with its temporal
links in registers) against the
FP64 oracle, each pinned through DL_TUNE so that none depends on which one the
autotuner prefers on the day.

Shapes are chosen so that a 64-site block and the region walk have ragged
ends: 6x4x6x10 has 720 sites per parity (11 full blocks and a 16-site tail),
and odd right-hand-side counts leave wavefronts of the LDS kernel idle; 300
right-hand sides take every wavefront count over more than one 64-lane chunk.

Tolerances are those of the parity suite: FP64 operators 1e-13 of max |ref|,
FP32 2e-6, FP16 4e-3, BF16 3e-2; FP64 solves to 1e-12 checked with the
oracle's operator; the truncated FP16 CGNR against the FP64 oracle run of the
same algorithm within 3e-2.
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# the two default pins, and LDS-link variants with other wavefront counts, occupancy limits and regions
@pytest.fixture(params=["item", "lds", "cfg:1:2:0:64", "cfg:1:4:2:32", "cfg:1:1:1:128"])
def kernel(request):
    old = os.environ.get("DL_TUNE")
    os.environ["DL_TUNE"] = request.param
    yield request.param
    if old is None:
        del os.environ["DL_TUNE"]
    else:
        os.environ["DL_TUNE"] = old


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev)


def from_dev(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dims,nrhs", [((6, 4, 6, 10), 5), ((4, 4, 4, 4), 1), ((8, 6, 4, 10), 3)])
def test_operators_fp64_both_kernels(dl, dev, kernel, dims, nrhs):
    U = synth.gauge_field(dims, 0.6, seed=301)
    lat = dl.Lattice(dims, 1)
    par = oracle.parity(dims)
    psi = synth.random_spinor(dims, nrhs, seed=302)
    x = to_dev(psi, dev)
    k = 0.131
    for recon in (12, 18):
        G = dl.Gauge(lat, U, precs=(dl.DL_F64,), recon=recon)
        for op in (dl.DL_OP_DHOP, dl.DL_OP_DHOPDAG, dl.DL_OP_MHAT, dl.DL_OP_MHATDAG):
            out = from_dev(dl.apply(G, k, op, x))
            for r in range(nrhs):
                if op in (dl.DL_OP_DHOP, dl.DL_OP_DHOPDAG):
                    ref = oracle.dhop(U, psi[r], dims, 1, dag=op == dl.DL_OP_DHOPDAG)
                else:
                    pe = psi[r].copy()
                    pe[par == 1] = 0
                    ref = oracle.apply_mhat(U, pe, dims, k, 1, dag=op == dl.DL_OP_MHATDAG)
                    ref[par == 1] = 0
                err = np.max(np.abs(out[r] - ref))
                assert err <= 1e-13 * np.max(np.abs(ref)), (kernel, recon, op, r, err)


@pytest.mark.parametrize("prec,tol", [(1, 2e-6), (2, 4e-3), (3, 3e-2)])
def test_operators_reduced_precision_both_kernels(dl, dev, kernel, prec, tol):
    dims = (6, 4, 6, 10)
    U = synth.gauge_field(dims, 0.6, seed=311)
    lat = dl.Lattice(dims, 1)
    psi = synth.random_spinor(dims, 3, seed=312)
    x = to_dev(psi, dev)
    for recon in (12, 18):
        G = dl.Gauge(lat, U, precs=(dl.DL_F64, prec), recon=recon)
        out = from_dev(dl.apply(G, 0.13, dl.DL_OP_DHOP, x, prec=prec))
        for r in range(3):
            ref = oracle.dhop(U, psi[r], dims)
            err = np.max(np.abs(out[r] - ref)) / np.max(np.abs(ref))
            assert err <= tol, (kernel, recon, prec, r, err)


def test_solve_fp64_both_kernels(dl, dev, kernel):
    """BiCGStab runs every reducing epilogue (dot products, the omega pair, the true residual)
    through the kernel under test; right-hand sides converge at different iterations, so the
    active masks are exercised too."""
    dims = (6, 4, 6, 10)
    U = synth.gauge_field(dims, 0.5, seed=321)
    kappa = 0.124
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    b = synth.random_spinor(dims, 5, seed=322)
    b[1] *= 1e-3  # a different scale changes nothing in relative terms but the rounding
    b[3, :, 2:] = 0  # a source on two spins only converges on its own schedule
    x, st = dl.solve(G, kappa, to_dev(b, dev), dl.solve_params(tol=1e-12, maxiter=800))
    x = from_dev(x)
    for r in range(5):
        status, iters, upd, res = st[r]
        assert status == dl.DL_OK and res <= 1e-12, (kernel, r, st[r])
        rr = np.linalg.norm(b[r] - oracle.apply_m(U, x[r], dims, kappa)) / np.linalg.norm(b[r])
        assert rr <= 1.5e-12, (kernel, r, rr)


def test_truncated_cgnr_fp16_both_kernels(dl, dev, kernel):
    dims = (6, 4, 6, 10)
    U = synth.gauge_field(dims, 0.5, seed=331)
    kappa = 0.125
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64, dl.DL_F16))
    b = synth.random_spinor(dims, 3, seed=332)
    x, st = dl.solve(G, kappa, to_dev(b, dev),
                     dl.solve_params(solver=dl.DL_CGNR, prec=dl.DL_F16, fixed_iters=25))
    x = from_dev(x)
    for r in range(3):
        ref = oracle.solve_lp(U, b[r], dims, kappa, niter=25)
        err = np.linalg.norm(x[r] - ref) / np.linalg.norm(ref)
        assert err < 3e-2, (kernel, r, err)


def test_mixed_fp32_both_kernels(dl, dev, kernel):
    dims = (6, 4, 6, 10)
    U = synth.gauge_field(dims, 0.5, seed=341)
    kappa = 0.12
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64, dl.DL_F32))
    b = synth.random_spinor(dims, 3, seed=342)
    x, st = dl.solve(G, kappa, to_dev(b, dev), dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000))
    x = from_dev(x)
    for r in range(3):
        assert st[r][0] == dl.DL_OK and st[r][3] <= 1e-10, (kernel, st[r])
        rr = np.linalg.norm(b[r] - oracle.apply_m(U, x[r], dims, kappa)) / np.linalg.norm(b[r])
        assert rr <= 1.2e-10, (kernel, r, rr)


def test_batch_segments_both_kernels(dl, dev, kernel):
    """Two lattices of different size in one batched launch sequence: each lattice's loops
    equal its own single-lattice run (the segment walk of either kernel must not mix operands)."""
    shapes = [((4, 4, 4, 6), 0.4, 0.12), ((6, 4, 6, 10), 0.5, 0.124)]
    gauges, kappas, srcs = [], [], []
    for i, (dims, eps, kap) in enumerate(shapes):
        U = synth.gauge_field(dims, eps, seed=351 + i)
        gauges.append(dl.Gauge(dl.Lattice(dims, 1), U))
        kappas.append(kap)
        srcs.append(dl.z2_sources(360 + i, 2, scheme=dl.DL_DIL_SPIN_COLOUR))
    prm = dl.solve_params(tol=1e-12, maxiter=800)
    Ls, sts = dl.batch_loops(gauges, kappas, srcs, [0, 15], prm)
    for G, kap, src, L, st in zip(gauges, kappas, srcs, Ls, sts):
        assert all(s[0] == dl.DL_OK for s in st)
        L1, _ = dl.loops(G, kap, src, [0, 15], prm)
        assert np.max(np.abs(L1 - L)) <= 1e-10 * np.max(np.abs(L1)), (kernel, np.max(np.abs(L1 - L)))


def test_many_rhs_chunks_both_kernels(dl, dev, kernel):
    """300 right-hand sides: more than one 64-lane chunk of every wavefront count (64 x 4 = 256
    at most), with a ragged last chunk.  The hopping term of all 300 equals the oracle's; then
    BiCGStab on sources of five kinds (random, scaled, point, one timeslice, two spins), which
    converge at different iterations, so that right-hand sides of later chunks stop while
    those of the first still iterate: every solution meets the oracle's operator residual."""
    dims = (6, 4, 6, 10)
    n = 300
    U = synth.gauge_field(dims, 0.3, seed=371)  # a rough field near the critical kappa: ~50 iterations
    kappa = 0.15
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    b = synth.random_spinor(dims, n, seed=372)
    V = int(np.prod(dims))
    tsl = np.arange(V) // (dims[0] * dims[1] * dims[2])
    for r in range(n):
        kind = r % 5
        if kind == 1:
            b[r] *= 1e-3
        elif kind == 2:
            site, sc = (37 * r) % V, r % 12
            b[r] = 0
            b[r, site, sc // 3, sc % 3] = 1.0 - 0.5j
        elif kind == 3:
            b[r][tsl != r % dims[3]] = 0
        elif kind == 4:
            b[r, :, 2:] = 0
    x = to_dev(b, dev)
    out = from_dev(dl.apply(G, kappa, dl.DL_OP_DHOP, x))
    for r in range(n):
        ref = oracle.dhop(U, b[r], dims, 1)
        err = np.max(np.abs(out[r] - ref))
        assert err <= 1e-13 * np.max(np.abs(ref)), (kernel, r, err)
    sol, st = dl.solve(G, kappa, x, dl.solve_params(tol=1e-12, maxiter=2000))
    sol = from_dev(sol)
    assert len({s[1] for s in st}) >= 3, (kernel, sorted({s[1] for s in st}))
    for r in range(n):
        status, iters, upd, res = st[r]
        assert status == dl.DL_OK and res <= 1e-12, (kernel, r, st[r])
        rr = np.linalg.norm(b[r] - oracle.apply_m(U, sol[r], dims, kappa)) / np.linalg.norm(b[r])
        assert rr <= 1.5e-12, (kernel, r, rr)


@pytest.mark.gpu
def test_stream_probe_copies_and_reads(dl, dev):
    """The streaming probe behind the bench's measured ceilings: mode 0 copies every byte of a
    ragged buffer (not a multiple of the 2048-word tiles: the tail loop runs too), mode 1 reads
    without writing, and both report a positive time."""
    n = (1 << 22) + 6  # complex128 entries: 16-byte words, ragged
    a = torch.randn(n, dtype=torch.complex128, device=dev)
    b = torch.zeros_like(a)
    sec = dl.stream_probe(a, b, 0, reps=2)
    torch.cuda.synchronize()
    assert sec > 0
    assert torch.equal(a, b)
    c = torch.zeros(1 << 14, dtype=torch.float64, device=dev)  # 128 KiB
    sec = dl.stream_probe(a, c, 1, reps=2)
    torch.cuda.synchronize()
    assert sec > 0
    assert torch.count_nonzero(c).item() == 0
    with pytest.raises(dl.DLError):
        dl.stream_probe(a, c, 0)  # dst too small for a copy
