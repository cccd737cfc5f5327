"""Gaussian smearing and loops of smeared quark fields on the HIP path against the oracle.

Tolerances: the smearing operator in FP64 to 1e-13 of max |ref| (a few ulps of
the 6-hop sums per step, over a few steps; iters = 0 is an exact copy); loops
with the Cauchy-Schwarz normalisation of the parity suite, with the smeared
noise xi in place of eta (FP64 solves: GPU to 1e-12, oracle to 1e-13, error
below 1e-10); the truncated CGNR path in FP64 against the oracle's FP64 run of
the same 25 iterations to 1e-10 of the same scale.
"""
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


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev)


def from_dev(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("recon", [12, 18])
def test_smear_operator(dl, dev, recon):
    dims = (6, 4, 6, 10)
    U = synth.gauge_field(dims, 0.6, seed=501)
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64,), recon=recon)
    psi = synth.random_spinor(dims, 3, seed=502)
    x = to_dev(psi, dev)
    for alpha, iters in [(0.5, 5), (2.0, 1), (0.25, 0)]:
        out = from_dev(dl.smear(G, alpha, iters, x))
        for r in range(3):
            ref = oracle.smear(U, psi[r], dims, alpha, iters)
            if iters == 0:
                assert np.array_equal(out[r], ref)
            assert np.max(np.abs(out[r] - ref)) <= 1e-13 * np.max(np.abs(ref)), (recon, alpha, iters, r)


def cs_norm(dims, xis, sols):
    T = dims[3]
    per_t = int(np.prod(dims[:3]))
    out = np.zeros(T)
    for e, s in zip(xis, sols):
        v = np.linalg.norm(e.reshape(-1, 12), axis=1) * np.linalg.norm(s.reshape(-1, 12), axis=1)
        out += v.reshape(T, per_t).sum(axis=1)
    return out


@pytest.mark.parametrize("scheme", [0, 1])
def test_smeared_loops_fp64(dl, dev, scheme):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, seed=511)
    kappa, alpha, iters = 0.122, 0.4, 3
    G = dl.Gauge(dl.Lattice(dims, 1), U)
    gam = [0, 15, 5]
    L, st = dl.loops_smeared(G, kappa, dl.z2_sources(5110, 2, first_noise=1, scheme=scheme), alpha, iters, gam,
                             dl.solve_params(tol=1e-12, maxiter=500))
    assert all(s[0] == dl.DL_OK for s in st)
    ref = oracle.loops_z2_smeared(U, dims, kappa, 5110, [1, 2], scheme, gam, alpha, iters, tol=1e-13)
    ncls = oracle.dilution_count(scheme)
    for n in range(2):
        xis, sols = [], []
        for d in range(ncls):
            eta = oracle.z2_source(dims, 5110, 1 + n, scheme, d if ncls > 1 else -1)
            xi = oracle.smear(U, eta, dims, alpha, iters)
            xis.append(xi)
            sols.append(oracle.solve(U, xi, dims, kappa, 1e-13)[0])
        norm = cs_norm(dims, xis, sols)
        err = np.abs(L[n] - ref[n]) / norm[None, :]
        assert np.max(err) < 1e-10, (scheme, n, np.max(err))


def test_smeared_loops_truncated_cgnr_fp64(dl, dev):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, seed=521)
    kappa, alpha, iters = 0.122, 0.6, 2
    G = dl.Gauge(dl.Lattice(dims, 1), U)
    gam = [0, 15]
    prm = dl.solve_params(solver=dl.DL_CGNR, prec=dl.DL_F64, fixed_iters=25)
    L, st = dl.loops_smeared(G, kappa, dl.z2_sources(5210, 2), alpha, iters, gam, prm)
    for n in range(2):
        xi = oracle.smear(U, oracle.z2_source(dims, 5210, n), dims, alpha, iters)
        s = oracle.solve_lp(U, xi, dims, kappa, niter=25)
        ref = oracle.loops_accumulate(dims, xi, s, gam)
        norm = cs_norm(dims, [xi], [s])
        assert np.max(np.abs(L[n] - ref) / norm[None, :]) < 1e-10, n
