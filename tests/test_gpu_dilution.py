"""Colour, spin, spin-parity and time dilution on the HIP path against the oracle.

Sources must be bit-exact (integer work: the noise stream and the class masks);
loop estimates follow the FP64 tolerance of the parity suite: the error
normalised by the Cauchy-Schwarz scale sum_d sum_{x in t} |eta_d(x)| |s_d(x)|
stays below 1e-10 with the GPU solving to 1e-12 and the oracle to 1e-13.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NEW_SCHEMES = [s for s in range(128) if oracle.dilution_valid(s) and s & (8 | 16 | 32 | 64)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def from_dev(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_sources_bit_exact_new_schemes(dl, dev):
    dims = (4, 2, 2, 6)
    lat = dl.Lattice(dims, 1)
    V = lat.V
    for scheme in NEW_SCHEMES:
        src = dl.z2_sources(3000 + scheme, 2, first_noise=7, scheme=scheme)
        n = dl.dl_sources_count(lat.h, src)
        ncls = oracle.dilution_count(scheme)
        assert n == 2 * ncls
        out = torch.empty((n, V, 4, 3), dtype=torch.complex128, device=dev)
        dl.dl_sources_fill(lat.h, src, 0, n, out)
        got = from_dev(out)
        for r in range(n):
            ref = oracle.z2_source(dims, 3000 + scheme, 7 + r // ncls, scheme, (r % ncls) if ncls > 1 else -1)
            assert np.array_equal(got[r], ref), (scheme, r)


def cs_norm(dims, etas, sols):
    T = dims[3]
    per_t = int(np.prod(dims[:3]))
    out = np.zeros(T)
    for e, s in zip(etas, sols):
        v = np.linalg.norm(e.reshape(-1, 12), axis=1) * np.linalg.norm(s.reshape(-1, 12), axis=1)
        out += v.reshape(T, per_t).sum(axis=1)
    return out


@pytest.mark.parametrize("scheme", [32 | 2, 8 | 4, 64, 64 | 16 | 8, 16])
def test_loops_new_schemes_fp64(dl, dev, scheme):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, seed=3131)
    kappa = 0.122
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    gam = [0, 15, 5]
    n_noise = 2
    L, st = dl.loops(G, kappa, dl.z2_sources(3200, n_noise, first_noise=5, scheme=scheme), gam,
                     dl.solve_params(tol=1e-12, maxiter=500))
    assert all(s[0] == dl.DL_OK for s in st)
    ref, sols = oracle.loops_z2(U, dims, kappa, 3200, range(5, 5 + n_noise), scheme, gam, tol=1e-13,
                                return_solutions=True)
    ncls = oracle.dilution_count(scheme)
    for n in range(n_noise):
        etas = [oracle.z2_source(dims, 3200, 5 + n, scheme, d if ncls > 1 else -1) for d in range(ncls)]
        norm = cs_norm(dims, etas, sols[n * ncls:(n + 1) * ncls])
        nz = norm > 0
        err = np.abs(L[n][:, nz] - ref[n][:, nz]) / norm[None, nz]
        assert np.max(err) < 1e-10, (scheme, n, np.max(err))
        if scheme & 64:  # time dilution: zero off the noise's timeslice, exactly
            off = np.arange(dims[3]) != (5 + n) % dims[3]
            assert np.all(L[n][:, off] == 0), scheme
