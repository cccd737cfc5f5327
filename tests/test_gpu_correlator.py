"""The disconnected correlator (Eq. 2) of the HIP path against the oracle's plain
double sum over distinct noise pairs, through the C ABI.

Inputs: seeded random per-noise loops, and per-noise loops the oracle computes
on a 4^4 field (5 complex-Z2 noises, Gamma = 1 and gamma5).  Tolerance: the
kernel sums all pairs minus the same-noise pairs, the oracle sums the distinct
pairs directly, both in FP64: |gpu - oracle| <= 1e-12 of the scale
sum_{n != m} sum_t |L_B^n(t)| |L_A^m(t + dt)| / (N (N-1) L^3 T).
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


def scale(lb, la, L3):
    n, T = lb.shape
    ab, aa = np.abs(lb).sum(axis=0), np.abs(la).sum(axis=0)
    # sum over all pairs bounds the distinct-pair sum
    return np.array([np.sum(ab * np.roll(aa, -dt)) for dt in range(T)]) / (n * (n - 1) * L3 * T)


@pytest.mark.parametrize("n,T", [(2, 1), (2, 4), (7, 10), (33, 6)])
def test_correlator_random_loops(dl, dev, n, T):
    rng = np.random.default_rng(400 + n * T)
    lb = rng.normal(size=(n, T)) + 1j * rng.normal(size=(n, T)) + 2.0
    la = rng.normal(size=(n, T)) + 1j * rng.normal(size=(n, T)) - 1.0j
    L3 = 512
    got = dl.disconnected_correlator(lb, la, L3)
    ref = oracle.disconnected_correlator(lb, la, L3)
    assert np.all(np.abs(got - ref) <= 1e-12 * scale(lb, la, L3)), np.max(np.abs(got - ref))


def test_correlator_of_oracle_loops(dl, dev):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, seed=411)
    L = oracle.loops_z2(U, dims, 0.12, 2411, range(5), oracle.SCHEME_SPIN_COLOUR, [0, 15], tol=1e-12)
    for b, a in ((0, 0), (1, 1), (1, 0)):
        got = dl.disconnected_correlator(L[:, b], L[:, a], 64)
        ref = oracle.disconnected_correlator(L[:, b], L[:, a], 64)
        assert np.all(np.abs(got - ref) <= 1e-12 * scale(L[:, b], L[:, a], 64)), (b, a)


def test_correlator_repeatable(dl, dev):
    rng = np.random.default_rng(420)
    lb = rng.normal(size=(50, 16)) + 1j * rng.normal(size=(50, 16))
    la = rng.normal(size=(50, 16)) + 1j * rng.normal(size=(50, 16))
    a = dl.disconnected_correlator(lb, la, 4096)
    b = dl.disconnected_correlator(lb, la, 4096)
    assert np.array_equal(a, b)
