"""Pins of the FP64 CPU oracle against things other than itself.

Each test ties one part of the oracle to mathematics or to a library routine
that does not share its code:

* Dirac algebra: Clifford relations, hermiticity, gamma_5 = g1 g2 g3 g4 =
  diag(1,1,-1,-1) (the chiral basis), Gamma_5 = g1 g3.
* Hopping term: the free-field (U = 1) propagator M^-1(x, 0) built in
  momentum space with numpy -- including the antiperiodic time momenta and the
  2-site extents where forward and backward hops reach the same site; gauge
  covariance D[U^Omega] Omega psi = Omega D[U] psi for a random SU(3) rotation;
  the diagonal of D^2, D^3 (zero) and D^4 (-8 times the sum of colour-traced
  plaquette paths, the paths built from the link array in the test); and
  gamma_5-hermiticity of the directly assembled M^dagger.
* Solver and contraction: dense LU (numpy.linalg.inv) on 2^4 and 4^3 x 4,
  point-source loops against the dense diagonal, the real / imaginary classes
  of Tr[Gamma M^-1(x,x)], gauge invariance of exact loops.
* Noise and dilution: the counter form of SplitMix64 against the generator
  stepped sequentially and against the published known-answer outputs for
  seed 0 (tests/golden/); every entry in {(+-1 +-i)/sqrt 2}, phase balance,
  unbiasedness and the closed-form variance sum_{i!=j} |A_ij|^2 of the complex
  Z2 trace estimator, dilution classes against coordinates computed here; for
  every valid scheme the diluted pieces partition the noise and each piece is
  supported where its class says (spin / colour / spin parity slices, cubic
  vertices, site parity, and the one timeslice noise mod T of time dilution,
  all sliced with numpy); the diluted estimator's expectation is the exact
  trace and its variance the closed form restricted to same-class pairs.
* Truncated solver method: exact when the low-precision solve is exact,
  unbiased (z-test against the dense exact answer).
* Derivatives: d/dkappa against central differences with identical noise and
  against the dense M^-1 D M^-1; the link gradient against directional
  central differences.
* Smearing: free-field plane waves are eigenvectors with eigenvalue
  [(1 + 2 alpha sum_i cos p_i) / (1 + 6 alpha)]^iters; gauge covariance;
  hermiticity; a field on one timeslice and one spin stays there; the smeared
  loop driver equals dense algebra (xi = S eta, s = M^-1 xi from numpy's
  inverse), and the smeared estimator's mean is Tr[P_t Gamma S M^-1 S] (z-test,
  S assembled column by column from the smearing of unit vectors).
* Disconnected correlator (Eq. 2): identical per-noise estimates against the
  circular cross-correlation computed with numpy's FFT (convolution theorem);
  unbiasedness over distinct noise pairs when the two loops of one noise are
  correlated (z-test), with the same-noise estimator's expectation z-tested
  against its closed-form bias -c E[xi^2] / (N L^3) at dt = 0, ten standard
  errors from zero on the same data; the B <-> A swap symmetry D^BA(dt) = D^AB(T - dt).
* eta' combination and ratio fit (Eqs. 3-4): noise-free correlators built
  here from chosen (A, B, m_eta', m_pi) are fitted back exactly, and a wrong
  sign of B or a dropped backward-propagating term in the model would not
  fit them; Eq. 3 elementwise; configurations that differ only by a factor
  have zero jackknife errors; configurations whose ratios differ only in A
  give A's jackknife error as the standard error of the mean of the A_n
  (the closed form of the jackknife for a mean) and zero errors for B and m.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------ helpers written here


def sigma():
    return [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]


def chiral_gammas():
    """g1..g4 of the chiral basis, written from their block form."""
    Z = np.zeros((2, 2), complex)
    out = []
    for s in sigma():
        out.append(np.block([[Z, -1j * s], [1j * s, Z]]))
    out.append(np.block([[Z, np.eye(2)], [np.eye(2), Z]]))
    return out


def coords_of(dims):
    X, Y, Z, T = dims
    idx = np.arange(X * Y * Z * T)
    return np.stack([idx % X, (idx // X) % Y, (idx // (X * Y)) % Z, idx // (X * Y * Z)], axis=1)


def site_of(dims, c):
    X, Y, Z, T = dims
    return c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))


def free_propagator_column(dims, kappa, antiperiodic=True):
    """G(x, 0) = (1/V) sum_p exp(i p x) M(p)^-1, M(p) = 1 - 2k sum cos p + 2ik sum g sin p, [V][4][4]."""
    g = chiral_gammas()
    V = int(np.prod(dims))
    moms = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        if mu == 3 and antiperiodic:
            moms.append(np.pi * (2 * n + 1) / L)
        else:
            moms.append(2 * np.pi * n / L)
    cs = coords_of(dims)
    G = np.zeros((V, 4, 4), complex)
    for p in itertools.product(*moms):
        p = np.array(p)
        Mp = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        Minv = np.linalg.inv(Mp)
        G += np.exp(1j * cs @ p)[:, None, None] * Minv[None]
    return G / V


# ------------------------------------------------------------ Dirac algebra


def test_gamma_clifford_and_basis():
    g = [oracle.gamma(1 << mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * (mu == nu) * np.eye(4), atol=0)
    g5 = oracle.gamma(15)
    assert np.array_equal(g5, np.diag([1, 1, -1, -1]).astype(complex))
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3], atol=0)
    assert np.allclose(oracle.gamma(5), g[0] @ g[2], atol=0)
    assert np.allclose(oracle.gamma(0), np.eye(4), atol=0)
    # the basis written in block form here
    for mu, ref in enumerate(chiral_gammas()):
        assert np.allclose(g[mu], ref, atol=0)
    # the 16 Gamma_n are linearly independent (a basis of 4x4 matrices)
    B = np.stack([oracle.gamma(n).reshape(-1) for n in range(16)])
    assert np.linalg.matrix_rank(B) == 16


# ------------------------------------------------------------ hopping term


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 2, 2, 2), (2, 4, 2, 6)])
def test_free_field_propagator(dims):
    """M^-1(x, 0) for U = 1 against the momentum-space inverse, every entry."""
    kappa = 0.12
    U = synth.unit_field(dims)
    G = free_propagator_column(dims, kappa)
    V = int(np.prod(dims))
    for be in range(4):
        for b in range(3):
            e = oracle.point_source(dims, 0, be, b)
            s, _, res = oracle.solve(U, e, dims, kappa, tol=1e-13)
            ref = np.zeros((V, 4, 3), complex)
            ref[:, :, b] = G[:, :, be]
            assert np.max(np.abs(s - ref)) < 1e-12, (be, b)


def test_free_field_trace_closed_form():
    """Tr M^-1(x,x) = (12/V) sum_p A/(A^2 + 4k^2 sum sin^2 p), A = 1 - 2k sum cos p; L_Gamma = 0 for Gamma != 1."""
    dims, kappa = (4, 4, 4, 4), 0.12
    V = 256
    total = 0.0
    for n in itertools.product(range(4), range(4), range(4), range(4)):
        p = np.array([2 * np.pi * n[0] / 4, 2 * np.pi * n[1] / 4, 2 * np.pi * n[2] / 4, np.pi * (2 * n[3] + 1) / 4])
        A = 1 - 2 * kappa * np.cos(p).sum()
        total += A / (A * A + 4 * kappa * kappa * (np.sin(p) ** 2).sum())
    closed = 12 * total / V
    L = oracle.loops_point(synth.unit_field(dims), dims, kappa, 0, list(range(16)))
    assert abs(L[0, 0] - closed) < 1e-12
    assert np.max(np.abs(L[1:, 0])) < 1e-12
    assert np.max(np.abs(L[:, 1:])) == 0.0


def test_gauge_covariance_of_dhop():
    """D[U'](Omega psi) = Omega D[U] psi with U'_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^+."""
    dims = (4, 2, 4, 6)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.7, seed=11)
    Om = synth.random_su3(V, seed=12)
    cs = coords_of(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        c2 = cs.copy()
        c2[:, mu] = (c2[:, mu] + 1) % dims[mu]
        nb = site_of(dims, c2.T)
        Up[mu] = Om @ U[mu] @ np.conj(np.transpose(Om[nb], (0, 2, 1)))
    psi = synth.random_spinor(dims, 1, seed=13)[0]
    om_psi = np.einsum("xab,xsb->xsa", Om, psi)
    lhs = oracle.dhop(Up, om_psi, dims)
    rhs = np.einsum("xab,xsb->xsa", Om, oracle.dhop(U, psi, dims))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_gamma5_hermiticity_of_direct_mdag():
    """M^dagger assembled from its own hopping blocks equals gamma5 M gamma5 and the adjoint of M."""
    for dims in [(4, 4, 4, 4), (2, 2, 2, 2)]:
        U = synth.gauge_field(dims, 0.5, seed=21)
        x, y = synth.random_spinor(dims, 2, seed=22)
        g5 = np.array([1, 1, -1, -1])[None, :, None]
        k = 0.13
        mdag_y = oracle.apply_m(U, y, dims, k, dag=True)
        assert np.max(np.abs(mdag_y - g5 * oracle.apply_m(U, g5 * y, dims, k))) < 1e-14
        lhs = np.vdot(y, oracle.apply_m(U, x, dims, k))
        rhs = np.vdot(mdag_y, x)
        assert abs(lhs - rhs) < 1e-11


def test_closed_hopping_paths():
    """Diagonal blocks of D^n: zero for n = 1, 2, 3; for n = 4 the spin-colour trace is
    -8 x sum over the 48 plaquette paths through x of the colour trace of the path."""
    dims = (6, 5, 5, 6)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.6, seed=31)
    cs = coords_of(dims)
    g = chiral_gammas()

    def step(c, mu, sgn):
        """link matrix and boundary sign of one hop from coordinates c, and the new coordinates"""
        c2 = list(c)
        c2[mu] = (c2[mu] + sgn) % dims[mu]
        b = 1.0
        if mu == 3 and sgn > 0 and c[3] == dims[3] - 1:
            b = -1.0
        if mu == 3 and sgn < 0 and c[3] == 0:
            b = -1.0
        if sgn > 0:
            W = U[mu][site_of(dims, c)]
        else:
            W = np.conj(U[mu][site_of(dims, c2)]).T
        P = np.eye(4) - sgn * g[mu]
        return c2, b * W, P

    for x in [0, site_of(dims, (5, 4, 4, 5)), site_of(dims, (2, 3, 1, 0))]:
        c0 = tuple(cs[x])
        expected = 0.0
        for mu in range(4):
            for nu in range(4):
                if mu == nu:
                    continue
                for s1, s2 in itertools.product((1, -1), (1, -1)):
                    c, W1, P1 = step(c0, mu, s1)
                    c, W2, P2 = step(c, nu, s2)
                    c, W3, P3 = step(c, mu, -s1)
                    c, W4, P4 = step(c, nu, -s2)
                    assert tuple(c) == c0
                    spin = np.trace(P1 @ P2 @ P3 @ P4)
                    assert abs(spin + 8) < 1e-12
                    expected += spin * np.trace(W1 @ W2 @ W3 @ W4)
        diag = np.zeros((5, 12, 12), complex)
        for al in range(4):
            for a in range(3):
                v = oracle.point_source(dims, x, al, a)
                for n in range(1, 5):
                    v = oracle.dhop(U, v, dims)
                    diag[n][:, 3 * al + a] = v[x].reshape(-1)
        for n in (1, 2, 3):
            assert np.max(np.abs(diag[n])) < 1e-13
        assert abs(np.trace(diag[4]) - expected) < 1e-11
    assert V > 0


# ------------------------------------------------------------ solver and loops


@pytest.fixture(scope="module")
def dense_2x2x2x2():
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 0.5, seed=41)
    kappa = 0.12
    M = oracle.dense_m(U, dims, kappa)
    return dims, U, kappa, M, np.linalg.inv(M)


def test_dense_lu_solves_and_loops(dense_2x2x2x2):
    dims, U, kappa, M, Minv = dense_2x2x2x2
    b = synth.random_spinor(dims, 1, seed=42)[0]
    x, it, res = oracle.solve(U, b, dims, kappa, tol=1e-13)
    assert res <= 1e-13
    assert np.max(np.abs(x.reshape(-1) - Minv @ b.reshape(-1))) < 1e-12
    exact = oracle.exact_loops_dense(Minv, dims, list(range(16)))
    for site in range(int(np.prod(dims))):
        t = site // 8
        L = oracle.loops_point(U, dims, kappa, site, list(range(16)))
        # exact_loops_dense sums over the 8 sites of a timeslice; compare one site's trace
        blocks = Minv.reshape(16, 12, 16, 12)[site, :, site, :].reshape(4, 3, 4, 3)
        sp = np.einsum("aibi->ab", blocks)
        for g in range(16):
            ref = np.trace(oracle.gamma(g) @ sp)
            assert abs(L[g, t] - ref) < 1e-12
    # real / imaginary classes: Gamma with gamma5 Gamma^+ gamma5 = +Gamma give real loops
    real_class = {0, 7, 11, 13, 14, 15}
    g5 = oracle.gamma(15)
    for g in range(16):
        G = oracle.gamma(g)
        sign = +1 if np.allclose(g5 @ G.conj().T @ g5, G) else -1
        assert (sign > 0) == (g in real_class)
        vals = exact[g]
        if g in real_class:
            assert np.max(np.abs(vals.imag)) < 1e-13 * max(1, np.max(np.abs(vals)))
        else:
            assert np.max(np.abs(vals.real)) < 1e-13 * max(1, np.max(np.abs(vals)))


def test_dense_lu_4x4x4x4_loops():
    """All 16 exact L_Gamma(t) on 4^3 x 4 from the dense inverse vs point-source solves at one site
    per timeslice (sum over a timeslice needs all sites, so compare per-site traces)."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, seed=51)
    kappa = 0.12
    M = oracle.dense_m(U, dims, kappa)
    Minv = np.linalg.inv(M)
    for site in (0, 77, 255):
        t = site // 64
        L = oracle.loops_point(U, dims, kappa, site, list(range(16)), tol=1e-13)
        blocks = Minv.reshape(256, 12, 256, 12)[site, :, site, :].reshape(4, 3, 4, 3)
        sp = np.einsum("aibi->ab", blocks)
        for g in range(16):
            assert abs(L[g, t] - np.trace(oracle.gamma(g) @ sp)) < 1e-11


def test_exact_loops_gauge_invariant():
    dims = (4, 4, 2, 4)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.5, seed=61)
    Om = synth.random_su3(V, seed=62)
    cs = coords_of(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        c2 = cs.copy()
        c2[:, mu] = (c2[:, mu] + 1) % dims[mu]
        nb = site_of(dims, c2.T)
        Up[mu] = Om @ U[mu] @ np.conj(np.transpose(Om[nb], (0, 2, 1)))
    L1 = oracle.loops_point(U, dims, 0.12, 5, list(range(16)))
    L2 = oracle.loops_point(Up, dims, 0.12, 5, list(range(16)))
    assert np.max(np.abs(L1 - L2)) < 1e-12


# ------------------------------------------------------------ noise and dilution


def test_z2_entries_and_balance():
    dims = (4, 4, 4, 4)
    vals = np.concatenate([oracle.z2_source(dims, 2000, n).reshape(-1) for n in range(8)])
    s2 = np.sqrt(2.0)
    assert np.all(np.abs(np.abs(vals.real) * s2 - 1) < 1e-15)
    assert np.all(np.abs(np.abs(vals.imag) * s2 - 1) < 1e-15)
    quad = (vals.real < 0).astype(int) + 2 * (vals.imag < 0).astype(int)
    counts = np.bincount(quad, minlength=4)
    n = len(vals)
    chi2 = np.sum((counts - n / 4) ** 2 / (n / 4))
    assert chi2 < 16.3  # 3 dof, p = 0.001
    # lag-1 correlation of the real signs along the counter
    r = np.sign(vals.real)
    assert abs(np.mean(r[1:] * r[:-1])) < 4 / np.sqrt(n)


def _splitmix64_stream(seed, n):
    """The generator as published (Steele, Lea and Flood 2014): the state advances by the golden
    gamma each step and every output is the mix of the new state; stepped here one output at a
    time."""
    m = (1 << 64) - 1
    state, out = seed & m, []
    for _ in range(n):
        state = (state + 0x9E3779B97F4A7C15) & m
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_counter_equals_sequential_stream():
    """The counter form (output c computed directly from seed + (c+1) gamma) equals output c of the
    sequentially stepped generator, for 64 consecutive outputs of several seeds and for a far
    counter reached by stepping, and the stream of seed 0 starts with the published outputs of the
    reference generator (tests/golden/splitmix64_seed0.txt)."""
    for seed in (0, 1, 2000, 0x1234_5678_9ABC_DEF0, (1 << 64) - 1):
        seq = _splitmix64_stream(seed, 64)
        assert [oracle.splitmix64(seed, c) for c in range(64)] == seq, seed
    seq = _splitmix64_stream(2001, 5000)
    assert oracle.splitmix64(2001, 4999) == seq[4999]
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        known = [int(tok, 16) for line in f if not line.startswith("#") for tok in line.split()]
    assert len(known) == 4
    assert [oracle.splitmix64(0, c) for c in range(4)] == known
    # bits 0 and 1 (the two signs of a complex Z2 entry) are balanced over a long counter range
    b = np.array([oracle.splitmix64(0x1234_5678_9ABC_DEF0, c) & 3 for c in range(4000)])
    cnt = np.bincount(b, minlength=4)
    assert np.all(np.abs(cnt - 1000) < 4 * np.sqrt(750))


def test_dilution_classes_exhaustive():
    dims = (4, 2, 6, 4)
    cs = coords_of(dims)
    V = len(cs)
    cub = (cs[:, 0] & 1) + 2 * (cs[:, 1] & 1) + 4 * (cs[:, 2] & 1)
    eo = cs.sum(axis=1) & 1
    for scheme in range(8):
        nd = oracle.dilution_count(scheme)
        for site in range(0, V, 7):
            for al in range(4):
                for a in range(3):
                    d = 0
                    if scheme & 1:
                        d = d * 12 + 3 * al + a
                    if scheme & 2:
                        d = d * 8 + cub[site]
                    if scheme & 4:
                        d = d * 2 + eo[site]
                    assert oracle.dilution_class(dims, scheme, site, al, a) == d < nd
    # the diluted pieces sum to the noise and are disjoint
    eta = oracle.z2_source(dims, 7, 3)
    for scheme in (1, 2, 3, 4):
        parts = [oracle.z2_source(dims, 7, 3, scheme, d) for d in range(oracle.dilution_count(scheme))]
        assert np.array_equal(np.sum(parts, axis=0), eta)
        assert np.all(np.sum([np.abs(p) > 0 for p in parts], axis=0) == 1)


def test_z2_trace_estimator_unbiased_with_closed_form_variance():
    dims = (2, 2, 2, 2)
    n = 192
    rng = np.random.default_rng(71)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    N = 4000
    est = np.empty(N, complex)
    for k in range(N):
        e = oracle.z2_source(dims, 99, k).reshape(-1)
        est[k] = np.vdot(e, A @ e)
    var_closed = np.sum(np.abs(A) ** 2) - np.sum(np.abs(np.diag(A)) ** 2)
    mean = est.mean()
    assert abs(mean - np.trace(A)) < 4 * np.sqrt(var_closed / N)
    var_emp = np.mean(np.abs(est - np.trace(A)) ** 2)
    assert abs(var_emp / var_closed - 1) < 4 * np.sqrt(2.0 / N) + 0.02
    # full (point) dilution is exact for every noise
    e = oracle.z2_source(dims, 99, 0).reshape(-1)
    full = sum(np.conj(e[i]) * A[i, i] * e[i] for i in range(n))
    assert abs(full - np.trace(A)) < 1e-10


def test_diluted_estimator_matches_exact_per_class_variance(dense_2x2x2x2):
    """Spin-colour dilution: every noise's estimate is unbiased and its error is the sum
    over off-diagonal pairs within a class only."""
    dims, U, kappa, M, Minv = dense_2x2x2x2
    est = oracle.loops_z2(U, dims, kappa, 5, [0], oracle.SCHEME_SPIN_COLOUR, [0, 15], tol=1e-13)[0]
    # same numbers from dense algebra with the same noise
    ref = np.zeros_like(est)
    for d in range(12):
        eta = oracle.z2_source(dims, 5, 0, oracle.SCHEME_SPIN_COLOUR, d)
        s = (Minv @ eta.reshape(-1)).reshape(eta.shape)
        for k, g in enumerate([0, 15]):
            G = oracle.gamma(g)
            w = np.einsum("ab,xbc->xac", G, s)
            per_site = np.sum(np.conj(eta) * w, axis=(1, 2))
            for t in range(2):
                ref[k, t] += per_site[8 * t:8 * t + 8].sum()
    assert np.max(np.abs(est - ref)) < 1e-12


# ------------------------------------------------------------ truncated solver method


def test_tsm_lp_solve_limits(dense_2x2x2x2):
    dims, U, kappa, M, Minv = dense_2x2x2x2
    b = synth.random_spinor(dims, 1, seed=81)[0]
    # enough iterations: the truncated solve is the exact solve
    x = oracle.solve_lp(U, b, dims, kappa, niter=200)
    assert np.max(np.abs(x.reshape(-1) - Minv @ b.reshape(-1))) < 1e-11
    # zero iterations: x_e = 0, x_o = b_o
    x0 = oracle.solve_lp(U, b, dims, kappa, niter=0)
    par = oracle.parity(dims)
    assert np.all(x0[par == 0] == 0) and np.array_equal(x0[par == 1], b[par == 1])
    # the CGNR residual of the Schur system decreases monotonically in the normal-equation norm
    prev = np.inf
    for n in (1, 3, 6, 12):
        xn = oracle.solve_lp(U, b, dims, kappa, niter=n)
        r = np.linalg.norm(M @ xn.reshape(-1) - b.reshape(-1))
        assert r < prev * 1.0000001
        prev = r


def test_tsm_unbiased_against_dense(dense_2x2x2x2):
    dims, U, kappa, M, Minv = dense_2x2x2x2
    gam = [0, 15, 5]
    exact = oracle.exact_loops_dense(Minv, dims, gam)
    n_lp, n_hp = 300, 60
    lp = oracle.loops_lp(U, dims, kappa, 123, range(n_lp), 0, gam, niter=2)
    hp_noises = range(n_lp, n_lp + n_hp)
    hp_hp = oracle.loops_z2(U, dims, kappa, 123, hp_noises, 0, gam, tol=1e-13)
    hp_lp = oracle.loops_lp(U, dims, kappa, 123, hp_noises, 0, gam, niter=2)
    est = oracle.tsm_combine(lp, hp_hp, hp_lp)
    err = np.sqrt(np.var(lp, axis=0) / n_lp + np.var(hp_hp - hp_lp, axis=0) / n_hp)
    z = np.abs(est - exact) / np.maximum(err, 1e-300)
    assert np.all(z < 4.5), z.max()
    # if the low-precision map were exact, the correction would vanish identically
    corr = oracle.loops_z2(U, dims, kappa, 123, range(3), 0, gam) - oracle.loops_lp(
        U, dims, kappa, 123, range(3), 0, gam, niter=300)
    assert np.max(np.abs(corr)) < 1e-10


# ------------------------------------------------------------ derivatives


def test_dkappa_against_finite_difference_and_dense(dense_2x2x2x2):
    dims, U, kappa, M, Minv = dense_2x2x2x2
    gam = [0, 15, 5, 1]
    h = 1e-5
    d = oracle.loops_dkappa(U, dims, kappa, 9, [0, 1], 1, gam, tol=1e-13)
    lp = oracle.loops_z2(U, dims, kappa + h, 9, [0, 1], 1, gam, tol=1e-13)
    lm = oracle.loops_z2(U, dims, kappa - h, 9, [0, 1], 1, gam, tol=1e-13)
    fd = (lp - lm) / (2 * h)
    assert np.max(np.abs(fd - d)) < 1e-6 * max(1.0, np.max(np.abs(d)))
    # exact Tr[Gamma M^-1 D M^-1] at one site through the dense matrices
    D = (np.eye(M.shape[0]) - M) / kappa
    dense = Minv @ D @ Minv
    # identity M^-1 D M^-1 = (M^-2 - M^-1) / kappa
    assert np.max(np.abs(dense - (Minv @ Minv - Minv) / kappa)) < 1e-10
    ex = oracle.exact_loops_dense(dense, dims, gam)
    # point-source derivative at every site of timeslice 0 sums to the timeslice value
    tot = np.zeros(len(gam), complex)
    for site in range(8):
        for al in range(4):
            for a in range(3):
                e = oracle.point_source(dims, site, al, a)
                s, _, _ = oracle.solve(U, e, dims, kappa, 1e-13)
                u, _, _ = oracle.solve(U, oracle.dhop(U, s, dims), dims, kappa, 1e-13)
                tot += oracle.loops_accumulate(dims, e, u, gam)[:, 0]
    assert np.max(np.abs(tot - ex[:, 0])) < 1e-10


def test_link_gradient_directional_difference():
    dims = (2, 2, 2, 4)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.5, seed=91)
    kappa = 0.12
    gam = [15, 0]
    rng = np.random.default_rng(92)
    W = rng.standard_normal((2, dims[3])) + 1j * rng.standard_normal((2, dims[3]))
    srcs = [oracle.z2_source(dims, 93, 0, 1, d) for d in range(12)]

    def F(Ux):
        tot = 0.0
        for eta in srcs:
            s, _, _ = oracle.solve(Ux, eta, dims, kappa, 1e-13)
            L = oracle.loops_accumulate(dims, eta, s, gam)
            tot += np.sum((np.conj(W) * L).real)
        return tot

    g = oracle.link_grad(U, dims, kappa, srcs, gam, W, tol=1e-13)
    for trial in range(2):
        dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        h = 1e-5
        fd = (F(U + h * dU) - F(U - h * dU)) / (2 * h)
        an = np.sum((np.conj(g) * dU).real)
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (fd, an)
    assert g.shape == (4, V, 3, 3)


# ------------------------------------------------------------ disconnected correlator (Eq. 2)

def test_correlator_identical_estimates_against_fft():
    """All noises give the same loops b, a: the estimate is -1/(L^3 T) sum_t b(t) a(t+dt),
    here from the convolution theorem: sum_t b(t) a(t+dt) = ifft(fft(a) conj(fft(conj b)))."""
    rng = np.random.default_rng(71)
    T, L3 = 7, 27
    b = rng.normal(size=T) + 1j * rng.normal(size=T)
    a = rng.normal(size=T) + 1j * rng.normal(size=T)
    got = oracle.disconnected_correlator(np.tile(b, (3, 1)), np.tile(a, (3, 1)), L3)
    ref = -np.fft.ifft(np.fft.fft(a) * np.conj(np.fft.fft(np.conj(b)))) / (L3 * T)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def test_correlator_unbiased_over_distinct_noise_pairs():
    """Per-noise loops L_A^n = mu_A + xi_n and L_B^n = mu_B + c xi_n share their fluctuation xi_n
    (real Gaussian of variance s2 = 0.49, so E[xi(t) xi(t)] != 0), as two loops from the same source
    do.  The estimate over n != m has expectation -1/(L^3 T) sum_t mu_B(t) mu_A(t+dt).  Including
    n == m (all N^2 ordered pairs) adds c E[Xi(t) Xi(t+dt)] with Xi = sum_n xi_n, i.e. c N s2 delta_{dt,0}
    per timeslice, so its expectation is off by the closed form -c s2 / (N L^3) at dt = 0 and exact
    elsewhere.  Both expectations are z-tested, and the sample is large enough that the closed-form
    bias is ten standard errors of the same-noise mean away from zero (the contrast that tells the
    two estimators apart)."""
    rng = np.random.default_rng(72)
    T, L3, N, reps, s2 = 4, 8, 5, 4000, 0.49
    mu_a = rng.normal(size=T) + 1j * rng.normal(size=T)
    mu_b = rng.normal(size=T) + 1j * rng.normal(size=T)
    c = 0.8 + 0.3j
    est, biased = [], []
    for _ in range(reps):
        xi = rng.normal(size=(N, T)) * np.sqrt(s2)
        la, lb = mu_a + xi, mu_b + c * xi
        est.append(oracle.disconnected_correlator(lb, la, L3))
        # all ordered pairs including n == m, written with numpy for the contrast
        sa, sb = la.sum(axis=0), lb.sum(axis=0)
        biased.append(np.array([-np.sum(sb * np.roll(sa, -dt)) / N ** 2 / (L3 * T) for dt in range(T)]))
    est, biased = np.array(est), np.array(biased)
    ref = np.array([-np.sum(mu_b * np.roll(mu_a, -dt)) / (L3 * T) for dt in range(T)])
    bias = np.zeros(T, dtype=np.complex128)
    bias[0] = -c * s2 / (N * L3)

    def z(sample, expect):
        se_re = sample.real.std(axis=0, ddof=1) / np.sqrt(reps)
        se_im = sample.imag.std(axis=0, ddof=1) / np.sqrt(reps)
        d = sample.mean(axis=0) - expect
        return np.concatenate([np.abs(d.real) / se_re, np.abs(d.imag) / se_im])

    assert np.all(z(est, ref) < 4.5), z(est, ref)
    assert np.all(z(biased, ref + bias) < 4.5), z(biased, ref + bias)
    se0 = np.abs(biased.std(axis=0, ddof=1)[0]) / np.sqrt(reps)
    assert abs(bias[0]) / se0 > 10, abs(bias[0]) / se0
    # and the measured offset of the same-noise estimator shows it too
    zb = np.abs(biased.mean(axis=0)[0] - ref[0]) / se0
    assert zb > 10, zb


def test_correlator_swap_symmetry():
    rng = np.random.default_rng(73)
    N, T, L3 = 4, 6, 64
    lb = rng.normal(size=(N, T)) + 1j * rng.normal(size=(N, T))
    la = rng.normal(size=(N, T)) + 1j * rng.normal(size=(N, T))
    dba = oracle.disconnected_correlator(lb, la, L3)
    dab = oracle.disconnected_correlator(la, lb, L3)
    for dt in range(T):
        assert abs(dba[dt] - dab[(T - dt) % T]) < 1e-14 * np.max(np.abs(dba))


VALID_SCHEMES = [s for s in range(128) if oracle.dilution_valid(s)]


def test_dilution_scheme_validity():
    """Spin-colour excludes the separate spin / spin-parity / colour factors; spin and spin parity
    exclude each other; everything else combines."""
    for s in range(128):
        bad = bool(s & 1 and s & (8 | 16 | 32)) or bool(s & 16 and s & 32)
        assert oracle.dilution_valid(s) == (not bad), s
    assert not oracle.dilution_valid(128) and not oracle.dilution_valid(-1)
    assert len(VALID_SCHEMES) == 2 * 2 * 2 * (1 + 2 * 3)  # time x cubic x site-parity x spin/colour options


@pytest.mark.parametrize("scheme", [s for s in VALID_SCHEMES if s & (8 | 16 | 32 | 64)])
def test_new_dilution_pieces_partition_and_support(scheme):
    dims = (4, 2, 2, 6)
    X, Y, Z, T = dims
    cs = coords_of(dims)
    noise = 11
    eta = oracle.z2_source(dims, 31, noise)  # whole noise vector, no masks at all
    if scheme & 64:
        eta = eta * (cs[:, 3] == noise % T)[:, None, None]
    nd = oracle.dilution_count(scheme)
    parts = [oracle.z2_source(dims, 31, noise, scheme, d if nd > 1 else -1) for d in range(nd)]
    assert np.array_equal(np.sum(parts, axis=0), eta)
    assert np.all(np.sum([np.abs(p) > 0 for p in parts], axis=0) == (np.abs(eta) > 0))
    # digits of d, slowest first, in the order spin-colour | spin | spin parity | colour | cubic | parity
    radices = []
    if scheme & 1:
        radices.append(("sc", 12))
    if scheme & 16:
        radices.append(("spin", 4))
    if scheme & 32:
        radices.append(("spar", 2))
    if scheme & 8:
        radices.append(("col", 3))
    if scheme & 2:
        radices.append(("cub", 8))
    if scheme & 4:
        radices.append(("eo", 2))
    spin = np.arange(4)[None, :, None]
    col = np.arange(3)[None, None, :]
    cub = ((cs[:, 0] & 1) + 2 * (cs[:, 1] & 1) + 4 * (cs[:, 2] & 1))[:, None, None]
    eo = (cs.sum(axis=1) & 1)[:, None, None]
    for d in range(nd):
        rem, digit = d, {}
        for name, r in reversed(radices):
            digit[name] = rem % r
            rem //= r
        allowed = np.ones((len(cs), 4, 3), bool)
        if "sc" in digit:
            allowed &= (3 * spin + col) == digit["sc"]
        if "spin" in digit:
            allowed &= spin == digit["spin"]
        if "spar" in digit:
            allowed &= (spin % 2) == digit["spar"]
        if "col" in digit:
            allowed &= col == digit["col"]
        if "cub" in digit:
            allowed &= cub == digit["cub"]
        if "eo" in digit:
            allowed &= eo == digit["eo"]
        assert np.array_equal(parts[d], np.where(allowed, eta, 0)), (scheme, d)


def test_spin_and_colour_equal_spin_colour():
    dims = (2, 2, 2, 4)
    for d in range(12):
        assert np.array_equal(oracle.z2_source(dims, 5, 2, 16 | 8, d), oracle.z2_source(dims, 5, 2, 1, d))


@pytest.mark.parametrize("scheme", [32, 8, 32 | 8, 64, 64 | 16, 4 | 32])
def test_new_dilution_estimators_unbiased_with_closed_form_variance(scheme):
    """eta^+ A eta summed over the classes of one noise: mean Tr[A restricted to the support],
    variance sum over same-class off-diagonal pairs |A_ij|^2 (complex Z2 entries: E[e_i* e_j] =
    delta_ij, E|e_i|^2 |e_j|^2 = 1, E[e_i*^2 e_j^2] = 0).  For time dilution the support of noise n
    is the timeslice n mod T, so the estimate is of the trace over that timeslice."""
    dims = (2, 2, 2, 2)
    n = 192
    rng = np.random.default_rng(80 + scheme)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    nd = oracle.dilution_count(scheme)
    cls = np.array([oracle.dilution_class(dims, scheme, i // 12, (i // 3) % 4, i % 3) for i in range(n)])
    tsl = coords_of(dims)[np.arange(n) // 12, 3]
    N = 2400
    for parity_t in ([0, 1] if scheme & 64 else [None]):
        noises = [k for k in range(N) if parity_t is None or k % 2 == parity_t]
        sup = np.ones(n, bool) if parity_t is None else (tsl == parity_t)
        est = []
        for k in noises:
            tot = 0j
            for d in range(nd):
                e = oracle.z2_source(dims, 77, k, scheme, d if nd > 1 else -1).reshape(-1)
                tot += np.vdot(e, A @ e)
            est.append(tot)
        est = np.array(est)
        same = (cls[:, None] == cls[None, :]) & sup[:, None] & sup[None, :]
        np.fill_diagonal(same, False)
        var_closed = np.sum(np.abs(A[same]) ** 2)
        exact = np.sum(np.diag(A)[sup])
        assert abs(est.mean() - exact) < 4.5 * np.sqrt(var_closed / len(est)), (scheme, parity_t)
        var_emp = np.mean(np.abs(est - exact) ** 2)
        assert abs(var_emp / var_closed - 1) < 5 * np.sqrt(2.0 / len(est)) + 0.03, (scheme, var_emp / var_closed)


# ------------------------------------------------------------ smearing (Section 2)

def test_smearing_free_field_plane_waves():
    dims = (4, 6, 4, 3)
    U = synth.unit_field(dims)
    cs = coords_of(dims)
    rng = np.random.default_rng(90)
    alpha, iters = 0.7, 3
    for n in [(0, 0, 0), (1, 2, 3), (2, 5, 1)]:
        p = 2 * np.pi * np.array(n) / np.array(dims[:3])
        chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        f_t = rng.normal(size=dims[3]) + 1j * rng.normal(size=dims[3])  # any time dependence
        psi = (np.exp(1j * cs[:, :3] @ p) * f_t[cs[:, 3]])[:, None, None] * chi[None]
        lam = ((1 + 2 * alpha * np.cos(p).sum()) / (1 + 6 * alpha)) ** iters
        got = oracle.smear(U, psi, dims, alpha, iters)
        assert np.max(np.abs(got - lam * psi)) < 1e-13 * np.max(np.abs(psi)), n


def test_smearing_gauge_covariant_hermitian_local():
    dims = (4, 2, 4, 6)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.7, seed=91)
    Om = synth.random_su3(V, seed=92)
    cs = coords_of(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        c2 = cs.copy()
        c2[:, mu] = (c2[:, mu] + 1) % dims[mu]
        nb = site_of(dims, c2.T)
        Up[mu] = Om @ U[mu] @ np.conj(np.transpose(Om[nb], (0, 2, 1)))
    phi, psi = synth.random_spinor(dims, 2, seed=93)
    a, n = 0.45, 4
    lhs = oracle.smear(Up, np.einsum("xab,xsb->xsa", Om, psi), dims, a, n)
    rhs = np.einsum("xab,xsb->xsa", Om, oracle.smear(U, psi, dims, a, n))
    assert np.max(np.abs(lhs - rhs)) < 1e-13
    assert abs(np.vdot(phi, oracle.smear(U, psi, dims, a, n)) - np.vdot(oracle.smear(U, phi, dims, a, n), psi)) \
        < 1e-12 * np.linalg.norm(phi) * np.linalg.norm(psi)
    # a point source on spin 1 at one site of timeslice 2 spreads over that timeslice and spin only
    one = np.zeros_like(psi)
    site = site_of(dims, np.array([1, 0, 2, 2]))
    one[site, 1, 0] = 1.0
    sm = oracle.smear(U, one, dims, a, n)
    sel = cs[:, 3] == 2
    assert np.all(sm[~sel] == 0) and np.all(sm[:, [0, 2, 3], :] == 0)
    assert np.count_nonzero(np.abs(sm[sel, 1, 0]) > 0) > 8


def dense_smearing(U, dims, alpha, iters):
    n = int(np.prod(dims)) * 12
    S = np.zeros((n, n), complex)
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1
        S[:, k] = oracle.smear(U, e.reshape(-1, 4, 3), dims, alpha, iters).reshape(-1)
    return S


def test_smeared_loops_against_dense(dense_2x2x2x2):
    dims, U, kappa, M, Minv = dense_2x2x2x2
    alpha, iters = 0.6, 2
    S = dense_smearing(U, dims, alpha, iters)
    assert np.max(np.abs(S - S.conj().T)) < 1e-14
    gam = [0, 15, 5]
    got = oracle.loops_z2_smeared(U, dims, kappa, 17, [3], 0, gam, alpha, iters, tol=1e-13)[0]
    eta = oracle.z2_source(dims, 17, 3).reshape(-1)
    xi = S @ eta
    s = Minv @ xi
    for k, g in enumerate(gam):
        G = np.kron(np.eye(16), np.kron(oracle.gamma(g), np.eye(3)))
        per_site = (np.conj(xi) * (G @ s)).reshape(16, 12).sum(axis=1)
        ref = per_site.reshape(2, 8).sum(axis=1)
        assert np.max(np.abs(got[k] - ref)) < 1e-11 * np.max(np.abs(ref)), g
    # the estimator's mean is the trace of the smeared propagator per timeslice
    B = S @ Minv @ S
    G5 = np.kron(np.eye(16), np.kron(oracle.gamma(15), np.eye(3)))
    A = G5 @ B
    tsl = np.repeat(np.arange(16) // 8, 12)
    N = 3000
    est = np.zeros((N, 2), complex)
    for i in range(N):
        e = oracle.z2_source(dims, 18, i).reshape(-1)
        x = S @ e
        v = np.conj(x) * (G5 @ (Minv @ x))
        est[i] = [v[tsl == 0].sum(), v[tsl == 1].sum()]
    exact = [np.trace(A[np.ix_(tsl == t, tsl == t)]) for t in (0, 1)]
    for t in (0, 1):
        se = np.std(est[:, t]) / np.sqrt(N)
        assert abs(est[:, t].mean() - exact[t]) < 4.5 * se, t



# ------------------------------------------------------------ eta' ratio fit (Eqs. 3-4)


def _ratio_model(T, m_pi, A, B, m):
    t = np.arange(T)
    gp = np.exp(-m_pi * t) + np.exp(-m_pi * (T - t))
    gm = np.exp(-m * t) + np.exp(-m * (T - t))
    return gp, A - B * gm / gp


def test_eta_prime_fit_recovers_noise_free_parameters():
    T, m_pi = 32, 0.6
    for A, B, m in [(0.8, 0.5, 0.45), (-0.2, 1.3, 0.9), (0.05, 0.02, 0.3)]:
        gp, r = _ratio_model(T, m_pi, A, B, m)
        C = 2.5 * gp
        D = C * r
        c_eta, p, err, chi2 = oracle.eta_prime_fit(D, C, m_pi, 2, 11)
        assert np.allclose(p, [A, B, m], rtol=1e-8, atol=1e-10), (p, A, B, m)
        assert chi2 < 1e-20 and np.all(err == 0)
        assert np.allclose(c_eta, C - 2 * D, rtol=1e-15, atol=0)
        # a model with the other sign of B, or without the backward term e^{-m (T-t)}, cannot fit these data
        t = np.arange(2, 12)
        wrong = [A + B * (np.exp(-m * t) + np.exp(-m * (T - t))) / gp[2:12],
                 A - B * np.exp(-m * t) / gp[2:12]]
        for wr in wrong:
            assert np.max(np.abs(wr - r[2:12])) > 1e-6


def test_eta_prime_fit_scaled_configurations_have_no_spread():
    T, m_pi = 24, 0.7
    gp, r = _ratio_model(T, m_pi, 0.6, 0.4, 0.5)
    lam = np.array([0.7, 1.0, 1.3, 2.1])[:, None]
    C = lam * gp[None]
    D = C * r[None]
    c_eta, p, err, chi2 = oracle.eta_prime_fit(D, C, m_pi, 1, 10)
    assert np.allclose(p, [0.6, 0.4, 0.5], rtol=1e-8)
    assert np.all(np.abs(err) < 1e-9)
    assert np.allclose(c_eta, (C - 2 * D).mean(axis=0), rtol=1e-14)


def test_eta_prime_fit_jackknife_of_a_shift_in_A():
    """Per-configuration ratios A_n - B g: every jackknife sample has the same B and m, and A_k is the
    leave-one-out mean, so the jackknife error of A is the standard error of the mean of the A_n."""
    T, m_pi, B, m = 32, 0.6, 0.5, 0.45
    rng = np.random.default_rng(71)
    An = 0.8 + 0.05 * rng.standard_normal(9)
    gp, _ = _ratio_model(T, m_pi, 0.0, B, m)
    t = np.arange(T)
    g = (np.exp(-m * t) + np.exp(-m * (T - t))) / gp
    C = np.tile(3.0 * gp, (len(An), 1))
    D = C * (An[:, None] - B * g[None])
    _, p, err, _ = oracle.eta_prime_fit(D, C, m_pi, 2, 12)
    sem = np.sqrt(np.sum((An - An.mean()) ** 2) / (len(An) * (len(An) - 1)))
    assert np.allclose(p, [An.mean(), B, m], rtol=1e-7)
    assert abs(err[0] - sem) < 1e-7 * sem and err[1] < 1e-8 and err[2] < 1e-8, (err, sem)
