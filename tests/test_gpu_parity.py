"""Parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Inputs come from :mod:`synth` (gauge fields, spinors) and the noise generator
each side implements; nothing the GPU produces feeds the oracle.

Tolerances:
* integer work (noise entries, dilution masks, point sources): bit-exact;
* FP64 operator applications: max |gpu - oracle| <= 1e-13 max |oracle| (a few
  ulps of the 1320-flop site sum, different summation order);
* reduced-precision operators: FP32 2e-6, FP16 (per-site scaled spinors,
  unscaled links) 4e-3, BF16 3e-2, all relative to max |oracle| -- from the
  storage rounding 2^-24 / 2^-11 / 2^-8 of inputs and links, amplified by the
  9-term colour sums;
* FP64 solves and loops: the loop error is normalised by the Cauchy-Schwarz
  bound sum_d sum_{x in t} |eta_d(x)| |s_d(x)| and must stay below 1e-10, with
  the GPU solving to 1e-12 and the oracle to 1e-13.
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


SHAPES = [(4, 4, 4, 4), (2, 2, 2, 2), (4, 4, 6, 8), (8, 6, 4, 10)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("tap", [1, 0])
def test_operators_fp64(dl, dev, dims, tap):
    U = synth.gauge_field(dims, 0.6, seed=101)
    lat = dl.Lattice(dims, tap)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64,), recon=12)
    G18 = dl.Gauge(lat, U, precs=(dl.DL_F64,), recon=18)
    psi = synth.random_spinor(dims, 3, seed=102)
    k = 0.137
    par = oracle.parity(dims)
    x = to_dev(psi, dev)
    for op in (dl.DL_OP_DHOP, dl.DL_OP_DHOPDAG, dl.DL_OP_M, dl.DL_OP_MDAG, dl.DL_OP_MHAT, dl.DL_OP_MHATDAG):
        for gauge in (G, G18):
            out = from_dev(dl.apply(gauge, k, op, x))
            for r in range(3):
                if op in (dl.DL_OP_DHOP, dl.DL_OP_DHOPDAG):
                    ref = oracle.dhop(U, psi[r], dims, tap, dag=op == dl.DL_OP_DHOPDAG)
                elif op in (dl.DL_OP_M, dl.DL_OP_MDAG):
                    ref = oracle.apply_m(U, psi[r], dims, k, tap, dag=op == dl.DL_OP_MDAG)
                else:
                    pe = psi[r].copy()
                    pe[par == 1] = 0
                    ref = oracle.apply_mhat(U, pe, dims, k, tap, dag=op == dl.DL_OP_MHATDAG)
                    ref[par == 1] = 0
                err = np.max(np.abs(out[r] - ref))
                assert err <= 1e-13 * np.max(np.abs(ref)), (op, r, err)


@pytest.mark.parametrize("prec,tol", [(1, 2e-6), (2, 4e-3), (3, 3e-2)])
def test_operators_reduced_precision(dl, dev, prec, tol):
    dims = (4, 4, 6, 8)
    U = synth.gauge_field(dims, 0.6, seed=111)
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64, prec), recon=12)
    psi = synth.random_spinor(dims, 2, seed=112)
    x = to_dev(psi, dev)
    for op in (dl.DL_OP_DHOP, dl.DL_OP_M, dl.DL_OP_MDAG):
        out = from_dev(dl.apply(G, 0.13, op, x, prec=prec))
        for r in range(2):
            if op == dl.DL_OP_DHOP:
                ref = oracle.dhop(U, psi[r], dims)
            else:
                ref = oracle.apply_m(U, psi[r], dims, 0.13, dag=op == dl.DL_OP_MDAG)
            err = np.max(np.abs(out[r] - ref)) / np.max(np.abs(ref))
            assert err <= tol, (op, err)


def test_sources_bit_exact(dl, dev):
    """Noise entries, dilution masks and point sources equal the oracle's exactly."""
    for dims, scheme in [((4, 4, 4, 4), 0), ((4, 4, 4, 4), 1), ((4, 2, 6, 4), 3), ((6, 4, 2, 4), 7),
                         ((4, 4, 4, 4), 4)]:
        lat = dl.Lattice(dims, 1)
        V = lat.V
        src = dl.z2_sources(2000 + scheme, 3, first_noise=5, scheme=scheme)
        n = dl.dl_sources_count(lat.h, src)
        out = torch.empty((n, V, 4, 3), dtype=torch.complex128, device=dev)
        dl.dl_sources_fill(lat.h, src, 0, n, out)
        got = from_dev(out)
        ncls = oracle.dilution_count(scheme)
        for r in range(n):
            ref = oracle.z2_source(dims, 2000 + scheme, 5 + r // ncls, scheme, (r % ncls) if scheme else -1)
            assert np.array_equal(got[r], ref), (dims, scheme, r)
    lat = dl.Lattice((4, 4, 4, 4), 1)
    out = torch.empty((12, 256, 4, 3), dtype=torch.complex128, device=dev)
    dl.dl_sources_fill(lat.h, dl.point_sources(77), 0, 12, out)
    got = from_dev(out)
    for r in range(12):
        assert np.array_equal(got[r], oracle.point_source((4, 4, 4, 4), 77, r // 3, r % 3))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 4, 6, 8), (2, 2, 2, 2)])
def test_solve_fp64(dl, dev, dims):
    U = synth.gauge_field(dims, 0.5, seed=121)
    kappa = 0.12
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    b = synth.random_spinor(dims, 3, seed=122)
    x, st = dl.solve(G, kappa, to_dev(b, dev), dl.solve_params(tol=1e-12, maxiter=500))
    x = from_dev(x)
    for r in range(3):
        status, iters, upd, res = st[r]
        assert status == dl.DL_OK and res <= 1e-12, st[r]
        # the residual measured by the oracle's operator
        rr = np.linalg.norm(b[r] - oracle.apply_m(U, x[r], dims, kappa)) / np.linalg.norm(b[r])
        assert rr <= 1.5e-12
        xo, _, _ = oracle.solve(U, b[r], dims, kappa, tol=1e-13)
        assert np.linalg.norm(x[r] - xo) / np.linalg.norm(xo) < 1e-10


def cs_norm(dims, etas, sols):
    """sum over sources of sum_{x in t} |eta(x)| |s(x)| per timeslice."""
    T = dims[3]
    per_t = int(np.prod(dims[:3]))
    out = np.zeros(T)
    for e, s in zip(etas, sols):
        v = np.linalg.norm(e.reshape(-1, 12), axis=1) * np.linalg.norm(s.reshape(-1, 12), axis=1)
        out += v.reshape(T, per_t).sum(axis=1)
    return out


def test_loops_point_sources_all_gammas(dl, dev):
    """The exact loop at one site from its 12 unit sources (4^3 x 4, eps 0.5, kappa 0.12)."""
    w = synth.WORKLOADS["plain_4x4x4x4"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    gam = list(range(16))
    for site in (0, 201):
        L, st = dl.loops(G, kappa, dl.point_sources(site), gam, dl.solve_params(tol=1e-12, maxiter=500))
        ref = oracle.loops_point(U, dims, kappa, site, gam, tol=1e-13)
        assert all(s[0] == dl.DL_OK for s in st)
        etas = [oracle.point_source(dims, site, a, c) for a in range(4) for c in range(3)]
        sols = [oracle.solve(U, e, dims, kappa, 1e-13)[0] for e in etas]
        norm = cs_norm(dims, etas, sols)
        err = np.abs(L[0] - ref) / np.maximum(norm, 1e-300)[None, :]
        assert np.max(err) < 1e-10, np.max(err)


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_loops_z2_fp64(dl, dev, scheme):
    dims = (4, 4, 4, 8)
    U = synth.gauge_field(dims, 0.5, seed=131)
    kappa = 0.125
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    gam = [0, 15, 5, 1, 7]
    n_noise = 2
    L, st = dl.loops(G, kappa, dl.z2_sources(2000, n_noise, first_noise=3, scheme=scheme), gam,
                     dl.solve_params(tol=1e-12, maxiter=500))
    ref, sols = oracle.loops_z2(U, dims, kappa, 2000, range(3, 3 + n_noise), scheme, gam, tol=1e-13,
                                return_solutions=True)
    ncls = oracle.dilution_count(scheme)
    for n in range(n_noise):
        etas = [oracle.z2_source(dims, 2000, 3 + n, scheme, d if scheme else -1) for d in range(ncls)]
        norm = cs_norm(dims, etas, sols[n * ncls:(n + 1) * ncls])
        err = np.abs(L[n] - ref[n]) / norm[None, :]
        assert np.max(err) < 1e-10, (n, np.max(err))
    assert all(s[0] == dl.DL_OK and s[3] <= 1e-12 for s in st)


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-5), (2, 3e-2), (3, 1.5e-1)])
def test_truncated_cgnr_against_oracle(dl, dev, prec, tol):
    """The truncated low-precision solve (25 CGNR iterations) against the same algorithm in FP64.
    The FP64 run must agree to rounding; reduced precision is reported against the stated bound."""
    dims = (4, 4, 4, 8)
    U = synth.gauge_field(dims, 0.5, seed=141)
    kappa = 0.125
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64, prec))
    b = synth.random_spinor(dims, 2, seed=142)
    x, st = dl.solve(G, kappa, to_dev(b, dev), dl.solve_params(solver=dl.DL_CGNR, prec=prec, fixed_iters=25))
    x = from_dev(x)
    for r in range(2):
        ref = oracle.solve_lp(U, b[r], dims, kappa, niter=25)
        err = np.linalg.norm(x[r] - ref) / np.linalg.norm(ref)
        assert err < tol, (prec, err)
        assert st[r][1] == 25


def test_mixed_precision_bicgstab_reaches_fp64_tolerance(dl, dev):
    dims = (4, 4, 6, 8)
    U = synth.gauge_field(dims, 0.5, seed=151)
    kappa = 0.12
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64, dl.DL_F32, dl.DL_F16))
    b = synth.random_spinor(dims, 2, seed=152)
    for prec in (dl.DL_F32, dl.DL_F16):
        x, st = dl.solve(G, kappa, to_dev(b, dev), dl.solve_params(prec=prec, tol=1e-10, maxiter=2000))
        x = from_dev(x)
        for r in range(2):
            assert st[r][0] == dl.DL_OK and st[r][3] <= 1e-10, (prec, st[r])
            assert st[r][2] >= 2  # reliable updates happened
            rr = np.linalg.norm(b[r] - oracle.apply_m(U, x[r], dims, kappa)) / np.linalg.norm(b[r])
            assert rr <= 1.2e-10


def test_full_size_operator_and_solve(dl, dev):
    """16^3 x 32, eps 0.35, kappa 0.150: one application of M against the oracle (every entry),
    and one FP64 solve whose residual is measured with the oracle's operator."""
    w = synth.WORKLOADS["plain_16x16x16x32"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    psi = synth.random_spinor(dims, 1, seed=161)
    out = from_dev(dl.apply(G, kappa, dl.DL_OP_M, to_dev(psi, dev)))
    ref = oracle.apply_m(U, psi[0], dims, kappa)
    assert np.max(np.abs(out[0] - ref)) <= 1e-13 * np.max(np.abs(ref))
    x, st = dl.solve(G, kappa, to_dev(psi, dev), dl.solve_params(tol=1e-10, maxiter=1000))
    x = from_dev(x)
    rr = np.linalg.norm(psi[0] - oracle.apply_m(U, x[0], dims, kappa)) / np.linalg.norm(psi[0])
    assert st[0][0] == dl.DL_OK and rr <= 1.1e-10, (st, rr)


def test_full_size_loops_batch_properties(dl, dev):
    """The timed workload's shape (16^3 x 32, spin-colour dilution) on 4 noises: every solve
    converges, the batch result equals single-noise runs, and the time sums of L_1 and L_gamma5
    are real per noise.  (For a source supported on one spin, gamma5 eta = +-eta, so
    conj(eta^+ Gamma M^-1 eta) = eta^+ gamma5 Gamma^+ gamma5 M^-1 eta by gamma5-hermiticity, which
    is the same number for Gamma = 1 and gamma5; the timeslice projector breaks this per t.)"""
    w = synth.WORKLOADS["plain_16x16x16x32"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U)
    prm = dl.solve_params(tol=1e-10, maxiter=1000)
    L, st = dl.loops(G, kappa, dl.z2_sources(w["noise_seed"], 4, scheme=dl.DL_DIL_SPIN_COLOUR), [0, 15], prm)
    assert len(st) == 48 and all(s[0] == dl.DL_OK and s[3] <= 1e-10 for s in st)
    L1, _ = dl.loops(G, kappa, dl.z2_sources(w["noise_seed"], 1, first_noise=2, scheme=dl.DL_DIL_SPIN_COLOUR),
                     [0, 15], prm)
    assert np.max(np.abs(L1[0] - L[2])) <= 1e-12 * np.max(np.abs(L[2]))
    tot = L.sum(axis=2)
    assert np.max(np.abs(tot.imag)) < 1e-8 * np.max(np.abs(tot.real))
    assert np.max(np.abs(L.imag)) > 1e-3  # per timeslice the imaginary parts do not vanish


def test_kappa_zero_solves_in_one_step(dl, dev):
    """kappa = 0 (M = 1): BiCGStab reaches x = b exactly in its first half step, where s = 0 makes
    t = 0 and omega = 0; the recursion must stop there and report the solve as converged (FP64 in
    one iteration; FP32 with FP64 reliable updates in a few, since its iterate holds b only to FP32
    rounding and the FP64 true residual restarts it), as the oracle's BiCGStab does, and the loops
    must equal the oracle's (Tr Gamma eta eta^+ summed per timeslice); the truncated CGNR gives
    x = b too."""
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.5, seed=393)
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64, dl.DL_F32))
    b = synth.random_spinor(dims, 3, seed=394)
    for prm in (dl.solve_params(tol=1e-12, maxiter=50), dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=50)):
        x, st = dl.solve(G, 0.0, to_dev(b, dev), prm)
        x = from_dev(x)
        for r in range(3):
            assert st[r][0] == dl.DL_OK and st[r][1] <= (1 if prm.prec == dl.DL_F64 else 3), (prm.prec, r, st[r])
            assert np.linalg.norm(x[r] - b[r]) <= 1e-6 * np.linalg.norm(b[r]), (prm.prec, r)
    x, st = dl.solve(G, 0.0, to_dev(b, dev), dl.solve_params(solver=dl.DL_CGNR, prec=dl.DL_F64, fixed_iters=25))
    x = from_dev(x)
    assert all(s[0] == dl.DL_OK for s in st)
    assert np.max(np.abs(x - b)) <= 1e-14 * np.max(np.abs(b))
    gam = [0, 15]
    L, st = dl.loops(G, 0.0, dl.z2_sources(395, 2, scheme=dl.DL_DIL_SPIN_COLOUR), gam,
                     dl.solve_params(tol=1e-12, maxiter=50))
    assert all(s[0] == dl.DL_OK for s in st), st
    ref = oracle.loops_z2(U, dims, 0.0, 395, range(2), oracle.SCHEME_SPIN_COLOUR, gam, tol=1e-13)
    assert np.max(np.abs(L - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_zero_and_empty_right_hand_sides(dl, dev):
    """Degenerate inputs: a zero right-hand side among others solves to x = 0 in no iterations with
    status OK (BiCGStab in FP64 and in FP32 with FP64 reliable updates, and the truncated CGNR),
    while its neighbours in the batch still meet the oracle's operator residual; an empty batch is
    refused with an error."""
    dims = (4, 4, 6, 8)
    U = synth.gauge_field(dims, 0.5, seed=391)
    kappa = 0.12
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64, dl.DL_F32, dl.DL_F16))
    b = synth.random_spinor(dims, 3, seed=392)
    b[1] = 0
    for prm in (dl.solve_params(tol=1e-12, maxiter=500), dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=1000)):
        x, st = dl.solve(G, kappa, to_dev(b, dev), prm)
        x = from_dev(x)
        assert st[1][0] == dl.DL_OK and st[1][1] == 0 and st[1][3] == 0.0, st[1]
        assert np.all(x[1] == 0)
        for r in (0, 2):
            assert st[r][0] == dl.DL_OK, st[r]
            rr = np.linalg.norm(b[r] - oracle.apply_m(U, x[r], dims, kappa)) / np.linalg.norm(b[r])
            assert rr <= 1.5 * prm.tol, (r, rr)
    x, st = dl.solve(G, kappa, to_dev(b, dev), dl.solve_params(solver=dl.DL_CGNR, prec=dl.DL_F16, fixed_iters=25))
    x = from_dev(x)
    assert np.all(x[1] == 0) and st[1][0] == dl.DL_OK
    for r in (0, 2):
        ref = oracle.solve_lp(U, b[r], dims, kappa, niter=25)
        assert np.linalg.norm(x[r] - ref) / np.linalg.norm(ref) < 3e-2
    V = int(np.prod(dims))
    empty = torch.zeros((0, V, 4, 3), dtype=torch.complex128, device=dev)
    with pytest.raises(dl.DLError):
        dl.solve(G, kappa, empty)
    with pytest.raises(dl.DLError):
        dl.apply(G, kappa, dl.DL_OP_DHOP, empty)
