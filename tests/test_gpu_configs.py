"""Parity of the HIP path against the FP64 CPU oracle on the workloads themselves.

* The plain method on 4^3 x 4 (eps 0.5, kappa 0.12, antiperiodic time): the 12
  spin-colour point sources at site 0 plus 16 complex-Z2 noises, every one of
  the 16 Gamma, solved to a relative residual of 1e-12.
* The paper-shape estimate on 16^3 x 32 (eps 0.35, kappa 0.150): 24 noises x 12
  spin-colour classes = 288 right-hand sides in one call (the batch the
  benchmark times), Gamma in {1, gamma5}, with a sampled noise compared against
  the oracle.
* One lattice of the batched workload (8^3 x 16, eps 0.30, kappa 0.145, 8-way
  cubic x 12 spin-colour dilution = 96 right-hand sides) inside the
  three-lattice batch call with FP32 iterations, FP64 reliable updates and
  graph replay, against the oracle.

Bar (the loop error is a solver error: |eta^+ Gamma M^-1 r| <= |M^-dag Gamma^+ eta| |r|
scales with |eta| |s|, not with |L|, and L_gamma5 can be small through
cancellation): |L_gpu(t) - L_oracle(t)| / sum_d sum_{x in t} |eta_d(x)| |s_d(x)| < 1e-10
with the GPU solving to 1e-12 and the oracle to 1e-13.  The raw |dL| / |L| is
reported beside it.
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


def cs_norm(dims, etas, sols):
    """sum over sources of sum_{x in t} |eta(x)| |s(x)| per timeslice."""
    T = dims[3]
    per_t = int(np.prod(dims[:3]))
    out = np.zeros(T)
    for e, s in zip(etas, sols):
        v = np.linalg.norm(e.reshape(-1, 12), axis=1) * np.linalg.norm(s.reshape(-1, 12), axis=1)
        out += v.reshape(T, per_t).sum(axis=1)
    return out


def errors(L_gpu, L_ref, norm):
    """(Cauchy-Schwarz-normalised error, raw relative error) over every Gamma and t."""
    cs = float(np.max(np.abs(L_gpu - L_ref) / norm[None, :]))
    raw = float(np.max(np.abs(L_gpu - L_ref)) / np.max(np.abs(L_ref)))
    return cs, raw


def report(name, cs, raw):
    print("PARITY %s: CS-normalised %.3e, raw |dL|/|L| %.3e" % (name, cs, raw), flush=True)


def test_plain_4x4x4x4_point_and_z2_all_gammas(dl, dev):
    w = synth.WORKLOADS["plain_4x4x4x4"]
    dims, kappa = w["dims"], w["kappa"]
    assert dims == (4, 4, 4, 4) and kappa == 0.12 and w["eps"] == 0.5
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    G = dl.Gauge(dl.Lattice(dims, 1), U)
    gam = list(range(16))
    prm = dl.solve_params(tol=1e-12, maxiter=500)
    # the 12 point sources at site 0: the exact loop Tr[Gamma M^-1(0, 0)] at t = 0
    L, st = dl.loops(G, kappa, dl.point_sources(0), gam, prm)
    assert len(st) == 12 and all(s[0] == dl.DL_OK and s[3] <= 1e-12 for s in st), st
    etas = [oracle.point_source(dims, 0, a, c) for a in range(4) for c in range(3)]
    sols = [oracle.solve(U, e, dims, kappa, 1e-13)[0] for e in etas]
    ref = np.zeros((16, dims[3]), dtype=np.complex128)
    for e, s in zip(etas, sols):
        ref = oracle.loops_accumulate(dims, e, s, gam, ref)
    norm = cs_norm(dims, etas, sols)
    # timeslices other than t = 0 hold exact zeros on both sides
    assert np.all(L[0][:, 1:] == 0) and np.all(ref[:, 1:] == 0)
    cs = float(np.max(np.abs(L[0][:, 0] - ref[:, 0]) / norm[0]))
    raw = float(np.max(np.abs(L[0] - ref)) / np.max(np.abs(ref)))
    report("4^3x4 point sources, 16 Gamma", cs, raw)
    assert cs < 1e-10, (cs, raw)
    # 16 complex-Z2 noises, undiluted
    n_noise = 16
    Lz, st = dl.loops(G, kappa, dl.z2_sources(w["noise_seed"], n_noise), gam, prm)
    assert len(st) == n_noise and all(s[0] == dl.DL_OK and s[3] <= 1e-12 for s in st), st
    refz, solz = oracle.loops_z2(U, dims, kappa, w["noise_seed"], range(n_noise), 0, gam, tol=1e-13,
                                 return_solutions=True)
    worst_cs = worst_raw = 0.0
    for n in range(n_noise):
        eta = oracle.z2_source(dims, w["noise_seed"], n)
        cs, raw = errors(Lz[n], refz[n], cs_norm(dims, [eta], [solz[n]]))
        worst_cs, worst_raw = max(worst_cs, cs), max(worst_raw, raw)
    report("4^3x4 16 Z2 noises, 16 Gamma", worst_cs, worst_raw)
    assert worst_cs < 1e-10, (worst_cs, worst_raw)


@pytest.mark.timeout(900)
def test_paper_shape_288_rhs_sampled_noises(dl, dev):
    """The timed workload's batch (24 noises x 12 spin-colour classes at 16^3 x 32) in one call,
    solved to 1e-12; noise 17 (a right-hand-side group inside the batch) compared with the oracle's
    loops, every Gamma and t."""
    w = synth.WORKLOADS["plain_16x16x16x32"]
    dims, kappa = w["dims"], w["kappa"]
    assert dims == (16, 16, 16, 32) and kappa == 0.150 and w["eps"] == 0.35
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    G = dl.Gauge(dl.Lattice(dims, 1), U)
    gam = [0, 15]
    src = dl.z2_sources(w["noise_seed"], 24, scheme=dl.DL_DIL_SPIN_COLOUR)
    L, st = dl.loops(G, kappa, src, gam, dl.solve_params(tol=1e-12, maxiter=2000))
    assert len(st) == 288 and all(s[0] == dl.DL_OK and s[3] <= 1e-12 for s in st)
    for n in (17,):
        print("oracle: noise %d, 12 solves at 16^3x32" % n, flush=True)
        ref, sols = oracle.loops_z2(U, dims, kappa, w["noise_seed"], [n], oracle.SCHEME_SPIN_COLOUR, gam,
                                    tol=1e-13, return_solutions=True)
        etas = [oracle.z2_source(dims, w["noise_seed"], n, oracle.SCHEME_SPIN_COLOUR, d) for d in range(12)]
        cs, raw = errors(L[n], ref[0], cs_norm(dims, etas, sols))
        report("16^3x32 288 RHS, noise %d, L_1 and L_g5" % n, cs, raw)
        assert cs < 1e-10, (n, cs, raw)


@pytest.mark.timeout(900)
def test_batch_paper_shapes_lattice_against_oracle(dl, dev):
    """The three-lattice batch (8^3x16, 12^3x24, 16^3x32), one noise x 96 classes each, FP32
    iterations with FP64 reliable updates to 1e-12 and graph replay; the 8^3x16 lattice's loops
    against the oracle's FP64 solves of the same 96 sources."""
    names = ["batch_8x8x8x16", "batch_12x12x12x24", "batch_16x16x16x32"]
    gs, ks, srcs, Us = [], [], [], []
    for nm in names:
        w = synth.WORKLOADS[nm]
        U = synth.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
        Us.append(U)
        gs.append(dl.Gauge(dl.Lattice(w["dims"], 1), U, precs=(dl.DL_F64, dl.DL_F32)))
        ks.append(w["kappa"])
        srcs.append(dl.z2_sources(w["noise_seed"], 1, scheme=dl.DL_DIL_SPIN_COLOUR | dl.DL_DIL_CUBIC))
    gam = [0, 15]
    prm = dl.solve_params(prec=dl.DL_F32, tol=1e-12, maxiter=4000, use_graph=True)
    L, st = dl.batch_loops(gs, ks, srcs, gam, prm)
    for i in range(3):
        assert len(st[i]) == 96 and all(s[0] == dl.DL_OK and s[3] <= 1e-12 for s in st[i]), i
    w = synth.WORKLOADS[names[0]]
    dims, kappa = w["dims"], w["kappa"]
    scheme = oracle.SCHEME_SPIN_COLOUR | oracle.SCHEME_CUBIC
    print("oracle: 96 solves at 8^3x16", flush=True)
    ref, sols = oracle.loops_z2(Us[0], dims, kappa, w["noise_seed"], [0], scheme, gam, tol=1e-13,
                                return_solutions=True)
    etas = [oracle.z2_source(dims, w["noise_seed"], 0, scheme, d) for d in range(96)]
    cs, raw = errors(L[0][0], ref[0], cs_norm(dims, etas, sols))
    report("batch 8^3x16 in the 3-lattice call, 96 RHS, FP32 + FP64 reliable updates", cs, raw)
    assert cs < 1e-10, (cs, raw)
