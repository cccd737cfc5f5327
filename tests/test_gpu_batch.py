"""Batched multi-lattice solves and captured-graph replays, through the C ABI.

* A batch over lattices of different shapes returns, per lattice, the loops
  of the single-lattice path (the batch may pick other launch shapes, so the
  reductions group differently: agreement within 1e-9 of the Cauchy-Schwarz
  scale) and of the oracle.
* Replaying the captured iteration chunks gives bit-identical loops to the
  eager launches of the same batch, call after call, with other GPU work in
  between.
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


SMALL = [((4, 4, 4, 4), 0.5, 0.12, 301), ((4, 4, 6, 8), 0.45, 0.125, 302), ((6, 4, 2, 8), 0.4, 0.118, 303)]


def build(dl, spec, precs=(0,)):
    out = []
    for dims, eps, kappa, seed in spec:
        U = synth.gauge_field(dims, eps, seed)
        lat = dl.Lattice(dims, 1)
        out.append((dims, U, kappa, dl.Gauge(lat, U, precs=precs)))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_matches_single_and_oracle(dl, dev, prec):
    lats = build(dl, SMALL, precs=(0, 1))
    gam = [0, 15, 5]
    srcs = [dl.z2_sources(400 + i, 2, scheme=dl.DL_DIL_SPIN_COLOUR if i != 1 else 0) for i in range(3)]
    prm = dl.solve_params(prec=prec, tol=1e-12, maxiter=2000)
    L, st = dl.batch_loops([g for *_, g in lats], [k for _, _, k, _ in lats], srcs, gam, prm)
    for i, (dims, U, kappa, G) in enumerate(lats):
        single, _ = dl.loops(G, kappa, srcs[i], gam, prm)
        scale = np.max(np.abs(single))
        assert np.max(np.abs(L[i] - single)) < 1e-9 * scale
        assert all(s[0] == dl.DL_OK and s[3] <= 1e-12 for s in st[i])
    # one lattice against the oracle
    dims, U, kappa, _ = lats[1]
    ref = oracle.loops_z2(U, dims, kappa, 401, [0, 1], 0, gam, tol=1e-13)
    assert np.max(np.abs(L[1] - ref)) < 1e-9 * np.max(np.abs(ref))


def test_graph_replay_bit_identical(dl, dev):
    lats = build(dl, SMALL)
    gam = [0, 15]
    srcs = [dl.z2_sources(500 + i, 3) for i in range(3)]
    ks = [k for _, _, k, _ in lats]
    gs = [g for *_, g in lats]
    eager, _ = dl.batch_loops(gs, ks, srcs, gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=3))
    for rep in range(3):
        graph, st = dl.batch_loops(gs, ks, srcs, gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=3, use_graph=True))
        for a, b in zip(eager, graph):
            assert np.array_equal(a, b), rep
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device=dev)
        torch.cuda.synchronize()
        assert float(x.abs().sum()) > 0
    # a single lattice in graph mode equals its eager run too
    dims, U, kappa, G = lats[0]
    e, _ = dl.loops(G, kappa, srcs[0], gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=2))
    g, _ = dl.loops(G, kappa, srcs[0], gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=2, use_graph=True))
    assert np.array_equal(e, g)


def test_batch_paper_shapes_mixed_precision(dl, dev):
    """The batch workload's three lattices (8^3x16, 12^3x24, 16^3x32; eps 0.30/0.35/0.40; kappa
    0.145/0.148/0.150) with spin-colour x cubic dilution, FP32 iterations with FP64 reliable updates,
    one noise each (96 right-hand sides per lattice), graph replay on."""
    names = ["batch_8x8x8x16", "batch_12x12x12x24", "batch_16x16x16x32"]
    gs, ks, srcs, Us = [], [], [], []
    for nm in names:
        w = synth.WORKLOADS[nm]
        U = synth.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
        lat = dl.Lattice(w["dims"], 1)
        gs.append(dl.Gauge(lat, U, precs=(0, 1)))
        ks.append(w["kappa"])
        srcs.append(dl.z2_sources(w["noise_seed"], 1, scheme=dl.DL_DIL_SPIN_COLOUR | dl.DL_DIL_CUBIC))
    prm = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000, use_graph=True)
    L, st = dl.batch_loops(gs, ks, srcs, [0, 15], prm)
    for i in range(3):
        assert len(st[i]) == 96 and all(s[0] == dl.DL_OK and s[3] <= 1e-10 for s in st[i])
        single, _ = dl.loops(gs[i], ks[i], srcs[i], [0, 15], dl.solve_params(tol=1e-10, maxiter=2000))
        # both solves meet 1e-10; the loops agree to that order on the Cauchy-Schwarz scale
        scale = 96 * np.prod(synth.WORKLOADS[names[i]]["dims"][:3]) / 8
        assert np.max(np.abs(L[i] - single)) < 1e-7 * scale


@pytest.mark.parametrize("own_stream", [False, True])
def test_capture_failure_leaves_the_stream_usable(dl, dev, monkeypatch, own_stream):
    """A failure inside a graph capture (forced from the host, after the capture has begun) comes back
    as an error; the capture is ended and its graph destroyed, so the same stream then runs an eager
    solve, a graph-replayed solve and ordinary torch work with correct results.  Covers the caller's
    own stream (captured directly) and the default stream (the library captures on a stream of its
    own ordered after it)."""
    dims, U, kappa, G = build(dl, SMALL[:1])[0]
    gam = [0, 15]
    src = dl.z2_sources(600, 2)
    ref, _ = dl.loops(G, kappa, src, gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=2))
    s = torch.cuda.Stream() if own_stream else torch.cuda.default_stream()
    with torch.cuda.stream(s):
        monkeypatch.setenv("DL_FAULT_INJECT", "capture")
        with pytest.raises(dl.DLError) as e:
            dl.loops(G, kappa, src, gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=2, use_graph=True))
        assert "injected" in str(e.value)
        monkeypatch.delenv("DL_FAULT_INJECT")
        assert not torch.cuda.is_current_stream_capturing()
        eager, st = dl.loops(G, kappa, src, gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=2))
        graph, st2 = dl.loops(G, kappa, src, gam, dl.solve_params(tol=1e-12, maxiter=2000, poll=2, use_graph=True))
        x = torch.arange(1 << 16, dtype=torch.float64, device=dev)
        total = float(x.sum())
    torch.cuda.synchronize()
    assert all(t[0] == dl.DL_OK for t in st + st2)
    assert np.array_equal(eager, ref) and np.array_equal(graph, ref)
    assert total == float((1 << 16) * ((1 << 16) - 1) // 2)
