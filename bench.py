#!/usr/bin/env python3
"""Benchmark of the disconnected-loop hot path on one MI355X.

One step = one full plain FP64 loop estimate on the paper-shape lattice
(16^3 x 32, synthetic SU(3) field with eps = 0.35, kappa = 0.150): 24 complex
Z2 noises, each spin-colour diluted (288 right-hand sides), even-odd
preconditioned BiCGStab to a true relative residual of 1e-10, and the loop
traces L_1(t), L_gamma5(t).  The gauge field and all workspaces are resident
on the GPU before the timed region; the sources are generated on the GPU
inside it.

The JSON line reports as `value` the achieved bandwidth of the plain half
dslash (the stencil without a fused epilogue: algorithmic bytes of every such
launch, each operand moved once, over their summed event-timed durations on
the library's stream), the same figure against the HBM roofline, the rate of
all hopping launches, the time per step / per converged solve, the truncated
solver method's time to equal variance with its measured per-loop error
against the FP64 oracle, and the CPU oracle timed on a bounded sample of the
same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--noises", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tsm", action="store_true", help="skip the truncated-solver-method comparison")
    ap.add_argument("--copy-reference", action="store_true",
                    help="first run a plain device copy (2 GiB read, 2 GiB written), the reference for hardware byte counters")
    ap.add_argument("--cpu-only", action="store_true", help="time only the CPU oracle sample")
    ap.add_argument("--dilution-study", action="store_true",
                    help="instead of the timed step: error of the time-averaged loop versus the number of "
                         "inversions for several dilution schemes (Gamma = 1, gamma5, gamma1 gamma3)")
    ap.add_argument("--batch", action="store_true",
                    help="instead of the timed step: the batched workload (8^3x16, 12^3x24, 16^3x32, 768 "
                         "right-hand sides each, FP32 iterations with FP64 reliable updates) with and without "
                         "graph replay")
    ap.add_argument("--differentiation", action="store_true",
                    help="instead of the timed step: the differentiation workload (24^3x48, 384 right-hand sides, "
                         "FP32 iterations with FP64 reliable updates; loops, their kappa derivative and their "
                         "link gradient)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="instead of the timed step: only the per-precision hopping-kernel sweep and the "
                         "single-right-hand-side figures")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the per-precision hopping-kernel sweep and the single-right-hand-side figures")
    return ap.parse_args()


def cpu_baseline(w, n_apply=10, n_solve=3):
    """The oracle (plain FP64, full lattice, OpenMP) on a bounded sample of the timed workload: the
    hopping-term rate from n_apply timed applications of D, and n_solve spin-colour-diluted sources of
    noise 0 (classes 0..n_solve-1) each solved to 1e-10 plus its trace; about 10 s on the 16 host
    threads of the GPU machine."""
    import numpy as np

    import oracle
    import synth

    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    V = int(np.prod(dims))
    psi = synth.random_spinor(dims, 1, seed=7)[0]
    oracle.dhop(U, psi, dims)  # page in
    t0 = time.perf_counter()
    for _ in range(n_apply):
        oracle.dhop(U, psi, dims)
    t_d = (time.perf_counter() - t0) / n_apply
    # a full-lattice application is two half-lattice ones: 2 * Vh * 1152 bytes (FP64, 12-param links)
    gbs = 2 * (V // 2) * 1152 / t_d / 1e9
    iters = []
    t0 = time.perf_counter()
    for c in range(n_solve):
        eta = oracle.z2_source(dims, w["noise_seed"], 0, oracle.SCHEME_SPIN_COLOUR, c)
        s, it, res = oracle.solve(U, eta, dims, kappa, tol=1e-10)
        oracle.loops_accumulate(dims, eta, s, [0, 15])
        iters.append(it)
    t_solve = (time.perf_counter() - t0) / n_solve
    return {
        "value": gbs,
        "unit": "GB/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "%d D applications on 16^3x32 (hopping-kernel rate) and %d FP64 BiCGStab solves to 1e-10 "
                  "(spin-colour classes 0-%d of noise 0, %s iterations) + traces: %.2f s per converged solve"
                  % (n_apply, n_solve, n_solve - 1, "/".join(str(i) for i in iters), t_solve),
        "seconds_per_solve": t_solve,
    }


def lp_error_vs_oracle(lp_loops, gammas):
    """Error of the low-precision loops of the first noises of the LP set against the FP64 run of the
    same truncated algorithm by the oracle, stored by tests/golden/make_tsm_lp_reference.py (no
    oracle code runs here): per Gamma, the largest over noises and t of |dL| / (sum_{x in t}
    |eta| |s|) (Cauchy-Schwarz-normalised) and of |dL(t)| / max_t |L(t)| (raw)."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "tsm_lp_fp64_16x16x16x32.json")
    with open(path) as f:
        ref = json.load(f)
    out = {"noises": len(ref["noises"]), "reference": "oracle FP64, same 25 CGNR iterations"}
    for k, g in enumerate(ref["gammas"]):
        gi = gammas.index(g)
        cs_max = raw_max = 0.0
        for r in ref["noises"]:
            L = np.array(r["loops_re"][k]) + 1j * np.array(r["loops_im"][k])
            d = np.abs(lp_loops[r["noise"]][gi] - L)
            cs_max = max(cs_max, float(np.max(d / np.array(r["cs_scale"]))))
            raw_max = max(raw_max, float(np.max(d) / np.max(np.abs(L))))
        out["gamma%d" % g] = {"cs_normalised_max": cs_max, "raw_max": raw_max}
    return out


def tsm_comparison(dl, G, w, L_plain, ms_plain, lp_prec=None):
    """Time per loop at fixed statistical error: the truncated solver method (400 low-precision
    truncated solves in FP16 storage (or lp_prec) / FP32 arithmetic, 25 CGNR iterations, plus 16
    high-precision corrections in FP32 with FP64 reliable updates to 1e-10, undiluted noises)
    against the plain FP64 estimate of the timed step (24 spin-colour-diluted noises), on the same
    field.  time_to_equal_variance = T_tsm * Var_tsm / Var_plain, per Gamma, averaged over t."""
    import numpy as np
    import torch

    t = synth_workload("tsm_16x16x16x32")
    gam = [0, 15]
    n_lp, n_hp = 400, 16
    lpp = dl.solve_params(solver=dl.DL_CGNR, prec=dl.DL_F16 if lp_prec is None else lp_prec, fixed_iters=25)
    hpp = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=1000)
    src = dl.z2_sources(t["noise_seed"], n_lp + n_hp)
    # warm-up on other noises with the same split: every launch shape of the timed call is tuned here
    dl.loops_tsm(G, t["kappa"], dl.z2_sources(t["noise_seed"] + 7, n_lp + n_hp), n_lp, n_hp, gam, lpp, hpp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, b, c, st = dl.loops_tsm(G, t["kappa"], src, n_lp, n_hp, gam, lpp, hpp)
    torch.cuda.synchronize()
    ms_tsm = (time.perf_counter() - t0) * 1e3
    est, var_t = dl.tsm_estimate(a, b, c)
    var_p = np.var(L_plain, axis=0, ddof=1) / len(L_plain)
    out = {"ms_tsm": round(ms_tsm, 2), "ms_plain": round(ms_plain, 2), "n_lp": n_lp, "n_hp": n_hp,
           "hp_converged": all(x[0] == dl.DL_OK for x in st[(n_lp + n_hp):]),
           "lp_loop_error_vs_fp64_oracle": lp_error_vs_oracle(a, gam)}
    # bootstrap over noises (LP set, HP set and the plain estimate's noises resampled independently)
    rng = np.random.default_rng(12345)
    nboot = 400
    ratios = np.empty((nboot, len(gam)))
    for i in range(nboot):
        il = rng.integers(0, n_lp, n_lp)
        ih = rng.integers(0, n_hp, n_hp)
        ip = rng.integers(0, len(L_plain), len(L_plain))
        _, vtb = dl.tsm_estimate(a[il], b[ih], c[ih])
        vpb = np.var(L_plain[ip], axis=0, ddof=1) / len(L_plain)
        ratios[i] = [np.mean(vtb[k].real) / np.mean(vpb[k].real) * ms_tsm / ms_plain for k in range(len(gam))]
    for k, g in enumerate(gam):
        vt = float(np.mean(var_t[k].real))
        vp = float(np.mean(var_p[k].real))
        lo, hi = np.percentile(ratios[:, k], [16, 84])
        out["gamma%d" % g] = {
            "var_tsm": vt, "var_plain": vp,
            "time_to_equal_variance_ms": round(ms_tsm * vt / vp, 2),
            "ratio_vs_plain": round(ms_tsm * vt / (vp * ms_plain), 4),
            "ratio_bootstrap_68": [round(float(lo), 4), round(float(hi), 4)],
        }
    return out


def copy_rate(torch):
    """Achievable HBM rate of a plain device copy: 2 GiB read + 2 GiB written, event-timed."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2 * 8 * n / (ms * 1e-3) / 1e9


def stream_rates(dl, torch):
    """The library's own streaming probe (dl_stream_probe: 16-byte non-temporal loads and stores,
    tiles of contiguous words, eight loads in flight per thread): a 2 GiB copy (2 GiB read + 2 GiB
    written) and a 4 GiB read, event-timed; GB/s of bytes moved."""
    a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB
    b = torch.empty_like(a)
    dl.stream_probe(a, b, 0, reps=1)
    copy_s = dl.stream_probe(a, b, 0, reps=5)
    big = torch.ones(1 << 29, dtype=torch.float64, device="cuda")  # 4 GiB
    dl.stream_probe(big, b, 1, reps=1)
    read_s = dl.stream_probe(big, b, 1, reps=5)
    out = {"copy_gbs": round(2 * a.numel() * 8 / copy_s / 1e9, 1), "read_gbs": round(big.numel() * 8 / read_s / 1e9, 1)}
    del a, b, big
    torch.cuda.empty_cache()
    return out


def hop_rate(dl, torch, G, nrhs, prec, reps=3):
    """Plain half-dslash launches of D applied to nrhs right-hand sides at one storage precision:
    (launches, algorithmic GB/s, mean event-timed launch in us, launch configuration).  The first
    application tunes; the profiled ones follow."""
    V = G.lattice.V
    x = torch.zeros((nrhs, V, 4, 3), dtype=torch.complex128, device="cuda")
    x.real.normal_()
    dl.apply(G, 0.15, dl.DL_OP_DHOP, x, prec=prec)
    torch.cuda.synchronize()
    dl.dl_profile_enable(True)
    for _ in range(reps):
        dl.apply(G, 0.15, dl.DL_OP_DHOP, x, prec=prec)
    torch.cuda.synchronize()
    n, ms, by = dl.dl_profile_read(3)
    cfg = dl.dl_profile_config(3)
    dl.dl_profile_enable(False)
    del x
    torch.cuda.empty_cache()
    return n, by / (ms * 1e-3) / 1e9, ms / max(n, 1) * 1e3, cfg


def dslash_sweep(dl, torch, G, copy_gbs):
    """The plain half dslash D_oe / D_eo at every storage precision on the timed workload's batch
    (16^3 x 32, 288 right-hand sides), the single-right-hand-side FP64 figure on the same lattice
    (its 75 MB working set sits in the 256 MB Infinity Cache), and the single-right-hand-side FP64
    figure on 24^3 x 48 (382 MB, larger than that cache)."""
    import synth

    out = {}
    names = {dl.DL_F64: "f64", dl.DL_F32: "f32", dl.DL_F16: "f16", dl.DL_BF16: "bf16"}
    for prec, nm in names.items():
        n, gbs, us, cfg = hop_rate(dl, torch, G, 288, prec)
        out[nm + "_288rhs"] = {"gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                               "frac_copy": round(gbs / copy_gbs, 4), "avg_launch_us": round(us, 1),
                               "launches": n, "config": list(cfg)}
    n, gbs, us, cfg = hop_rate(dl, torch, G, 1, dl.DL_F64, reps=20)
    out["f64_1rhs_cache_resident"] = {"gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                      "avg_launch_us": round(us, 1), "launches": n, "config": list(cfg)}
    w = synth.WORKLOADS["grad_24x24x24x48"]
    U = synth.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
    G2 = dl.Gauge(dl.Lattice(w["dims"], 1), U, precs=(dl.DL_F64,), recon=12)
    n, gbs, us, cfg = hop_rate(dl, torch, G2, 1, dl.DL_F64, reps=20)
    out["f64_1rhs_24x24x24x48"] = {"gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                   "frac_copy": round(gbs / copy_gbs, 4), "avg_launch_us": round(us, 1),
                                   "launches": n, "config": list(cfg)}
    del G2
    # one smearing step on 24 right-hand sides (FP64, 12-parameter links), profile kind 4
    x = torch.zeros((24, G.lattice.V, 4, 3), dtype=torch.complex128, device="cuda")
    x.real.normal_()
    dl.smear(G, 0.5, 2, x)
    torch.cuda.synchronize()
    dl.dl_profile_enable(True)
    dl.smear(G, 0.5, 10, x)
    torch.cuda.synchronize()
    n, ms, by = dl.dl_profile_read(4)
    dl.dl_profile_enable(False)
    del x
    out["smear_f64_24rhs"] = {"gbs": round(by / (ms * 1e-3) / 1e9, 1), "frac_hbm_peak": round(by / (ms * 1e-3) / 1e9
                                                                                               / HBM_PEAK_GBS, 4),
                              "avg_step_us": round(ms / max(n, 1) * 1e3, 1), "steps": n}
    return out


def differentiation_measurement(dl, torch, n_noise=32):
    """The differentiation row on its workload (24^3 x 48, eps 0.35, kappa 0.148, 32 spin-colour-
    diluted complex-Z2 noises = 384 right-hand sides, FP32 iterations with FP64 reliable updates to
    1e-10, Gamma = gamma5 and 1): wall time of the loop estimate, of its kappa derivative (two solves
    per right-hand side) and of its link gradient (forward and adjoint solves plus the outer-product
    kernel), each after a warm-up call of the same shape, with the kernel-time split of the gradient
    call."""
    import numpy as np
    import synth

    w = synth.WORKLOADS["grad_24x24x24x48"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64, dl.DL_F32), recon=12)
    src = dl.z2_sources(w["noise_seed"], n_noise, scheme=dl.DL_DIL_SPIN_COLOUR)
    nrhs = dl.dl_sources_count(G.lattice.h, src)
    gam = [15, 0]
    prm = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000)
    W = np.ones((len(gam), dims[3]), dtype=np.complex128)
    calls = {
        "loops": lambda: dl.loops(G, kappa, src, gam, prm),
        "dkappa": lambda: dl.loops_dkappa(G, kappa, src, gam, prm),
        "link_grad": lambda: dl.loops_link_grad(G, kappa, src, gam, W, prm),
    }
    out = {"workload": "24^3x48, kappa 0.148, %d spin-colour-diluted noises (%d RHS), FP32 iterations with FP64 "
                       "reliable updates to 1e-10" % (n_noise, nrhs)}
    for name, f in calls.items():
        f()
        torch.cuda.synchronize()
        if name == "link_grad":
            dl.dl_profile_enable(True)
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        out["ms_" + name] = round((time.perf_counter() - t0) * 1e3, 1)
        st = r[-1]
        assert all(x[0] == dl.DL_OK for x in st), name
        out["ms_per_rhs_" + name] = round(out["ms_" + name] / nrhs, 3)
    kinds = {"dslash": 0, "krylov_vectors": 1, "sources_traces_gradient": 2}
    split = {}
    for k, v in kinds.items():
        n, ms, by = dl.dl_profile_read(v)
        split[k] = {"ms": round(ms, 2), "gbs": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
    dl.dl_profile_enable(False)
    out["link_grad_kernel_split"] = split
    out["dkappa_vs_loops"] = round(out["ms_dkappa"] / out["ms_loops"], 3)
    out["link_grad_vs_loops"] = round(out["ms_link_grad"] / out["ms_loops"], 3)
    del G
    return out


def dilution_study(dl, G, w, n_noise=16):
    """The error-versus-inversions comparison of dilution schemes (Section 4, on the synthetic field):
    for each scheme, n_noise noises give per-noise estimates e_n of the time-averaged loop
    (1/T) sum_t L_Gamma(t) (under time dilution a noise sees one timeslice, so e_n = L_Gamma(t_n));
    the error after N noises is sigma / sqrt(N) at N_inv = N x (solves per noise).  `vs_optimal` is
    sigma sqrt(solves per noise) / sigma_undiluted: the scheme's error at equal N_inv relative to the
    1/sqrt(N_inv) extrapolation from the undiluted estimator (below 1: dilution pays)."""
    import numpy as np

    T = w["dims"][3]
    gam = {"1": 0, "gamma5": 15, "gamma1gamma3": 5}
    schemes = {"none": 0, "time": dl.DL_DIL_TIME, "colour": dl.DL_DIL_COLOUR, "spin": dl.DL_DIL_SPIN,
               "spin_even_odd": dl.DL_DIL_SPIN_EVEN_ODD, "spin_colour": dl.DL_DIL_SPIN_COLOUR,
               "spin_colour_time": dl.DL_DIL_SPIN_COLOUR | dl.DL_DIL_TIME,
               "spin_colour_even_odd": dl.DL_DIL_SPIN_COLOUR | dl.DL_DIL_EVEN_ODD,
               "spin_colour_cubic": dl.DL_DIL_SPIN_COLOUR | dl.DL_DIL_CUBIC}
    prm = dl.solve_params(tol=1e-10, maxiter=1000)
    res, sig0 = {}, {}
    for name, sch in schemes.items():
        src = dl.z2_sources(w["noise_seed"] + 500, n_noise, scheme=sch)
        per = dl.dl_sources_count(G.lattice.h, src) // n_noise
        t0 = time.perf_counter()
        L, st = dl.loops(G, w["kappa"], src, list(gam.values()), prm)
        secs = time.perf_counter() - t0
        assert all(x[0] == dl.DL_OK for x in st), name
        if sch & dl.DL_DIL_TIME:
            e = np.array([L[n][:, n % T] for n in range(n_noise)])  # [noise][gamma]
        else:
            e = L.mean(axis=2)
        out = {"solves_per_noise": per, "seconds": round(secs, 3)}
        for k, g in enumerate(gam):
            sigma = float(np.sqrt(np.mean(np.abs(e[:, k] - e[:, k].mean()) ** 2) * n_noise / (n_noise - 1)))
            if name == "none":
                sig0[g] = sigma
            out[g] = {"sigma_per_noise": sigma, "mean": [float(e[:, k].mean().real), float(e[:, k].mean().imag)],
                      "error_at_n_inv": [[per * m, sigma / np.sqrt(m)] for m in (1, 2, 4, 8, n_noise)],
                      "vs_optimal": sigma * np.sqrt(per) / sig0[g]}
        res[name] = out
    return {"study": "error of the time-averaged loop versus inversions per dilution scheme",
            "lattice": list(w["dims"]), "kappa": w["kappa"], "n_noise": n_noise, "schemes": res}


def batch_measurement(dl, torch):
    """The batched workload: three lattices (8^3x16, 12^3x24, 16^3x32; eps 0.30/0.35/0.40; kappa
    0.145/0.148/0.150), each with 8 complex-Z2 noises x 12 spin-colour x 8 cubic classes = 768
    right-hand sides, solved together (one launch per kernel over all lattices) in FP32 with FP64
    reliable updates to 1e-10, L_1 and L_gamma5; timed with hipGraph replay of the iteration chunks
    and without, after one untimed run that tunes every launch shape."""
    import synth

    names = ["batch_8x8x8x16", "batch_12x12x12x24", "batch_16x16x16x32"]
    gs, ks, srcs = [], [], []
    for nm in names:
        w = synth.WORKLOADS[nm]
        U = synth.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
        gs.append(dl.Gauge(dl.Lattice(w["dims"], 1), U, precs=(dl.DL_F64, dl.DL_F32)))
        ks.append(w["kappa"])
        srcs.append(dl.z2_sources(w["noise_seed"], 8, scheme=dl.DL_DIL_SPIN_COLOUR | dl.DL_DIL_CUBIC))
    out = {"workload": "3 lattices x 768 right-hand sides, FP32 iterations with FP64 reliable updates to 1e-10"}
    for graph in (True, False):
        prm = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000, use_graph=graph)
        dl.batch_loops(gs, ks, srcs, [0, 15], prm)  # tunes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, st = dl.batch_loops(gs, ks, srcs, [0, 15], prm)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        nsolve = sum(len(x) for x in st)
        assert all(s[0] == dl.DL_OK for x in st for s in x)
        out["graph" if graph else "no_graph"] = {"seconds": round(secs, 3), "solves": nsolve,
                                                 "solves_per_second": round(nsolve / secs, 1)}
    # kernel rates from a profiled eager run (launches inside a captured graph carry no events)
    prm = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000, use_graph=False)
    dl.dl_profile_enable(True)
    dl.batch_loops(gs, ks, srcs, [0, 15], prm)
    torch.cuda.synchronize()
    n_d, ms_d, by_d = dl.dl_profile_read(0)
    n_b, ms_b, by_b = dl.dl_profile_read(1)
    dl.dl_profile_enable(False)
    out["kernels"] = {"dslash_gbs": round(by_d / (ms_d * 1e-3) / 1e9, 1), "dslash_launches": n_d,
                      "dslash_ms": round(ms_d, 1), "krylov_vectors_gbs": round(by_b / (ms_b * 1e-3) / 1e9, 1),
                      "krylov_vectors_ms": round(ms_b, 1)}
    return out


def synth_workload(name):
    import synth

    return synth.WORKLOADS[name]


# Memory-side bytes per launch of the plain FP64 hopping kernel, from the two
# rocprofv3 counter runs of profiles/dslash_plain_f64_16x16x16x32_288rhs.md
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, KiB -> bytes, mean over the 174
# dispatches of the warm-up, timed and unprofiled steps), keyed by the launch
# configuration they were taken with.  Another configuration reports null.
PROFILED_TRAFFIC = {(1, 1, 0, 128): 7.42e9}


def kernel_name(cfg):
    """The plain FP64 hopping kernel the autotuner chose, as rocprofv3 names it."""
    kind, nr, bs, pg = cfg
    what = "plain half dslash D_oe, FP64, 12-parameter links"
    if kind == 1:
        # four 64-site blocks per CU fit the LDS (36 KiB of spatial FP64 links as stored each; the
        # temporal links sit in registers)
        occ = ("%d per CU, set by the LDS" % (4 * nr)) if bs == 0 else "at most %d per SIMD" % bs
        return ("dslash_lds_kernel<double,6,false,0,%d,%d> (%s; spatial links of 64-site blocks in LDS, temporal "
                "links in registers, %d wavefronts per block (%s), regions of %d blocks)" % (nr, bs, what, nr, occ, pg))
    return "dslash_kernel<double,6,false,0,%d> (%s; %d sites per workgroup%s)" % (
        nr, what, bs, ", persistent grid of %d" % pg if pg else "")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synth

    w = synth.WORKLOADS["plain_16x16x16x32"]
    if args.cpu_only:
        print(json.dumps(cpu_baseline(w)))
        return

    import torch

    import paper_1012_5168_amd as dl

    dl.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    # this process owns the GPU: keep the workspaces of every workload in the library's memory cache
    dl.dl_cache_set_limit(256 << 30)
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64, dl.DL_F32, dl.DL_F16, dl.DL_BF16), recon=12)
    stream = torch.cuda.current_stream()
    if args.dilution_study:
        print(json.dumps(dilution_study(dl, G, w)), flush=True)
        return
    if args.batch:
        del G
        print(json.dumps(batch_measurement(dl, torch)), flush=True)
        return
    if args.differentiation:
        del G
        print(json.dumps(differentiation_measurement(dl, torch)), flush=True)
        return
    if args.sweep_only:
        cg = copy_rate(torch)  # its copies (2 GiB read, 2 GiB written) also serve as the counters' reference
        print(json.dumps({"copy_reference_gbs": round(cg, 1), "dslash_by_precision": dslash_sweep(dl, torch, G, cg)}),
              flush=True)
        return
    prm = dl.solve_params(tol=1e-10, maxiter=1000)
    gam = [0, 15]
    src = dl.z2_sources(w["noise_seed"], args.noises, scheme=dl.DL_DIL_SPIN_COLOUR)
    nrhs = dl.dl_sources_count(lat.h, src)

    def step():
        return dl.loops(G, kappa, src, gam, prm)

    if args.copy_reference:
        n = 1 << 28  # 2^28 doubles: 2 GiB read once and written once
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print("copy reference: %d bytes read, %d bytes written" % (8 * n, 8 * n), file=sys.stderr, flush=True)
        del a, b

    for _ in range(args.warmup):
        L, st = step()
        print("warmup step done", flush=True, file=sys.stderr)
    torch.cuda.synchronize()
    dl.dl_profile_enable(True)
    t0 = time.perf_counter()
    iters = []
    for k in range(args.steps):
        L, st = step()
        iters.extend(s[1] for s in st)
        print("step %d done" % k, flush=True, file=sys.stderr)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_d, ms_d, by_d = dl.dl_profile_read(0)
    n_b, ms_b, by_b = dl.dl_profile_read(1)
    n_t, ms_t, by_t = dl.dl_profile_read(2)
    n_p, ms_p, by_p = dl.dl_profile_read(3)
    cfg = dl.dl_profile_config(3)
    dl.dl_profile_enable(False)
    assert all(s[0] == dl.DL_OK for s in st), "a solve did not converge"

    ms_step = elapsed / args.steps * 1e3
    # one more step without the per-launch profiling events, for the truncated solver method's time
    # ratio (its calls run unprofiled too)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    ms_step_unprofiled = (time.perf_counter() - t0) * 1e3
    dslash_gbs = by_d / (ms_d * 1e-3) / 1e9
    plain_gbs = by_p / (ms_p * 1e-3) / 1e9
    out = {
        "metric": "dslash HBM GB/s; time per loop at fixed stat. error vs plain FP64 solver",
        "value": round(plain_gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain FP64 loop estimate, 16^3x32, eps 0.35, kappa 0.150, 24 Z2 noises x 12 "
                        "spin-colour dilution = %d right-hand sides, even-odd BiCGStab to 1e-10, L_1 and L_g5"
                        % nrhs,
            "lattice": list(dims),
            "rhs": nrhs,
        },
        "ms_per_step_unprofiled": round(ms_step_unprofiled, 2),
        "ms_per_converged_solve": round(ms_step / nrhs, 4),
        "mean_iterations": float(np.mean(iters)),
        "kernel_ms_per_step": {
            "dslash": round(ms_d / args.steps, 2),
            "krylov_vectors": round(ms_b / args.steps, 2),
            "sources_traces": round(ms_t / args.steps, 2),
        },
        "dslash_launches_per_step": n_d // args.steps,
        "kernel_gbs": {
            "dslash": round(dslash_gbs, 1),
            "krylov_vectors": round(by_b / (ms_b * 1e-3) / 1e9, 1),
            "sources_traces": round(by_t / (ms_t * 1e-3) / 1e9, 1) if ms_t > 0 else None,
        },
        "roofline": {
            "kernel": kernel_name(cfg),
            "bound": "hbm",
            "achieved": round(plain_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(plain_gbs / HBM_PEAK_GBS, 4),
            "traffic": PROFILED_TRAFFIC.get(tuple(cfg)),
            "traffic_unit": "bytes per launch (L2 fill + write-back, rocprofv3 FETCH_SIZE/WRITE_SIZE)",
            "launches": n_p,
            "avg_launch_us": round(ms_p / max(n_p, 1) * 1e3, 1),
            "algorithmic_bytes_per_launch": round(by_p / max(n_p, 1)),
        },
    }
    if not args.no_tsm:
        out["tsm"] = tsm_comparison(dl, G, w, L, ms_step_unprofiled)
        # the same split with the low-precision solves in BF16 storage (coarser mantissa, no scales)
        out["tsm_bf16_lp"] = tsm_comparison(dl, G, w, L, ms_step_unprofiled, lp_prec=dl.DL_BF16)
        # the same 288 solves with FP32 iterations and FP64 reliable updates to the same 1e-10
        pm = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000)
        dl.loops(G, kappa, src, gam, pm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Lm, stm = dl.loops(G, kappa, src, gam, pm)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t0) * 1e3
        assert all(x[0] == dl.DL_OK for x in stm), "a mixed-precision solve did not converge"
        out["ms_per_converged_solve_mixed"] = round(ms_m / nrhs, 4)
        out["mixed_vs_fp64_max_loop_diff_rel"] = float(np.max(np.abs(Lm - L)) / np.max(np.abs(L)))
    if not args.no_sweep:
        cg = copy_rate(torch)
        out["copy_reference_gbs"] = round(cg, 1)
        out["roofline"]["frac_of_copy"] = round(plain_gbs / cg, 4)
        # the library's own streaming kernels: the rate its access pattern gets from the memory system
        st = stream_rates(dl, torch)
        out["stream_reference_gbs"] = st
        out["roofline"]["frac_of_stream_copy"] = round(plain_gbs / st["copy_gbs"], 4)
        out["roofline"]["frac_of_stream_read"] = round(plain_gbs / st["read_gbs"], 4)
        out["dslash_by_precision"] = dslash_sweep(dl, torch, G, cg)
        out["differentiation"] = differentiation_measurement(dl, torch)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_seconds_per_solve"] = round(cb["seconds_per_solve"], 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
