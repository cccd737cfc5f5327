#!/usr/bin/env python3
"""Benchmark of the disconnected-loop hot path on one MI355X.

One step = one full plain FP64 loop estimate on the paper-shape lattice
(16^3 x 32, synthetic SU(3) field with eps = 0.35, kappa = 0.150): 24 complex
Z2 noises, each spin-colour diluted (288 right-hand sides), even-odd
preconditioned BiCGStab to a true relative residual of 1e-10, and the loop
traces L_1(t), L_gamma5(t).  The gauge field and all workspaces are resident
on the GPU before the timed region; the sources are generated on the GPU
inside it.

The JSON line reports the hopping kernel's achieved bandwidth (algorithmic
bytes of every launch, each operand moved once, over the summed event-timed
kernel durations on the library's stream) as `value` and against the HBM
roofline, the time per step / per converged solve, and the CPU oracle timed
on a bounded sample of the same workload.

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
    ap.add_argument("--cpu-only", action="store_true", help="time only the CPU oracle sample")
    return ap.parse_args()


def cpu_baseline(w):
    """The oracle (plain FP64, full lattice, OpenMP) on a bounded sample: one
    spin-colour-diluted source of noise 0 solved to 1e-10 plus its trace; the
    hopping-term rate is taken from one timed application of D."""
    import numpy as np

    import oracle
    import synth

    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    V = int(np.prod(dims))
    psi = synth.random_spinor(dims, 1, seed=7)[0]
    oracle.dhop(U, psi, dims)  # page in
    t0 = time.perf_counter()
    oracle.dhop(U, psi, dims)
    t_d = time.perf_counter() - t0
    # a full-lattice application is two half-lattice ones: 2 * Vh * 1152 bytes (FP64, 12-param links)
    gbs = 2 * (V // 2) * 1152 / t_d / 1e9
    eta = oracle.z2_source(dims, w["noise_seed"], 0, oracle.SCHEME_SPIN_COLOUR, 0)
    t0 = time.perf_counter()
    s, iters, res = oracle.solve(U, eta, dims, kappa, tol=1e-10)
    oracle.loops_accumulate(dims, eta, s, [0, 15])
    t_solve = time.perf_counter() - t0
    return {
        "value": gbs,
        "unit": "GB/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "one D application on 16^3x32 (hopping-kernel rate) and one FP64 BiCGStab solve to 1e-10 "
                  "(%d iterations) + trace: %.2f s per converged solve" % (iters, t_solve),
        "seconds_per_solve": t_solve,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
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
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    lat = dl.Lattice(dims, 1)
    G = dl.Gauge(lat, U, precs=(dl.DL_F64,), recon=12)
    stream = torch.cuda.current_stream()
    prm = dl.solve_params(tol=1e-10, maxiter=1000)
    gam = [0, 15]
    src = dl.z2_sources(w["noise_seed"], args.noises, scheme=dl.DL_DIL_SPIN_COLOUR)
    nrhs = dl.dl_sources_count(lat.h, src)

    def step():
        return dl.loops(G, kappa, src, gam, prm)

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
    dl.dl_profile_enable(False)
    assert all(s[0] == dl.DL_OK for s in st), "a solve did not converge"

    ms_step = elapsed / args.steps * 1e3
    dslash_gbs = by_d / (ms_d * 1e-3) / 1e9
    plain_gbs = by_p / (ms_p * 1e-3) / 1e9
    out = {
        "metric": "dslash HBM GB/s; time per loop at fixed stat. error vs plain FP64 solver",
        "value": round(dslash_gbs, 1),
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
        "ms_per_converged_solve": round(ms_step / nrhs, 4),
        "mean_iterations": float(np.mean(iters)),
        "kernel_ms_per_step": {
            "dslash": round(ms_d / args.steps, 2),
            "krylov_vectors": round(ms_b / args.steps, 2),
            "sources_traces": round(ms_t / args.steps, 2),
        },
        "dslash_launches_per_step": n_d // args.steps,
        "roofline": {
            "kernel": "dslash_kernel<double,6,false,0,*> (plain half dslash D_oe, FP64, 12-parameter links)",
            "bound": "hbm",
            "achieved": round(plain_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(plain_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
            "launches": n_p,
            "avg_launch_us": round(ms_p / max(n_p, 1) * 1e3, 1),
            "algorithmic_bytes_per_launch": round(by_p / max(n_p, 1)),
        },
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_seconds_per_solve"] = round(cb["seconds_per_solve"], 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
