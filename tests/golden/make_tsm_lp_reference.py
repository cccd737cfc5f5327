#!/usr/bin/env python3
"""Writes tests/golden/tsm_lp_fp64_16x16x16x32.json: the oracle's low-precision loops of the
truncated solver method's workload, computed in FP64, for the error of the GPU's FP16 / BF16 runs
of the same algorithm.

Workload (the truncated-solver leg of the benchmark): 16^3 x 32, eps 0.35, kappa 0.150, antiperiodic
time; undiluted complex-Z2 noises 0..7 of seed 2002 (the first noises of the low-precision set); the
low-precision solve is CG on the normal equations of the even-site Schur system, exactly 25
iterations from x0 = 0 (the truncated solve of Section 2 as this library reads it), here in FP64.
Stored per noise: L_Gamma(t) = eta^+ P_t Gamma s for Gamma in {1, gamma5} and the Cauchy-Schwarz
scale sum_{x in t} |eta(x)| |s(x)| of the loop error.  Calls only oracle/ (and synth/ for the
inputs); takes about half a minute on 8 cores.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

N_NOISE = 8
GAMMAS = [0, 15]


def main():
    w = synth.WORKLOADS["tsm_16x16x16x32"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    T, per_t = dims[3], int(np.prod(dims[:3]))
    out = {"workload": "16^3x32, eps 0.35, kappa 0.150, undiluted complex-Z2 noises 0-7 of seed %d, 25 CGNR "
                       "iterations (even-odd Schur normal equations, x0 = 0) in FP64" % w["noise_seed"],
           "gammas": GAMMAS, "noises": []}
    for n in range(N_NOISE):
        eta = oracle.z2_source(dims, w["noise_seed"], n)
        s = oracle.solve_lp(U, eta, dims, kappa, niter=25)
        L = oracle.loops_accumulate(dims, eta, s, GAMMAS)
        cs = (np.linalg.norm(eta.reshape(-1, 12), axis=1) * np.linalg.norm(s.reshape(-1, 12), axis=1))
        cs = cs.reshape(T, per_t).sum(axis=1)
        out["noises"].append({"noise": n, "loops_re": L.real.tolist(), "loops_im": L.imag.tolist(),
                              "cs_scale": cs.tolist()})
        print("noise %d done" % n, flush=True)
    with open(os.path.join(HERE, "tsm_lp_fp64_16x16x16x32.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
