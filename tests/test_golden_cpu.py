"""The stored expected values under tests/golden/ are the oracle's (recomputed here for a sample)."""
import json
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tsm_lp_reference_is_the_oracle_s():
    """Noise 5 of tests/golden/tsm_lp_fp64_16x16x16x32.json recomputed with the oracle: the FP64
    25-iteration CGNR loops and their Cauchy-Schwarz scales (summation order may differ with the
    thread count: 1e-12 relative)."""
    with open(os.path.join(GOLDEN, "tsm_lp_fp64_16x16x16x32.json")) as f:
        ref = json.load(f)
    w = synth.WORKLOADS["tsm_16x16x16x32"]
    dims, kappa = w["dims"], w["kappa"]
    U = synth.gauge_field(dims, w["eps"], w["gauge_seed"])
    r = next(x for x in ref["noises"] if x["noise"] == 5)
    eta = oracle.z2_source(dims, w["noise_seed"], 5)
    s = oracle.solve_lp(U, eta, dims, kappa, niter=25)
    L = oracle.loops_accumulate(dims, eta, s, ref["gammas"])
    stored = np.array(r["loops_re"]) + 1j * np.array(r["loops_im"])
    assert np.max(np.abs(L - stored)) <= 1e-12 * np.max(np.abs(stored))
    cs = np.linalg.norm(eta.reshape(-1, 12), axis=1) * np.linalg.norm(s.reshape(-1, 12), axis=1)
    cs = cs.reshape(dims[3], -1).sum(axis=1)
    assert np.max(np.abs(cs - np.array(r["cs_scale"]))) <= 1e-12 * np.max(cs)
