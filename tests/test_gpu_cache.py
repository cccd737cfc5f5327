"""The device memory cache: calls served from cached blocks (including a block
larger than the request) give the same results, bit for bit, as calls that
allocate afresh, and dl_cache_release empties the cache between calls."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_cached_workspaces_repeat_bit_for_bit(dl, dev):
    dims = (6, 4, 6, 10)
    U = synth.gauge_field(dims, 0.5, seed=601)
    G = dl.Gauge(dl.Lattice(dims, 1), U, precs=(dl.DL_F64, dl.DL_F32))
    prm = dl.solve_params(prec=dl.DL_F32, tol=1e-10, maxiter=2000)
    gam = [0, 15]
    src5 = dl.z2_sources(6010, 5, scheme=dl.DL_DIL_SPIN_COLOUR)
    src4 = dl.z2_sources(6010, 4, scheme=dl.DL_DIL_SPIN_COLOUR)
    dl.dl_cache_release()
    fresh5, _ = dl.loops(G, 0.124, src5, gam, prm)
    dl.dl_cache_release()
    fresh4, _ = dl.loops(G, 0.124, src4, gam, prm)
    # now the cache holds the 4-noise workspaces; a 5-noise call allocates, then releases
    again5, _ = dl.loops(G, 0.124, src5, gam, prm)
    # a 4-noise call may now be served by 5-noise blocks (48 of 60 right-hand sides: 4/5 of a block)
    again4, _ = dl.loops(G, 0.124, src4, gam, prm)
    assert np.array_equal(fresh5, again5)
    assert np.array_equal(fresh4, again4)
    dl.dl_cache_release()
    last4, _ = dl.loops(G, 0.124, src4, gam, prm)
    assert np.array_equal(last4, fresh4)
