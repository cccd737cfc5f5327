"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds input generation only -- gauge fields, random spinors and
random gauge rotations -- and none of the method's arithmetic (no Dirac
operator, no solver, no noise of the estimator, no contraction).  Both sides
read the bytes it produces.

Gauge fields stand in for the N_f = 2 Wilson ensemble of Section 2 of the
paper (16^3 x 32), which is not available: every link is
``U = exp(i eps H)`` with ``H = sum_a h_a lambda_a`` a traceless Hermitian
3x3 matrix built from eight unit-normal draws ``h_a`` and the Gell-Mann
matrices (normalised Tr lambda_a lambda_b = 2 delta_ab).  The exponential is
taken through the eigen-decomposition of ``H``; the rows are then
re-orthonormalised and the third row is rebuilt as the conjugated cross
product of the first two, so that every link is special unitary to rounding.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "gauge_field",
    "unit_field",
    "random_spinor",
    "random_su3",
    "WORKLOADS",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), complex128."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]).astype(np.complex128) / np.sqrt(3.0)
    return lam


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


_CACHE: dict = {}


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Seeded SU(3) field, complex128 array [4][V][3][3] (mu, site, row, col).

    Sites are ordered x fastest: i = x + X*(y + Y*(z + Z*t)).  The result is
    read-only and memoised per (dims, eps, seed) within the process.
    """
    dims = tuple(int(d) for d in dims)
    key = (dims, float(eps), int(seed))
    if key in _CACHE:
        return _CACHE[key]
    out = _gauge_field(dims, eps, seed, chunk)
    out.flags.writeable = False
    if len(_CACHE) > 8:
        _CACHE.clear()
    _CACHE[key] = out
    return out


def _gauge_field(dims, eps, seed, chunk):
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    lam = gell_mann()
    n = 4 * V
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        h = rng.standard_normal((hi - lo, 8))
        H = np.einsum("na,aij->nij", h, lam)
        w, vec = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        u = np.einsum("nij,nj,nkj->nik", vec, ph, np.conj(vec))
        out[lo:hi] = _reunitarise(u)
    return out.reshape(4, V, 3, 3)


def unit_field(dims) -> np.ndarray:
    """The free field U = 1, complex128 [4][V][3][3]."""
    V = int(np.prod(dims))
    u = np.zeros((4, V, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def random_spinor(dims, nrhs: int, seed: int) -> np.ndarray:
    """Gaussian complex spinor fields, complex128 [nrhs][V][4][3]."""
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nrhs, V, 4, 3))
    im = rng.standard_normal((nrhs, V, 4, 3))
    return (re + 1j * im) / np.sqrt(2.0)


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-random SU(3) matrices (QR of a complex Gaussian, phase-fixed)."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 0] /= det[:, None]
    return q


# The workloads: lattice shape, link spread eps, hopping parameter kappa,
# gauge-field seed and noise seed.  The shapes are those of the paper's
# 16^3 x 32 ensemble and of smaller or larger test lattices around it.
WORKLOADS = {
    "plain_4x4x4x4": dict(dims=(4, 4, 4, 4), eps=0.5, kappa=0.12, gauge_seed=1000, noise_seed=2000),
    "plain_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.35, kappa=0.150, gauge_seed=1001,
                              noise_seed=2001),
    "tsm_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.35, kappa=0.150, gauge_seed=1001,
                            noise_seed=2002),
    "batch_8x8x8x16": dict(dims=(8, 8, 8, 16), eps=0.30, kappa=0.145, gauge_seed=1003, noise_seed=2003),
    "batch_12x12x12x24": dict(dims=(12, 12, 12, 24), eps=0.35, kappa=0.148, gauge_seed=1013,
                              noise_seed=2013),
    "batch_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.40, kappa=0.150, gauge_seed=1023,
                              noise_seed=2023),
    "grad_24x24x24x48": dict(dims=(24, 24, 24, 48), eps=0.35, kappa=0.148, gauge_seed=1004, noise_seed=2004),
    "grad_4x4x4x4": dict(dims=(4, 4, 4, 4), eps=0.35, kappa=0.148, gauge_seed=1104, noise_seed=2104),
}
