"""Plain FP64 CPU oracle for the disconnected-loop method (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP path; both sides read inputs from :mod:`synth` only.

The arithmetic lives in ``wilson_oracle.c`` (plain C, FP64, full lattice,
4x4 spin matrices applied as matrices).  This module loads it through ctypes
and adds the estimator drivers, each a direct transcription of the method:

* :func:`loops_point` -- the exact local loop at one site from its twelve
  unit (point) sources (Section 2, exact all-to-all evaluation, restricted to
  one site);
* :func:`loops_z2` -- the stochastic estimate with complex Z2 noise and an
  optional dilution (Section 2): for each noise and each dilution class,
  solve ``M s = eta_d`` and contract ``eta_d^+ Gamma s`` per timeslice
  (Section 3, zero-momentum local loop);
* :func:`loops_lp` -- the same with the truncated low-precision solve of the
  truncated solver method (Section 2), run in FP64;
* :func:`tsm_combine` -- the truncated solver method's estimate: mean of the
  low-precision set plus the mean high-minus-low correction (Section 2);
* :func:`loops_dkappa` and :func:`loops_link_grad` -- derivatives of the same
  estimators, from ``dM^-1/dkappa = M^-1 D M^-1`` and the adjoint solve;
* :func:`disconnected_correlator` -- the two-loop (disconnected) correlator of
  Section 3, Eq. (2), from per-noise loop estimates over distinct noise pairs;
* :func:`smear` and :func:`loops_z2_smeared` -- gauge-covariant Gaussian
  smearing of quark fields (Section 2) and the loop of smeared fields,
  estimated with the smeared noise xi = S eta at source and sink;
* :func:`eta_prime_fit` -- the flavour-singlet combination (Section 3, Eq. 3)
  and the fit of the disconnected-to-connected ratio (Eq. 4) with the pion
  mass given, jackknife errors over configurations.

Parity is pinned against closed forms, invariants and dense linear algebra in
``tests/test_oracle_pins.py``; the pins are listed in the header of that file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP); returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
             _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, i64, f64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        sig = {
            "or_dhop": (None, [P, i32, P, P, P]),
            "or_dhop_dag": (None, [P, i32, P, P, P]),
            "or_apply_m": (None, [P, i32, P, f64, P, P]),
            "or_apply_mdag": (None, [P, i32, P, f64, P, P]),
            "or_apply_mhat": (None, [P, i32, P, f64, P, P, i32]),
            "or_bicgstab": (i32, [P, i32, P, f64, P, P, f64, i32, P]),
            "or_cgnr_eo": (None, [P, i32, P, f64, P, P, i32]),
            "or_splitmix64": (u64, [u64, u64]),
            "or_z2_source": (None, [P, u64, i64, i32, i32, P]),
            "or_dilution_class": (i32, [P, i32, i64, i32, i32]),
            "or_dilution_count": (i32, [i32]),
            "or_dilution_valid": (i32, [i32]),
            "or_smear": (None, [P, P, ctypes.c_double, i32, P, P]),
            "or_loops_accumulate": (None, [P, P, P, i32, P, P]),
            "or_link_grad_accumulate": (None, [P, i32, f64, P, P, P]),
            "or_gamma5": (None, [P, P]),
            "or_weighted_gamma_dag": (None, [P, P, i32, P, P, P]),
            "or_gamma": (None, [i32, P]),
            "or_parity": (i32, [P, i64]),
            "or_num_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _dims(dims) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- operators


def gamma(n: int) -> np.ndarray:
    """Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3 (chiral basis), 4x4 complex."""
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().or_gamma(int(n), _ptr(out))
    return out


def dhop(U, psi, dims, tap=1, dag=False) -> np.ndarray:
    """D psi (or D^dagger psi) on the full lattice; psi is [V][4][3] complex."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    f = lib().or_dhop_dag if dag else lib().or_dhop
    f(_ptr(_dims(dims)), int(tap), _ptr(U), _ptr(psi), _ptr(out))
    return out


def apply_m(U, psi, dims, kappa, tap=1, dag=False) -> np.ndarray:
    """M psi = psi - kappa D psi (or M^dagger psi, assembled directly)."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    f = lib().or_apply_mdag if dag else lib().or_apply_m
    f(_ptr(_dims(dims)), int(tap), _ptr(U), float(kappa), _ptr(psi), _ptr(out))
    return out


def apply_mhat(U, psi, dims, kappa, tap=1, dag=False) -> np.ndarray:
    """Even-site Schur operator 1 - k^2 D_eo D_oe (psi supported on even sites)."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_apply_mhat(_ptr(_dims(dims)), int(tap), _ptr(U), float(kappa), _ptr(psi), _ptr(out), int(dag))
    return out


def parity(dims) -> np.ndarray:
    """(x+y+z+t)&1 per site, computed from the coordinates."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return ((x + y + z + t) & 1).reshape(-1).astype(np.int32)


# ---------------------------------------------------------------- solvers


def solve(U, b, dims, kappa, tol=1e-13, maxiter=20000, tap=1):
    """Full-lattice FP64 BiCGStab for M x = b; returns (x, iterations, true residual)."""
    U, b = _c128(U), _c128(b)
    x = np.empty_like(b)
    res = ctypes.c_double(0.0)
    it = lib().or_bicgstab(_ptr(_dims(dims)), int(tap), _ptr(U), float(kappa), _ptr(b), _ptr(x), float(tol),
                           int(maxiter), ctypes.byref(res))
    if it < 0:
        raise RuntimeError("oracle BiCGStab did not reach %g (true residual %g)" % (tol, res.value))
    return x, int(it), float(res.value)


def solve_lp(U, b, dims, kappa, niter=25, tap=1):
    """The truncated low-precision solve (even-odd CGNR, x0 = 0, niter iterations), in FP64."""
    U, b = _c128(U), _c128(b)
    x = np.empty_like(b)
    lib().or_cgnr_eo(_ptr(_dims(dims)), int(tap), _ptr(U), float(kappa), _ptr(b), _ptr(x), int(niter))
    return x


# ---------------------------------------------------------------- noise


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().or_splitmix64(seed & (2**64 - 1), counter & (2**64 - 1)))


SCHEME_NONE, SCHEME_SPIN_COLOUR, SCHEME_CUBIC, SCHEME_EVEN_ODD = 0, 1, 2, 4
SCHEME_COLOUR, SCHEME_SPIN, SCHEME_SPIN_EVEN_ODD, SCHEME_TIME = 8, 16, 32, 64


def dilution_valid(scheme: int) -> bool:
    return bool(lib().or_dilution_valid(int(scheme)))


def dilution_count(scheme: int) -> int:
    return int(lib().or_dilution_count(int(scheme)))


def dilution_class(dims, scheme, site, spin, col) -> int:
    return int(lib().or_dilution_class(_ptr(_dims(dims)), int(scheme), int(site), int(spin), int(col)))


def z2_source(dims, seed, noise, scheme=0, d=-1) -> np.ndarray:
    """Complex Z2 noise vector number `noise`, masked to dilution class d (d=-1: whole)."""
    V = int(np.prod(dims))
    out = np.empty((V, 4, 3), dtype=np.complex128)
    lib().or_z2_source(_ptr(_dims(dims)), int(seed) & (2**64 - 1), int(noise), int(scheme), int(d), _ptr(out))
    return out


def point_source(dims, site, spin, col) -> np.ndarray:
    V = int(np.prod(dims))
    out = np.zeros((V, 4, 3), dtype=np.complex128)
    out[site, spin, col] = 1.0
    return out


# ---------------------------------------------------------------- contractions


def loops_accumulate(dims, eta, s, gammas, out=None) -> np.ndarray:
    """out[g][t] += sum_{x in t} eta^+ Gamma_g s (complex, [n_gamma][T])."""
    gam = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    T = int(dims[3])
    buf = np.zeros((len(gam), T, 2), dtype=np.float64)
    if out is not None:
        buf[..., 0], buf[..., 1] = out.real, out.imag
    lib().or_loops_accumulate(_ptr(_dims(dims)), _ptr(_c128(eta)), _ptr(_c128(s)), len(gam), _ptr(gam), _ptr(buf))
    return buf[..., 0] + 1j * buf[..., 1]


def _sources(dims, seed, noise, scheme):
    nd = dilution_count(scheme)
    for d in range(nd):
        yield z2_source(dims, seed, noise, scheme, d if nd > 1 else -1)


def loops_point(U, dims, kappa, site, gammas, tol=1e-13, tap=1):
    """Exact L_Gamma(t) from the 12 unit sources at `site` ([n_gamma][T] complex).

    Only t = t(site) is non-zero; it equals Tr[Gamma M^-1(site, site)].
    """
    L = np.zeros((len(gammas), dims[3]), dtype=np.complex128)
    for al in range(4):
        for a in range(3):
            e = point_source(dims, site, al, a)
            s, _, _ = solve(U, e, dims, kappa, tol, tap=tap)
            L = loops_accumulate(dims, e, s, gammas, L)
    return L


def loops_z2(U, dims, kappa, seed, noises, scheme, gammas, tol=1e-13, tap=1, return_solutions=False):
    """Per-noise estimates L^(n)_Gamma(t) = sum_d eta_d^+ P_t Gamma M^-1 eta_d.

    Returns complex [len(noises)][n_gamma][T] (sums over dilution classes, not means).
    """
    out = np.zeros((len(noises), len(gammas), dims[3]), dtype=np.complex128)
    sols = []
    for k, n in enumerate(noises):
        for eta in _sources(dims, seed, n, scheme):
            s, _, _ = solve(U, eta, dims, kappa, tol, tap=tap)
            out[k] = loops_accumulate(dims, eta, s, gammas, out[k])
            if return_solutions:
                sols.append(s)
    return (out, sols) if return_solutions else out


def loops_lp(U, dims, kappa, seed, noises, scheme, gammas, niter=25, tap=1):
    """Per-noise estimates with the truncated low-precision solve (FP64 arithmetic)."""
    out = np.zeros((len(noises), len(gammas), dims[3]), dtype=np.complex128)
    for k, n in enumerate(noises):
        for eta in _sources(dims, seed, n, scheme):
            s = solve_lp(U, eta, dims, kappa, niter, tap=tap)
            out[k] = loops_accumulate(dims, eta, s, gammas, out[k])
    return out


def tsm_combine(lp_set_lp, hp_set_hp, hp_set_lp):
    """Truncated solver method estimate (Section 2):
    mean over the low-precision ensemble of its LP loops, plus the mean over the
    high-precision ensemble of (HP loop - LP loop of the same noise)."""
    return np.mean(lp_set_lp, axis=0) + np.mean(np.asarray(hp_set_hp) - np.asarray(hp_set_lp), axis=0)


# ---------------------------------------------------------------- derivatives


def loops_dkappa(U, dims, kappa, seed, noises, scheme, gammas, tol=1e-13, tap=1):
    """d/dkappa of the per-noise estimator: eta_d^+ P_t Gamma u_d, u_d = M^-1 D M^-1 eta_d."""
    out = np.zeros((len(noises), len(gammas), dims[3]), dtype=np.complex128)
    for k, n in enumerate(noises):
        for eta in _sources(dims, seed, n, scheme):
            s, _, _ = solve(U, eta, dims, kappa, tol, tap=tap)
            u, _, _ = solve(U, dhop(U, s, dims, tap), dims, kappa, tol, tap=tap)
            out[k] = loops_accumulate(dims, eta, u, gammas, out[k])
    return out


def link_grad(U, dims, kappa, sources, gammas, W, tol=1e-13, tap=1):
    """Gradient [4][V][3][3] of F = Re sum_{g,t} conj(W[g,t]) sum_src eta^+ P_t Gamma_g M^-1 eta
    with respect to the unconstrained complex links, in the dF = Re(conj(grad) dU) convention.

    The adjoint vector a = M^-dagger (sum W Gamma^+ P_t eta) is obtained by solving
    with M^dagger = gamma5 M gamma5: a = gamma5 M^-1 gamma5 (...).
    """
    U = _c128(U)
    V = int(np.prod(dims))
    gam = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    Wb = np.zeros((len(gam), dims[3], 2))
    Wb[..., 0], Wb[..., 1] = np.real(W), np.imag(W)
    grad = np.zeros((4, V, 3, 3, 2))
    d = _dims(dims)
    for eta in sources:
        eta = _c128(eta)
        s, _, _ = solve(U, eta, dims, kappa, tol, tap=tap)
        w = np.empty_like(eta)
        lib().or_weighted_gamma_dag(_ptr(d), _ptr(eta), len(gam), _ptr(gam), _ptr(Wb), _ptr(w))
        lib().or_gamma5(_ptr(d), _ptr(w))
        a, _, _ = solve(U, w, dims, kappa, tol, tap=tap)
        lib().or_gamma5(_ptr(d), _ptr(a))
        lib().or_link_grad_accumulate(_ptr(d), int(tap), float(kappa), _ptr(a), _ptr(s), _ptr(grad))
    return grad[..., 0] + 1j * grad[..., 1]


# ---------------------------------------------------------------- dense helpers


def dense_m(U, dims, kappa, tap=1, dag=False) -> np.ndarray:
    """The 12V x 12V matrix M, column by column from unit vectors (small lattices only)."""
    V = int(np.prod(dims))
    n = 12 * V
    Md = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[:] = 0
        flat[j] = 1
        Md[:, j] = apply_m(U, e, dims, kappa, tap, dag).reshape(-1)
    return Md


def dense_dhop(U, dims, tap=1) -> np.ndarray:
    V = int(np.prod(dims))
    n = 12 * V
    D = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[:] = 0
        flat[j] = 1
        D[:, j] = dhop(U, e, dims, tap).reshape(-1)
    return D


def exact_loops_dense(Minv: np.ndarray, dims, gammas) -> np.ndarray:
    """L_Gamma(t) = sum_{x in t} Tr[Gamma M^-1(x,x)] from a dense inverse ([n_gamma][T])."""
    V = int(np.prod(dims))
    T = dims[3]
    blocks = Minv.reshape(V, 12, V, 12)
    diag = np.stack([blocks[i, :, i, :] for i in range(V)])  # [V][12][12]
    diag = diag.reshape(V, 4, 3, 4, 3)
    sp = np.einsum("xaibi->xab", diag)  # colour trace -> [V][4][4] spin matrix
    tsite = np.arange(V) // (V // T)
    out = np.zeros((len(gammas), T), dtype=np.complex128)
    for k, g in enumerate(gammas):
        G = gamma(g)
        vals = np.einsum("ab,xba->x", G, sp)
        np.add.at(out[k], tsite, vals)
    return out


def disconnected_correlator(loops_b, loops_a, spatial_volume):
    """Disconnected two-loop correlator of Section 3, Eq. (2), at zero momentum:

        D(dt) = -1/(L^3 T) sum_t < L_B(t) L_A(t + dt) >,

    the two loops closing on themselves at t and t + dt (t + dt taken modulo T:
    the sum over t runs over the periodic time direction).  The gauge-field
    expectation is not taken here; the noise expectation of the product is
    estimated from per-noise loops over ordered pairs of distinct noises
    n != m only, since a product of two estimates on the same noise carries
    the noise's own fluctuation as a bias:

        < L_B(t) L_A(t') > ~ 1/(N (N-1)) sum_{n != m} L_B^n(t) L_A^m(t').

    loops_b, loops_a: complex [N][T] per-noise loops (N >= 2); returns complex [T]
    indexed by dt.  Written as the plain double sum over pairs.
    """
    lb = np.asarray(loops_b, dtype=np.complex128)
    la = np.asarray(loops_a, dtype=np.complex128)
    n, T = lb.shape
    if la.shape != (n, T) or n < 2:
        raise ValueError("need two [N][T] loop arrays with N >= 2")
    out = np.zeros(T, dtype=np.complex128)
    for dt in range(T):
        acc = 0j
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                for t in range(T):
                    acc += lb[i, t] * la[j, (t + dt) % T]
        out[dt] = -acc / (n * (n - 1)) / (spatial_volume * T)
    return out


def smear(U, psi, dims, alpha, iters) -> np.ndarray:
    """S psi = F^iters psi, F psi = [psi + alpha sum_i (U_i psi(x+i) + U_i(x-i)^+ psi(x-i))] / (1 + 6 alpha)."""
    out = np.empty_like(_c128(psi))
    lib().or_smear(_ptr(_dims(dims)), _ptr(_c128(U)), float(alpha), int(iters), _ptr(_c128(psi)), _ptr(out))
    return out


def loops_z2_smeared(U, dims, kappa, seed, noises, scheme, gammas, alpha, iters, tol=1e-13, tap=1):
    """Per-noise loops of smeared quark fields, L^S_Gamma(t) = sum_{x in t} Tr[Gamma (S M^-1 S)(x,x)],
    estimated as sum_d xi_d^+ P_t Gamma M^-1 xi_d with xi_d = S eta_d (S is hermitian and acts within
    timeslices and trivially on spin, so it moves from the sink onto the noise).  [len(noises)][n_gamma][T]."""
    out = np.zeros((len(noises), len(gammas), dims[3]), dtype=np.complex128)
    for k, n in enumerate(noises):
        for eta in _sources(dims, seed, n, scheme):
            xi = smear(U, eta, dims, alpha, iters)
            s, _, _ = solve(U, xi, dims, kappa, tol, tap=tap)
            out[k] = loops_accumulate(dims, xi, s, gammas, out[k])
    return out



def eta_prime_fit(d, c_pi, m_pi, tmin, tmax):
    """Section 3, Eqs. (3) and (4), on per-configuration correlators.

    Eq. (3): the eta' correlator is the connected pion correlator minus twice
    the disconnected one, C_eta'(t) = C_pi(t) - 2 D(t) (configuration mean).
    Eq. (4): for large t the ratio of the disconnected to the connected
    correlator behaves as

        R(t) = D(t) / C_pi(t) ~ A - B (e^{-m t} + e^{-m (T-t)}) / (e^{-m_pi t} + e^{-m_pi (T-t)}),

    with m the eta' mass and the pion mass inserted as a prior, leaving the
    three parameters (A, B, m).  R(t) is the ratio of the configuration sums;
    the fit minimises sum_t w_t (R - model)^2 on tmin <= t <= tmax, w_t = 1 /
    var R(t) from a jackknife over configurations (unit weights for one
    configuration or where a variance vanishes), m in [1e-3, 10].  Errors are
    jackknife errors, each leave-one-out sample refitted with the same weights.

    The fit is a full three-parameter nonlinear least squares
    (scipy.optimize.least_squares, trust-region reflective) from twelve
    starting masses, the start of (A, B) at each a linear least squares; the
    leave-one-out fits start from the full-sample minimum.
    d, c_pi: real [ncfg][T] (or [T]).  Returns (c_eta[T], params[3],
    errors[3], chi2).
    """
    from scipy.optimize import least_squares

    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    c = np.atleast_2d(np.asarray(c_pi, dtype=np.float64))
    ncfg, T = d.shape
    ts = np.arange(tmin, tmax + 1, dtype=np.float64)

    def g(m):
        return np.exp(-m * ts) + np.exp(-m * (T - ts))

    gpi = g(m_pi)
    c_eta = (c - 2.0 * d).mean(axis=0)

    def ratio(keep):
        return d[keep][:, tmin:tmax + 1].sum(axis=0) / c[keep][:, tmin:tmax + 1].sum(axis=0)

    R = ratio(np.arange(ncfg))
    jk = [ratio(np.array([n for n in range(ncfg) if n != k])) for k in range(ncfg)] if ncfg >= 2 else []
    w = np.ones_like(R)
    if ncfg >= 2:
        J = np.array(jk)
        var = (ncfg - 1) / ncfg * ((J - J.mean(axis=0)) ** 2).sum(axis=0)
        if np.all(var > 0):
            w = 1.0 / var
    sw = np.sqrt(w)

    def fit(y, starts):
        def resid(p):
            A, B, m = p
            return sw * (y - (A - B * g(m) / gpi))

        best = None
        for p0 in starts:
            r = least_squares(resid, p0, bounds=([-np.inf, -np.inf, 1e-3], [np.inf, np.inf, 10.0]),
                              xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
            c2 = float(np.sum(r.fun ** 2))
            if best is None or c2 < best[1]:
                best = (r.x.copy(), c2)
        return best

    starts = []
    for m0 in np.geomspace(2e-3, 5.0, 12):
        X = np.stack([np.ones_like(ts), -g(m0) / gpi], axis=1)
        ab0 = np.linalg.lstsq(X * sw[:, None], R * sw, rcond=None)[0]
        starts.append([ab0[0], ab0[1], m0])
    p, chi2 = fit(R, starts)
    err = np.zeros(3)
    if ncfg >= 2:
        # each leave-one-out sample starts from the full-sample minimum
        P = np.array([fit(y, [p])[0] for y in jk])
        err = np.sqrt((ncfg - 1) / ncfg * ((P - P.mean(axis=0)) ** 2).sum(axis=0))
    return c_eta, p, err, chi2
