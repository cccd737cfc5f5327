"""Python binding of ``libdloops.so``, the MI355X (gfx950) library for
disconnected quark loops with N_f = 2 Wilson fermions.

The binding only marshals arguments: every step of the computation runs in
the library's HIP kernels.  Torch supplies device memory and the stream.
Function names match the C ABI declared in ``include/dloops.h``; the classes
:class:`Lattice` and :class:`Gauge` own the library handles, and
:func:`apply`, :func:`solve` and :func:`loops` are tensor-level shorthands.

The library is built in-tree by :func:`paper_1012_5168_amd._build.build`.
Loading fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_HERE, "libdloops.so")

# ------------------------------------------------------------------ constants (dloops.h)
DL_OK, DL_EINVAL, DL_ENOMEM, DL_EHIP, DL_ENOCONV, DL_EBREAKDOWN, DL_ENAN, DL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
DL_F64, DL_F32, DL_F16, DL_BF16 = 0, 1, 2, 3
DL_OP_DHOP, DL_OP_M, DL_OP_MDAG, DL_OP_MHAT, DL_OP_MHATDAG, DL_OP_DHOPDAG = 0, 1, 2, 3, 4, 5
DL_BICGSTAB, DL_CGNR = 0, 1
DL_SRC_Z2, DL_SRC_POINT = 0, 1
DL_DIL_SPIN_COLOUR, DL_DIL_CUBIC, DL_DIL_EVEN_ODD = 1, 2, 4
DL_DIL_COLOUR, DL_DIL_SPIN, DL_DIL_SPIN_EVEN_ODD, DL_DIL_TIME = 8, 16, 32, 64

_STATUS = {
    DL_EINVAL: "DL_EINVAL",
    DL_ENOMEM: "DL_ENOMEM",
    DL_EHIP: "DL_EHIP",
    DL_ENOCONV: "DL_ENOCONV",
    DL_EBREAKDOWN: "DL_EBREAKDOWN",
    DL_ENAN: "DL_ENAN",
    DL_EUNSUPPORTED: "DL_EUNSUPPORTED",
}


class DLError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code


class dl_solve_params(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("fixed_iters", ctypes.c_int32),
        ("delta", ctypes.c_double),
        ("poll", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
    ]


class dl_solve_stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("reliable_updates", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("true_rel_residual", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


class dl_tsm(ctypes.Structure):
    _fields_ = [
        ("n_lp", ctypes.c_int32),
        ("n_hp", ctypes.c_int32),
        ("lp", dl_solve_params),
        ("hp", dl_solve_params),
    ]


class dl_sources(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("first_noise", ctypes.c_int64),
        ("n_noise", ctypes.c_int32),
        ("point_site", ctypes.c_int32),
    ]


_P = ctypes.c_void_p
_SIGNATURES = {
    "dl_last_error": (ctypes.c_char_p, []),
    "dl_version": (ctypes.c_char_p, []),
    "dl_lattice_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "dl_lattice_destroy": (None, [_P]),
    "dl_lattice_volume": (ctypes.c_int64, [_P]),
    "dl_gauge_create": (ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "dl_gauge_create_device": (ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "dl_gauge_destroy": (None, [_P]),
    "dl_apply": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int64, _P]),
    "dl_apply_noalloc": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int64,
                                        _P]),
    "dl_solve": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(dl_solve_params), _P, _P, ctypes.c_int64,
                                ctypes.POINTER(dl_solve_stats), _P]),
    "dl_loops": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(dl_sources), ctypes.POINTER(dl_solve_params), _P,
                                ctypes.c_int32, _P, ctypes.POINTER(dl_solve_stats), _P]),
    "dl_smear": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, _P, _P, ctypes.c_int64, _P]),
    "dl_loops_smeared": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(dl_sources), ctypes.c_double,
                                        ctypes.c_int32, ctypes.POINTER(dl_solve_params), _P, ctypes.c_int32, _P,
                                        ctypes.POINTER(dl_solve_stats), _P]),
    "dl_loops_tsm": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(dl_sources), ctypes.POINTER(dl_tsm), _P,
                                    ctypes.c_int32, _P, ctypes.POINTER(dl_solve_stats), _P]),
    "dl_loops_dkappa": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(dl_sources),
                                       ctypes.POINTER(dl_solve_params), _P, ctypes.c_int32, _P,
                                       ctypes.POINTER(dl_solve_stats), _P]),
    "dl_loops_link_grad": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(dl_sources),
                                          ctypes.POINTER(dl_solve_params), _P, ctypes.c_int32, _P, _P, _P, _P,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(dl_solve_stats), _P]),
    "dl_tsm_combine": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      _P, _P]),
    "dl_batch_loops": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, ctypes.POINTER(dl_solve_params), _P,
                                      ctypes.c_int32, _P, _P, _P]),
    "dl_sources_count": (ctypes.c_int64, [_P, ctypes.POINTER(dl_sources)]),
    "dl_sources_fill": (ctypes.c_int, [_P, ctypes.POINTER(dl_sources), ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "dl_disconnected_correlator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "dl_eta_prime_fit": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_int32, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "dl_cache_release": (ctypes.c_int, []),
    "dl_cache_set_limit": (ctypes.c_int, [ctypes.c_uint64]),
    "dl_cache_bytes": (ctypes.c_uint64, []),
    "dl_profile_enable": (ctypes.c_int, [ctypes.c_int32]),
    "dl_profile_config": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "dl_stream_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dl_profile_read": (ctypes.c_int64, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def load(path: str | None = None):
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIBRARY_PATH
    if not os.path.exists(path):
        raise RuntimeError("libdloops.so is not built (%s); run paper_1012_5168_amd._build.build()" % path)
    # torch ships its own HIP runtime under the same soname as the system's: loaded first, it is the one
    # the library binds to, so the process holds a single runtime (with the library loaded first, torch
    # would load a second one and the first would find no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(rc: int, allow=()):
    if rc != DL_OK and rc not in allow:
        raise DLError(rc, load().dl_last_error().decode())
    return rc


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _as_complex(buf):
    """A float64 [..., 2] (re, im) buffer read as complex128 [...] in place (no copy, no arithmetic)."""
    return buf.view(np.complex128)[..., 0]


def _as_pairs(z, shape=None):
    """complex values as a contiguous float64 [..., 2] (re, im) array (a reinterpretation of the bytes)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    if shape is not None:
        z = np.ascontiguousarray(np.broadcast_to(z, shape))
    return z.view(np.float64).reshape(z.shape + (2,))


# ------------------------------------------------------------------ same-name wrappers


def dl_last_error() -> str:
    return load().dl_last_error().decode()


def dl_version() -> str:
    return load().dl_version().decode()


def dl_lattice_create(dims, t_antiperiodic: int = 1):
    d = (ctypes.c_int32 * 4)(*[int(x) for x in dims])
    h = _P()
    _check(load().dl_lattice_create(d, int(t_antiperiodic), ctypes.byref(h)))
    return h


def dl_lattice_destroy(h):
    load().dl_lattice_destroy(h)


def dl_gauge_create(lat, links: np.ndarray, prec_mask: int, recon: int = 12, stream=None):
    links = np.ascontiguousarray(links, dtype=np.complex128)
    h = _P()
    _check(load().dl_gauge_create(lat, links.ctypes.data_as(_P), int(prec_mask), int(recon), _stream(stream),
                                  ctypes.byref(h)))
    return h


def dl_gauge_create_device(lat, links, prec_mask: int, recon: int = 12, stream=None):
    """links: a contiguous complex128 device tensor [4][V][3][3]."""
    h = _P()
    _check(load().dl_gauge_create_device(lat, _dptr(links), int(prec_mask), int(recon), _stream(stream),
                                         ctypes.byref(h)))
    return h


def dl_gauge_destroy(h):
    load().dl_gauge_destroy(h)


def dl_apply(gauge, kappa, op, prec, inp, out, nrhs, stream=None):
    _check(load().dl_apply(gauge, float(kappa), int(op), int(prec), _dptr(inp), _dptr(out), int(nrhs),
                           _stream(stream)))


def dl_apply_noalloc(gauge, kappa, op, prec, inp, out, nrhs, stream=None):
    """As dl_apply, with the library's static scratch instead of allocated workspaces (no synchronisation:
    out is complete when the stream reaches the end of the call's work)."""
    _check(load().dl_apply_noalloc(gauge, float(kappa), int(op), int(prec), _dptr(inp), _dptr(out), int(nrhs),
                                   _stream(stream)))


def dl_solve(gauge, kappa, params, b, x, nrhs, stats=None, stream=None):
    st = (dl_solve_stats * int(nrhs))() if stats is None else stats
    rc = load().dl_solve(gauge, float(kappa), ctypes.byref(params), _dptr(b), _dptr(x), int(nrhs), st,
                         _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc, st


def dl_loops(gauge, kappa, sources, params, gammas, loops_out: np.ndarray, stats=None, stream=None):
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    rc = load().dl_loops(gauge, float(kappa), ctypes.byref(sources), ctypes.byref(params), g.ctypes.data_as(_P),
                         len(g), loops_out.ctypes.data_as(_P), stats, _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc


def dl_smear(gauge, alpha, iters, inp, out, nrhs, stream=None):
    _check(load().dl_smear(gauge, float(alpha), int(iters), _dptr(inp), _dptr(out), int(nrhs), _stream(stream)))


def dl_loops_smeared(gauge, kappa, sources, alpha, iters, params, gammas, loops_out: np.ndarray, stats=None,
                     stream=None):
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    rc = load().dl_loops_smeared(gauge, float(kappa), ctypes.byref(sources), float(alpha), int(iters),
                                 ctypes.byref(params), g.ctypes.data_as(_P), len(g), loops_out.ctypes.data_as(_P),
                                 stats, _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc


def dl_loops_tsm(gauge, kappa, sources, tsm, gammas, loops_out: np.ndarray, stats=None, stream=None):
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    rc = load().dl_loops_tsm(gauge, float(kappa), ctypes.byref(sources), ctypes.byref(tsm), g.ctypes.data_as(_P),
                             len(g), loops_out.ctypes.data_as(_P), stats, _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc


def dl_loops_dkappa(gauge, kappa, sources, params, gammas, dloops_out: np.ndarray, stats=None, stream=None):
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    rc = load().dl_loops_dkappa(gauge, float(kappa), ctypes.byref(sources), ctypes.byref(params),
                                g.ctypes.data_as(_P), len(g), dloops_out.ctypes.data_as(_P), stats, _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc


def dl_loops_link_grad(gauge, kappa, sources, params, gammas, w: np.ndarray, grad_out,
                       loops_out: np.ndarray | None = None, dloops_out: np.ndarray | None = None,
                       dF_dkappa=None, stats=None, stream=None):
    """grad_out: a host float64 array [4][V][3][3][2] or a device tensor of the same bytes."""
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    w = np.ascontiguousarray(w, dtype=np.float64)
    ptr = lambda a: None if a is None else a.ctypes.data_as(_P)  # noqa: E731
    gp = grad_out.ctypes.data_as(_P) if isinstance(grad_out, np.ndarray) else _dptr(grad_out)
    rc = load().dl_loops_link_grad(gauge, float(kappa), ctypes.byref(sources), ctypes.byref(params),
                                   g.ctypes.data_as(_P), len(g), w.ctypes.data_as(_P), gp, ptr(loops_out),
                                   ptr(dloops_out), None if dF_dkappa is None else ctypes.byref(dF_dkappa), stats,
                                   _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc


def dl_tsm_combine(lp_set_lp, n_lp, hp_set_hp, hp_set_lp, n_hp, n_gamma, T, est, var=None):
    _check(load().dl_tsm_combine(lp_set_lp.ctypes.data_as(_P), int(n_lp), hp_set_hp.ctypes.data_as(_P),
                                 hp_set_lp.ctypes.data_as(_P), int(n_hp), int(n_gamma), int(T),
                                 est.ctypes.data_as(_P), None if var is None else var.ctypes.data_as(_P)))


def dl_batch_loops(gauges, kappas, sources, params, gammas, loops_out, stats=None, stream=None):
    n = len(gauges)
    gh = (_P * n)(*[g for g in gauges])
    ks = (ctypes.c_double * n)(*[float(k) for k in kappas])
    ss = (dl_sources * n)(*sources)
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.int32))
    lp = (_P * n)(*[a.ctypes.data_as(_P) for a in loops_out])
    sp = None if stats is None else (_P * n)(*[ctypes.cast(x, _P) for x in stats])
    rc = load().dl_batch_loops(n, gh, ks, ss, ctypes.byref(params), g.ctypes.data_as(_P), len(g), lp, sp,
                               _stream(stream))
    _check(rc, allow=(DL_ENOCONV,))
    return rc


def dl_sources_count(lat, sources) -> int:
    n = load().dl_sources_count(lat, ctypes.byref(sources))
    if n < 0:
        _check(int(n))
    return int(n)


def dl_sources_fill(lat, sources, first_rhs, nrhs, out, stream=None):
    _check(load().dl_sources_fill(lat, ctypes.byref(sources), int(first_rhs), int(nrhs), _dptr(out), _stream(stream)))


def dl_profile_enable(on: bool = True):
    load().dl_profile_enable(1 if on else 0)


def dl_disconnected_correlator(loops_b, loops_a, n_noise, T, spatial_volume, corr, stream=None):
    _check(load().dl_disconnected_correlator(loops_b.ctypes.data, loops_a.ctypes.data, int(n_noise), int(T),
                                             int(spatial_volume), corr.ctypes.data, _stream(stream)))


def disconnected_correlator(loops_b, loops_a, spatial_volume, stream=None):
    """D(dt) of two per-noise loop sets (complex [n_noise][T] each), over distinct noise pairs;
    returns complex [T]."""
    lb, la = _as_pairs(loops_b), _as_pairs(loops_a)
    if lb.shape != la.shape or lb.ndim != 3:
        raise ValueError("loops_b and loops_a must both be [n_noise][T] complex")
    n, T = lb.shape[0], lb.shape[1]
    out = np.zeros((T, 2), dtype=np.float64)
    dl_disconnected_correlator(lb, la, n, T, spatial_volume, out, stream)
    return _as_complex(out)


def dl_eta_prime_fit(d, c_pi, ncfg, T, m_pi, tmin, tmax, c_eta, params, errors):
    chi2 = ctypes.c_double()
    _check(load().dl_eta_prime_fit(d.ctypes.data, c_pi.ctypes.data, int(ncfg), int(T), float(m_pi), int(tmin),
                                   int(tmax), c_eta.ctypes.data, params.ctypes.data, errors.ctypes.data,
                                   ctypes.byref(chi2)))
    return chi2.value


def eta_prime_fit(d, c_pi, m_pi, tmin, tmax):
    """Eqs. 3-4 on per-configuration correlators d, c_pi (real [ncfg][T] or [T]): returns
    (c_eta[T], (A, B, m_eta'), jackknife errors, chi2)."""
    d = np.ascontiguousarray(np.atleast_2d(np.asarray(d, dtype=np.float64)))
    c = np.ascontiguousarray(np.atleast_2d(np.asarray(c_pi, dtype=np.float64)))
    if d.shape != c.shape:
        raise ValueError("d and c_pi must have the same shape")
    ncfg, T = d.shape
    c_eta = np.zeros(T)
    params, errors = np.zeros(3), np.zeros(3)
    chi2 = dl_eta_prime_fit(d, c, ncfg, T, m_pi, tmin, tmax, c_eta, params, errors)
    return c_eta, params, errors, chi2


def dl_cache_release():
    """Free the device buffers the library keeps for reuse."""
    _check(load().dl_cache_release())


def dl_cache_set_limit(nbytes: int):
    """Cap the bytes the library's device memory cache may hold (0 turns caching off)."""
    _check(load().dl_cache_set_limit(int(nbytes)))


def dl_cache_bytes() -> int:
    return int(load().dl_cache_bytes())


def dl_profile_config(kind: int):
    """(kernel, right-hand sides or wavefronts, sites per workgroup, grid cap or region blocks) of the
    last profiled hopping launch of that kind; all -1 if none."""
    cfg = (ctypes.c_int32 * 4)()
    _check(load().dl_profile_config(int(kind), cfg))
    return tuple(int(v) for v in cfg)


def stream_probe(src, dst, mode: int, reps: int = 5, stream=None) -> float:
    """Mean seconds of one pass of the library's streaming probe (dl_stream_probe): mode 0 copies
    src's bytes into dst, mode 1 reads them.  src and dst are device tensors; dst holds at least
    src's bytes (copy) or 128 KiB (read)."""
    nbytes = src.numel() * src.element_size()
    need = nbytes if mode == 0 else 131072
    if dst.numel() * dst.element_size() < need:
        raise DLError(DL_EINVAL, "stream_probe: dst too small")
    sec = ctypes.c_double()
    _check(load().dl_stream_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  ctypes.c_uint64(nbytes), int(mode), int(reps), _stream(stream), ctypes.byref(sec)))
    return sec.value


def dl_profile_read(kind: int):
    ms, by = ctypes.c_double(), ctypes.c_double()
    n = load().dl_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(by))
    return int(n), ms.value, by.value


# ------------------------------------------------------------------ handles and shorthands


def solve_params(solver=DL_BICGSTAB, prec=DL_F64, tol=1e-10, maxiter=1000, fixed_iters=0, delta=0.0, poll=0,
                 use_graph=False):
    return dl_solve_params(int(solver), int(prec), float(tol), int(maxiter), int(fixed_iters), float(delta), int(poll),
                           1 if use_graph else 0)


def z2_sources(seed, n_noise, first_noise=0, scheme=0):
    return dl_sources(DL_SRC_Z2, int(scheme), int(seed) & 0xFFFFFFFFFFFFFFFF, int(first_noise), int(n_noise), 0)


def point_sources(site):
    return dl_sources(DL_SRC_POINT, 0, 0, 0, 1, int(site))


class Lattice:
    def __init__(self, dims, t_antiperiodic=True):
        self.dims = tuple(int(d) for d in dims)
        self.h = dl_lattice_create(self.dims, 1 if t_antiperiodic else 0)
        self.V = int(load().dl_lattice_volume(self.h))

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            dl_lattice_destroy(self.h)
            self.h = None


class Gauge:
    """A gauge field resident on the device.  links: a host complex128 array [4][V][3][3], or a
    contiguous complex128 torch tensor of that shape on the GPU (uploaded without a host copy)."""

    def __init__(self, lattice: Lattice, links, precs=(DL_F64,), recon=12, stream=None):
        self.lattice = lattice
        mask = 0
        for p in precs:
            mask |= 1 << int(p)
        if isinstance(links, np.ndarray):
            self.h = dl_gauge_create(lattice.h, links, mask, recon, stream)
        else:
            if not links.is_contiguous():
                raise ValueError("device links must be a contiguous complex128 tensor [4][V][3][3]")
            self.h = dl_gauge_create_device(lattice.h, links, mask, recon, stream)

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            dl_gauge_destroy(self.h)
            self.h = None


def apply(gauge: Gauge, kappa: float, op: int, psi, prec=DL_F64):
    """op(psi) for a device complex128 tensor psi of shape [n][V][4][3] (or [V][4][3])."""
    import torch

    x = psi.contiguous()
    if x.dim() == 3:
        x = x.unsqueeze(0)
    out = torch.empty_like(x)
    dl_apply(gauge.h, kappa, op, prec, x, out, x.shape[0])
    return out.reshape(psi.shape)


def solve(gauge: Gauge, kappa: float, b, params=None):
    """Solve M x = b for a device complex128 tensor b [n][V][4][3]; returns (x, stats list)."""
    import torch

    params = params or solve_params()
    bb = b.contiguous()
    if bb.dim() == 3:
        bb = bb.unsqueeze(0)
    x = torch.empty_like(bb)
    _, st = dl_solve(gauge.h, kappa, params, bb, x, bb.shape[0])
    return x.reshape(b.shape), [(s.status, s.iters, s.reliable_updates, s.true_rel_residual) for s in st]


def smear(gauge: Gauge, alpha: float, iters: int, psi):
    """S psi (gauge-covariant Gaussian smearing, FP64) for a device complex128 tensor [n][V][4][3]."""
    import torch

    x = psi.contiguous()
    if x.dim() == 3:
        x = x.unsqueeze(0)
    out = torch.empty_like(x)
    dl_smear(gauge.h, alpha, iters, x, out, x.shape[0])
    return out.reshape(psi.shape)


def loops_smeared(gauge: Gauge, kappa: float, sources: dl_sources, alpha: float, iters: int, gammas, params=None,
                  stream=None):
    """Per-noise loops of smeared quark fields, complex [n_noise][n_gamma][T], and per-solve stats."""
    params = params or solve_params()
    T = gauge.lattice.dims[3]
    buf = np.zeros((int(sources.n_noise), len(gammas), T, 2), dtype=np.float64)
    st = (dl_solve_stats * dl_sources_count(gauge.lattice.h, sources))()
    dl_loops_smeared(gauge.h, kappa, sources, alpha, iters, params, gammas, buf, st, stream)
    return _as_complex(buf), _stats_list(st)


def loops(gauge: Gauge, kappa: float, sources: dl_sources, gammas, params=None, stream=None):
    """Per-noise loop estimates, complex [n_noise][n_gamma][T], and per-solve stats."""
    params = params or solve_params()
    T = gauge.lattice.dims[3]
    n = int(sources.n_noise)
    buf = np.zeros((n, len(gammas), T, 2), dtype=np.float64)
    nrhs = dl_sources_count(gauge.lattice.h, sources)
    st = (dl_solve_stats * nrhs)()
    dl_loops(gauge.h, kappa, sources, params, gammas, buf, st, stream)
    return _as_complex(buf), _stats_list(st)


def _stats_list(st):
    return [(s.status, s.iters, s.reliable_updates, s.true_rel_residual) for s in st]


def loops_tsm(gauge: Gauge, kappa: float, sources: dl_sources, n_lp: int, n_hp: int, gammas, lp_params, hp_params,
              stream=None):
    """Truncated solver method: returns (lp_set_lp, hp_set_hp, hp_set_lp, stats), each complex
    [n][n_gamma][T]; the estimate is mean(lp_set_lp) + mean(hp_set_hp - hp_set_lp)."""
    T = gauge.lattice.dims[3]
    buf = np.zeros((n_lp + 2 * n_hp, len(gammas), T, 2), dtype=np.float64)
    ncls = dl_sources_count(gauge.lattice.h, sources) // int(sources.n_noise)
    st = (dl_solve_stats * ((n_lp + 2 * n_hp) * ncls))()
    dl_loops_tsm(gauge.h, kappa, sources, dl_tsm(n_lp, n_hp, lp_params, hp_params), gammas, buf, st, stream)
    z = _as_complex(buf)
    return z[:n_lp], z[n_lp:n_lp + n_hp], z[n_lp + n_hp:], _stats_list(st)


def tsm_estimate(lp_set_lp, hp_set_hp, hp_set_lp):
    """The truncated solver method's estimate and its variance (library, FP64): complex
    [n_gamma][T] and real [n_gamma][T] from per-noise loops (complex [n][n_gamma][T])."""
    lp, hh, hl = _as_pairs(lp_set_lp), _as_pairs(hp_set_hp), _as_pairs(hp_set_lp)
    if lp.ndim != 4 or hh.shape != hl.shape or hh.shape[1:] != lp.shape[1:]:
        raise ValueError("tsm_estimate: expected per-noise loops [n][n_gamma][T] with matching shapes")
    n_gamma, T = lp.shape[1], lp.shape[2]
    est = np.zeros((n_gamma, T, 2), dtype=np.float64)
    var = np.zeros((n_gamma, T), dtype=np.float64)
    dl_tsm_combine(lp, lp.shape[0], hh, hl, hh.shape[0], n_gamma, T, est, var)
    return _as_complex(est), var


def loops_dkappa(gauge: Gauge, kappa: float, sources: dl_sources, gammas, params=None, stream=None):
    """d/dkappa of the per-noise loop estimates, complex [n_noise][n_gamma][T]."""
    params = params or solve_params()
    T = gauge.lattice.dims[3]
    buf = np.zeros((int(sources.n_noise), len(gammas), T, 2), dtype=np.float64)
    nrhs = dl_sources_count(gauge.lattice.h, sources)
    st = (dl_solve_stats * (2 * nrhs))()
    dl_loops_dkappa(gauge.h, kappa, sources, params, gammas, buf, st, stream)
    return _as_complex(buf), _stats_list(st)


def loops_link_grad(gauge: Gauge, kappa: float, sources: dl_sources, gammas, w, params=None, with_dkappa=False,
                    stream=None, grad_out=None):
    """Gradient of F = Re sum conj(w[n][g][t]) L[n][g][t] with respect to the links, complex [4][V][3][3]
    (dF = Re sum conj(grad) dU); w is [n_noise][n_gamma][T] (or [n_gamma][T], the same for every
    noise).  grad_out: None (a page-locked host array is returned) or a complex128 device tensor
    [4][V][3][3] that receives the gradient.  Returns (grad, loops, dloops or None, dF/dkappa or None,
    stats); with_dkappa adds the kappa derivative (a third solve per right-hand side)."""
    params = params or solve_params()
    T = gauge.lattice.dims[3]
    V = gauge.lattice.V
    n = int(sources.n_noise)
    wb = _as_pairs(np.reshape(np.asarray(w, dtype=np.complex128), (-1, len(gammas), T)), (n, len(gammas), T))
    grad = _pinned_host((4, V, 3, 3, 2)) if grad_out is None else grad_out
    loops = np.zeros((n, len(gammas), T, 2), dtype=np.float64)
    dk = np.zeros((n, len(gammas), T, 2), dtype=np.float64) if with_dkappa else None
    dfk = ctypes.c_double() if with_dkappa else None
    nrhs = dl_sources_count(gauge.lattice.h, sources)
    st = (dl_solve_stats * (3 * nrhs))()
    dl_loops_link_grad(gauge.h, kappa, sources, params, gammas, wb, grad, loops, dk, dfk, st, stream)
    g = _as_complex(grad) if grad_out is None else grad_out
    return (g, _as_complex(loops), None if dk is None else _as_complex(dk), None if dfk is None else dfk.value,
            _stats_list(st))


def _pinned_host(shape):
    """An FP64 host array in page-locked memory (allocated as such, never registered after the fact):
    the library's device-to-host copy into it is a direct transfer, without staging or first-touch
    page faults.  The array keeps its torch storage alive."""
    import torch

    return torch.empty(shape, dtype=torch.float64, pin_memory=True).numpy()


def batch_loops(gauges, kappas, sources, gammas, params=None, stream=None):
    """Loop estimates on several lattices in one batched solve; returns lists of per-lattice
    complex [n_noise][n_gamma][T] loops and stats."""
    params = params or solve_params()
    outs, stats = [], []
    for G, src in zip(gauges, sources):
        T = G.lattice.dims[3]
        outs.append(np.zeros((int(src.n_noise), len(gammas), T, 2), dtype=np.float64))
        stats.append((dl_solve_stats * dl_sources_count(G.lattice.h, src))())
    dl_batch_loops([G.h for G in gauges], kappas, sources, params, gammas, outs, stats, stream)
    return [_as_complex(o) for o in outs], [_stats_list(s) for s in stats]
