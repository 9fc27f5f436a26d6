"""Oracle for the Nyx-RT adaptive ray-tracing sweep -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 CPU implementation written from the paper (arXiv
2512.12466); see oracle.h for the passage each function follows and the
readings taken where the paper is silent.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It shares no
code with the GPU library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

CORR_NONE, CORR_LINEAR, CORR_CONSERVATIVE, CORR_SQUARED, CORR_NAIVE = range(5)
SPEC_MONO, SPEC_BLACKBODY, SPEC_POWERLAW = range(3)
MAX_LEVEL = 24


class Params(C.Structure):
    _fields_ = [("n", C.c_int32), ("h_cm", C.c_double), ("periodic", C.c_int32),
                ("sigma0", C.c_double), ("n_min_ray", C.c_double), ("l_max", C.c_int32),
                ("tau_max", C.c_double), ("n_th", C.c_double), ("corr", C.c_int32),
                ("spectrum", C.c_int32), ("spec_param", C.c_double)]


class Budget(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed", C.c_double),
                ("escaped", C.c_double), ("truncated", C.c_double),
                ("segments", C.c_uint64), ("rays", C.c_uint64), ("splits", C.c_uint64),
                ("rays_per_level", C.c_uint64 * (MAX_LEVEL + 1))]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "rays_per_level"}
        d["rays_per_level"] = list(self.rays_per_level)
        return d


class MergeParams(C.Structure):
    _fields_ = [("dr", C.c_double), ("x_th", C.c_double), ("f_req", C.c_double),
                ("n_min", C.c_int32), ("r_max", C.c_double), ("f_ov", C.c_double),
                ("eps", C.c_double), ("shell_level", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        L.orc_pix2vec_nest.argtypes = [C.c_int, C.c_uint64, dp]
        L.orc_trace.argtypes = [C.POINTER(Params), dp, dp, C.c_int64, dp, dp, C.c_int, dp,
                                C.POINTER(Budget)]
        L.orc_trace_rays.argtypes = [C.POINTER(Params), dp, dp, C.c_int64, dp, dp, ip, dp,
                                     dp, C.POINTER(Budget), C.c_int64, lp, dp, lp, lp]
        L.orc_spectrum_eval.argtypes = [C.c_int32, C.c_double, C.c_int64, dp, dp, dp, dp, dp]
        L.orc_dedupe_sort.argtypes = [C.c_int32, C.c_int64, dp, dp, ip, dp]
        L.orc_dedupe_sort.restype = C.c_int64
        L.orc_max_radius.argtypes = [C.POINTER(MergeParams), C.c_int32, C.c_int32, dp,
                                     C.c_int64, ip, dp]
        L.orc_merge_sources.argtypes = [C.POINTER(MergeParams), C.c_int32, C.c_int32, dp,
                                        C.c_int64, dp, dp, ip, dp, dp]
        L.orc_merge_sources.restype = C.c_int64
        L.orc_chem_update.argtypes = [C.c_int64, dp, dp, dp, C.c_double, C.c_double, dp, dp,
                                      dp]
        L.orc_rt_step.argtypes = [C.POINTER(Params), dp, dp, C.c_int64, dp, dp, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, dp,
                                  C.POINTER(Budget), C.POINTER(C.c_int)]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_params(n, h_cm, periodic=False, sigma0=6.30e-18, n_min_ray=4.0, l_max=10,
                tau_max=30.0, n_th=0.0, corr=CORR_CONSERVATIVE, spectrum=SPEC_MONO,
                spec_param=0.0):
    return Params(int(n), float(h_cm), int(bool(periodic)), float(sigma0), float(n_min_ray),
                  int(l_max), float(tau_max), float(n_th), int(corr), int(spectrum),
                  float(spec_param))


def spectrum_eval(kind, param, tau, dtau=None):
    """Frequency integrals of Eq. lut_eqn per unit photon rate at threshold
    optical depths tau (cell depths dtau): returns (F, D, G) arrays."""
    tau = _f64(tau).reshape(-1)
    dt = np.zeros_like(tau) if dtau is None else _f64(np.broadcast_to(dtau, tau.shape))
    F, D, G = np.zeros_like(tau), np.zeros_like(tau), np.zeros_like(tau)
    if lib().orc_spectrum_eval(int(kind), float(param), tau.size, _d(tau), _d(dt), _d(F),
                               _d(D), _d(G)):
        raise ValueError(f"bad spectrum ({kind}, {param})")
    return F, D, G


def pix2vec_nest(level, pix):
    out = np.zeros(3)
    lib().orc_pix2vec_nest(int(level), int(pix), _d(out))
    return out


def healpix_dirs(level):
    """All 12*4^level nested pixel-centre unit vectors, shape (npix, 3)."""
    npix = 12 * 4 ** level
    out = np.zeros((npix, 3))
    L = lib()
    for p in range(npix):
        L.orc_pix2vec_nest(int(level), p, _d(out[p]))
    return out


def trace(params, n_H, x, pos, ndot, nthreads=None):
    """One trace pass.  n_H, x: (n,n,n) arrays indexed [k,j,i].  Returns
    (gamma (n,n,n), budget dict)."""
    n = params.n
    n_H = _f64(n_H, (n, n, n))
    x = _f64(x, (n, n, n))
    pos = _f64(pos).reshape(-1, 3)
    ndot = _f64(ndot).reshape(-1)
    assert pos.shape[0] == ndot.shape[0]
    gamma = np.zeros((n, n, n))
    b = Budget()
    nt = nthreads or max(1, min(16, os.cpu_count() or 1))
    rc = lib().orc_trace(C.byref(params), _d(n_H), _d(x), pos.shape[0], _d(pos), _d(ndot),
                         int(nt), _d(gamma), C.byref(b))
    if rc:
        raise ValueError(f"orc_trace failed ({rc})")
    return gamma, b.as_dict()


def trace_rays(params, n_H, x, origin, direction, level, L, max_log=0):
    """Injected rays (no splitting).  Returns (gamma, budget, log) where log
    is a dict of per-segment arrays (cell, ds, ijk) when max_log > 0."""
    n = params.n
    n_H = _f64(n_H, (n, n, n))
    x = _f64(x, (n, n, n))
    origin = _f64(origin).reshape(-1, 3)
    direction = _f64(direction).reshape(-1, 3)
    k = origin.shape[0]
    level = np.ascontiguousarray(np.broadcast_to(level, (k,)), dtype=np.int32)
    L = _f64(np.broadcast_to(L, (k,)))
    gamma = np.zeros((n, n, n))
    b = Budget()
    cell = np.zeros(max(max_log, 1), dtype=np.int64)
    ds = np.zeros(max(max_log, 1))
    ijk = np.zeros((max(max_log, 1), 3), dtype=np.int64)
    nlog = np.zeros(1, dtype=np.int64)
    rc = lib().orc_trace_rays(C.byref(params), _d(n_H), _d(x), k, _d(origin), _d(direction),
                              _i(level), _d(L), _d(gamma), C.byref(b), int(max_log),
                              _l(cell) if max_log else None, _d(ds) if max_log else None,
                              _l(ijk) if max_log else None, _l(nlog))
    if rc:
        raise ValueError(f"orc_trace_rays failed ({rc})")
    m = int(min(nlog[0], max_log))
    log = {"cell": cell[:m], "ds": ds[:m], "ijk": ijk[:m], "count": int(nlog[0])}
    return gamma, b.as_dict(), log


def make_merge_params(dr=2.0, x_th=0.9, f_req=0.9, n_min=8, r_max=8.0, f_ov=1.0, eps=1e-6,
                      shell_level=3):
    return MergeParams(float(dr), float(x_th), float(f_req), int(n_min), float(r_max),
                       float(f_ov), float(eps), int(shell_level))


def dedupe_sort(n, pos, ndot):
    pos = _f64(pos).reshape(-1, 3)
    ndot = _f64(ndot).reshape(-1)
    m = pos.shape[0]
    cells = np.zeros((max(m, 1), 3), dtype=np.int32)
    flux = np.zeros(max(m, 1))
    r = lib().orc_dedupe_sort(int(n), m, _d(pos), _d(ndot), _i(cells), _d(flux))
    if r < 0:
        raise ValueError(f"orc_dedupe_sort failed ({r})")
    return cells[:r].copy(), flux[:r].copy()


def max_radius(mp, n, periodic, x, cells):
    x = _f64(x, (n, n, n))
    cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(max(cells.shape[0], 1))
    rc = lib().orc_max_radius(C.byref(mp), int(n), int(bool(periodic)), _d(x),
                              cells.shape[0], _i(cells), _d(out))
    if rc:
        raise ValueError(f"orc_max_radius failed ({rc})")
    return out[:cells.shape[0]].copy()


def merge_sources(mp, n, periodic, x, pos, ndot):
    """Returns (cells (m',3) int32, flux (m'), radius (m'))."""
    x = _f64(x, (n, n, n))
    pos = _f64(pos).reshape(-1, 3)
    ndot = _f64(ndot).reshape(-1)
    m = pos.shape[0]
    cells = np.zeros((max(m, 1), 3), dtype=np.int32)
    flux = np.zeros(max(m, 1))
    rad = np.zeros(max(m, 1))
    r = lib().orc_merge_sources(C.byref(mp), int(n), int(bool(periodic)), _d(x), m, _d(pos),
                                _d(ndot), _i(cells), _d(flux), _d(rad))
    if r < 0:
        raise ValueError(f"orc_merge_sources failed ({r})")
    return cells[:r].copy(), flux[:r].copy(), rad[:r].copy()


def chem_update(gamma, n_H, x0, dt, alpha, x_avg_guess=None):
    gamma = _f64(gamma)
    shape = gamma.shape
    gamma = gamma.reshape(-1)
    n_H = _f64(n_H).reshape(-1)
    x0 = _f64(x0).reshape(-1)
    guess = x0.copy() if x_avg_guess is None else _f64(x_avg_guess).reshape(-1)
    xn = np.zeros_like(x0)
    xa = np.zeros_like(x0)
    lib().orc_chem_update(gamma.size, _d(gamma), _d(n_H), _d(x0), float(dt), float(alpha),
                          _d(guess), _d(xn), _d(xa))
    return xn.reshape(shape), xa.reshape(shape)


def rt_step(params, n_H, x, pos, ndot, dt, alpha, tol=1e-6, max_iter=200, nthreads=None,
            conv_frac=0.0):
    """One radiation step.  Returns (x_new, gamma, budget, iterations).  The
    iteration stops once at most conv_frac of the cells moved their step
    average by tol or more (0: none did)."""
    n = params.n
    n_H = _f64(n_H, (n, n, n))
    x = _f64(x, (n, n, n)).copy()
    pos = _f64(pos).reshape(-1, 3)
    ndot = _f64(ndot).reshape(-1)
    gamma = np.zeros((n, n, n))
    b = Budget()
    it = C.c_int(0)
    nt = nthreads or max(1, min(16, os.cpu_count() or 1))
    rc = lib().orc_rt_step(C.byref(params), _d(n_H), _d(x), pos.shape[0], _d(pos), _d(ndot),
                           float(dt), float(alpha), float(tol), float(conv_frac), int(max_iter),
                           int(nt),
                           _d(gamma), C.byref(b), C.byref(it))
    if rc:
        raise ValueError(f"orc_rt_step failed ({rc})")
    return x, gamma, b.as_dict(), it.value
