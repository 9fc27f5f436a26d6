"""nyxrt: MI355X-native adaptive ray-tracing sweep of Nyx-RT (arXiv 2512.12466).

Thin Python binding of libnyxrt.so (C ABI in include/nyxrt.h).  It only
marshals arguments: PyTorch supplies device memory (the workspace, fields
and Gamma are torch tensors on the GPU) and the stream; every step of the
sweep runs in the library's HIP kernels.  The binding raises if the library
has not been built; there is no other code path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnyxrt.so")
MAX_LEVEL = 14

FP64, MIXED = 0, 1
CORR_NONE, CORR_LINEAR, CORR_CONSERVATIVE, CORR_SQUARED, CORR_NAIVE = range(5)
SPEC_MONO, SPEC_BLACKBODY, SPEC_POWERLAW = range(3)
STATUS = {0: "NRT_OK", 1: "NRT_ERR_ARG", 2: "NRT_ERR_STATE", 3: "NRT_ERR_NOMEM",
          4: "NRT_ERR_OVERFLOW", 5: "NRT_ERR_DEVICE", 6: "NRT_ERR_INTERNAL"}


class NyxRTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("h_cm", C.c_double), ("periodic", C.c_int32),
                ("sigma0", C.c_double), ("n_min_ray", C.c_double), ("l_max", C.c_int32),
                ("tau_max", C.c_double), ("n_th", C.c_double), ("corr", C.c_int32),
                ("precision", C.c_int32), ("spectrum", C.c_int32), ("spec_param", C.c_double)]


class MergeParams(C.Structure):
    _fields_ = [("dr", C.c_double), ("x_th", C.c_double), ("f_req", C.c_double),
                ("n_min", C.c_int32), ("r_max", C.c_double), ("f_ov", C.c_double),
                ("eps", C.c_double), ("shell_level", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("refill_min", C.c_int32), ("claim", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("graph", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Budget(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed", C.c_double),
                ("escaped", C.c_double), ("truncated", C.c_double),
                ("segments", C.c_uint64), ("rays", C.c_uint64), ("splits", C.c_uint64),
                ("rays_per_level", C.c_uint64 * (MAX_LEVEL + 1))]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "rays_per_level"}
        d["rays_per_level"] = list(self.rays_per_level)
        return d


_lib = None
_P = C.c_void_p
_D = C.POINTER(C.c_double)


def load():
    """Load libnyxrt.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -c "
                          "'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    sig = {
        "nrt_workspace_bytes": (st, [C.POINTER(GridDesc), C.c_int64, C.c_int64,
                                     C.POINTER(C.c_size_t)]),
        "nrt_init_grid": (st, [C.POINTER(_P), C.POINTER(GridDesc), _P, _P, C.c_int64,
                               C.c_int64, _P, C.c_size_t, _P]),
        "nrt_set_ionization": (st, [_P, _P]),
        "nrt_get_ionization": (st, [_P, _P]),
        "nrt_add_sources": (st, [_P, C.c_int64, _D, _D]),
        "nrt_clear_sources": (st, [_P]),
        "nrt_source_count": (st, [_P, C.POINTER(C.c_int64)]),
        "nrt_get_sources": (st, [_P, _D, _D, _D]),
        "nrt_merge_sources": (st, [_P, C.POINTER(MergeParams), C.POINTER(C.c_int64)]),
        "nrt_trace_step": (st, [_P, _P, C.POINTER(Budget)]),
        "nrt_trace_step_async": (st, [_P, _P, _P, _P]),
        "nrt_trace_step_noalloc": (st, [C.POINTER(GridDesc), _P, _P, C.c_int64, _D, _D,
                                        C.c_int64, _P, C.POINTER(Budget), _P]),
        "nrt_rt_step": (st, [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32, _P,
                             C.POINTER(Budget), C.POINTER(C.c_int32)]),
        "nrt_trace_rays_debug": (st, [_P, C.c_int64, _D, _D, C.POINTER(C.c_int32), _D, _P,
                                      C.POINTER(Budget)]),
        "nrt_healpix_dirs": (st, [_P, C.c_int32, C.c_int64, C.c_int64, _D]),
        "nrt_last_kernel_time": (st, [_P, _D, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "nrt_set_tuning": (st, [_P, C.POINTER(Tuning)]),
        "nrt_get_tuning": (st, [_P, C.POINTER(Tuning)]),
        "nrt_autotune": (st, [_P, _P, C.c_int32, C.POINTER(Tuning)]),
        "nrt_destroy": (st, [_P]),
        "nrt_status_str": (C.c_char_p, [C.c_int]),
        "nrt_last_error": (C.c_char_p, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status, ctx=None):
    if status != 0:
        msg = load().nrt_last_error(ctx)
        raise NyxRTError(status, msg.decode() if msg else "")


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _dp(a):
    return a.ctypes.data_as(_D)


def make_desc(n, h_cm, periodic=False, sigma0=6.30e-18, n_min_ray=4.0, l_max=10, tau_max=30.0,
              n_th=0.0, corr=CORR_CONSERVATIVE, precision=FP64, spectrum=SPEC_MONO,
              spec_param=0.0):
    return GridDesc(int(n), float(h_cm), int(bool(periodic)), float(sigma0), float(n_min_ray),
                    int(l_max), float(tau_max), float(n_th), int(corr), int(precision),
                    int(spectrum), float(spec_param))


def make_merge_params(dr=2.0, x_th=0.9, f_req=0.9, n_min=8, r_max=8.0, f_ov=1.0, eps=1e-6,
                      shell_level=3):
    return MergeParams(float(dr), float(x_th), float(f_req), int(n_min), float(r_max),
                       float(f_ov), float(eps), int(shell_level))


def budget_from_device(t):
    """The nrt_budget a device tensor holds (written by trace_step_async), as a dict."""
    raw = bytes(t.detach().cpu().contiguous().view(-1).numpy().view(np.uint8)[:C.sizeof(Budget)])
    return Budget.from_buffer_copy(raw).as_dict()


def workspace_bytes(desc, max_sources, ray_capacity):
    out = C.c_size_t(0)
    _check(load().nrt_workspace_bytes(C.byref(desc), int(max_sources), int(ray_capacity),
                                      C.byref(out)))
    return out.value


class Context:
    """One nrt_ctx: a grid, a source table and a caller-owned device workspace."""

    def __init__(self, desc, n_H, x, max_sources=1 << 16, ray_capacity=1 << 22, device=None,
                 stream=None):
        import torch
        L = load()
        self.desc = desc
        self.n = desc.n
        self.device = torch.device(device if device is not None else "cuda")
        shape = (desc.n,) * 3
        n_H = torch.as_tensor(n_H, dtype=torch.float64).reshape(shape)
        x = torch.as_tensor(x, dtype=torch.float64).reshape(shape)
        n_H = n_H.to(self.device).contiguous()
        x = x.to(self.device).contiguous()
        nbytes = workspace_bytes(desc, max_sources, ray_capacity)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = _P()
        with torch.cuda.device(self.device):
            _check(L.nrt_init_grid(C.byref(self._ctx), C.byref(desc), n_H.data_ptr(),
                                   x.data_ptr(), int(max_sources), int(ray_capacity),
                                   self._ws_ptr, nbytes, self.stream.cuda_stream))

    # -- fields --
    def set_ionization(self, x):
        import torch
        x = torch.as_tensor(x, dtype=torch.float64).reshape((self.n,) * 3)
        x = x.to(self.device).contiguous()
        _check(load().nrt_set_ionization(self._ctx, x.data_ptr()), self._ctx)

    def get_ionization(self):
        import torch
        out = torch.empty((self.n,) * 3, dtype=torch.float64, device=self.device)
        _check(load().nrt_get_ionization(self._ctx, out.data_ptr()), self._ctx)
        return out

    # -- sources --
    def add_sources(self, pos, ndot):
        pos = _f64(pos).reshape(-1, 3)
        ndot = _f64(ndot).reshape(-1)
        if pos.shape[0] != ndot.shape[0]:
            raise ValueError("pos and ndot disagree in length")
        _check(load().nrt_add_sources(self._ctx, pos.shape[0], _dp(pos), _dp(ndot)), self._ctx)

    def clear_sources(self):
        _check(load().nrt_clear_sources(self._ctx), self._ctx)

    def source_count(self):
        m = C.c_int64(0)
        _check(load().nrt_source_count(self._ctx, C.byref(m)), self._ctx)
        return m.value

    def get_sources(self):
        m = self.source_count()
        pos, ndot, rad = np.zeros((max(m, 1), 3)), np.zeros(max(m, 1)), np.zeros(max(m, 1))
        _check(load().nrt_get_sources(self._ctx, _dp(pos), _dp(ndot), _dp(rad)), self._ctx)
        return pos[:m], ndot[:m], rad[:m]

    def merge_sources(self, mp=None):
        mp = mp if mp is not None else make_merge_params()
        m = C.c_int64(0)
        _check(load().nrt_merge_sources(self._ctx, C.byref(mp), C.byref(m)), self._ctx)
        return m.value

    # -- tracing --
    def _gamma(self, gamma):
        import torch
        if gamma is None:
            gamma = torch.empty((self.n,) * 3, dtype=torch.float64, device=self.device)
        assert gamma.dtype == torch.float64 and gamma.is_contiguous()
        assert gamma.numel() == self.n ** 3 and gamma.device == self.device
        return gamma

    def trace_step(self, gamma=None):
        gamma = self._gamma(gamma)
        b = Budget()
        _check(load().nrt_trace_step(self._ctx, gamma.data_ptr(), C.byref(b)), self._ctx)
        return gamma, b.as_dict()

    def trace_step_async(self, gamma=None, budget=None, dropped=None):
        """nrt_trace_step_async: enqueue one pass on the context's stream and
        return at once (capture-safe).  budget / dropped: device tensors of
        sizeof(nrt_budget) bytes / one int64, allocated when None.  Returns
        (gamma, budget, dropped); decode the budget with budget_from_device()
        once the stream has finished."""
        import torch
        gamma = self._gamma(gamma)
        # empty, not zeros: a fill on torch's stream could land after the pass,
        # which writes every byte of both
        if budget is None:
            budget = torch.empty(C.sizeof(Budget), dtype=torch.uint8, device=self.device)
        if dropped is None:
            dropped = torch.empty(1, dtype=torch.int64, device=self.device)
        assert budget.numel() * budget.element_size() >= C.sizeof(Budget)
        assert budget.device == self.device and dropped.device == self.device
        _check(load().nrt_trace_step_async(self._ctx, gamma.data_ptr(), budget.data_ptr(),
                                           dropped.data_ptr()), self._ctx)
        return gamma, budget, dropped

    def rt_step(self, dt_s, alpha, tol=1e-6, max_iter=200, gamma=None, conv_frac=0.0):
        """nrt_rt_step: one radiation step; returns (gamma, budget, passes)."""
        gamma = self._gamma(gamma)
        b = Budget()
        it = C.c_int32(0)
        _check(load().nrt_rt_step(self._ctx, float(dt_s), float(alpha), float(tol),
                                  float(conv_frac), int(max_iter), gamma.data_ptr(), C.byref(b),
                                  C.byref(it)),
               self._ctx)
        return gamma, b.as_dict(), it.value

    def trace_rays_debug(self, origin, direction, level, L, gamma=None):
        origin = _f64(origin).reshape(-1, 3)
        direction = _f64(direction).reshape(-1, 3)
        k = origin.shape[0]
        level = np.ascontiguousarray(np.broadcast_to(level, (k,)), dtype=np.int32)
        L = _f64(np.broadcast_to(L, (k,)))
        gamma = self._gamma(gamma)
        b = Budget()
        _check(load().nrt_trace_rays_debug(self._ctx, k, _dp(origin), _dp(direction),
                                           level.ctypes.data_as(C.POINTER(C.c_int32)), _dp(L),
                                           gamma.data_ptr(), C.byref(b)), self._ctx)
        return gamma, b.as_dict()

    def healpix_dirs(self, level, first=0, count=None):
        count = 12 * 4 ** level - first if count is None else count
        out = np.zeros((max(count, 1), 3))
        _check(load().nrt_healpix_dirs(self._ctx, int(level), int(first), int(count),
                                       _dp(out)), self._ctx)
        return out[:count]

    def last_kernel_time(self):
        """(average march launch duration in ms, number of launches) of the
        last pass, from HIP events on the context's stream."""
        ms = C.c_double(0.0)
        n = C.c_int32(0)
        _check(load().nrt_last_kernel_time(self._ctx, C.byref(ms), C.byref(n), None), self._ctx)
        return ms.value, n.value

    def last_pass_was_graph(self):
        g = C.c_int32(0)
        _check(load().nrt_last_kernel_time(self._ctx, None, None, C.byref(g)), self._ctx)
        return bool(g.value)

    def set_tuning(self, refill_min=0, claim=0, blocks_per_cu=0, graph=0):
        """graph: 0 replay a captured pass once eligible, 1 never, 2 always try."""
        _check(load().nrt_set_tuning(self._ctx, C.byref(Tuning(refill_min, claim, blocks_per_cu,
                                                                graph))), self._ctx)

    def get_tuning(self):
        t = Tuning()
        _check(load().nrt_get_tuning(self._ctx, C.byref(t)), self._ctx)
        return t.as_dict()

    def autotune(self, passes=1, gamma=None):
        """nrt_autotune: time candidate launch parameters on this context's
        workload, keep and return the fastest."""
        gamma = self._gamma(gamma)
        t = Tuning()
        _check(load().nrt_autotune(self._ctx, gamma.data_ptr(), int(passes), C.byref(t)),
               self._ctx)
        return t.as_dict()

    def destroy(self):
        if getattr(self, "_ctx", None):
            load().nrt_destroy(self._ctx)  # synchronises the context's stream
            self._ctx = None
            self.workspace = None  # the device memory is free for the next context

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def trace_step_noalloc(desc, n_H, x, pos, ndot, gamma, ray_capacity, stream=None):
    """nrt_trace_step_noalloc: one monochromatic trace pass with no context
    and no allocation (the library's state lives in its static device
    scratch).  n_H, x, gamma: float64 CUDA tensors of n^3 elements on the
    current device; pos (m,3) and ndot (m,) host arrays.  Returns the budget
    dict; gamma is overwritten."""
    import torch
    for t in (n_H, x, gamma):
        assert t.dtype == torch.float64 and t.is_contiguous() and t.is_cuda
        assert t.numel() == desc.n ** 3
    pos = _f64(pos).reshape(-1, 3)
    ndot = _f64(ndot).reshape(-1)
    assert pos.shape[0] == ndot.shape[0]
    s = stream if stream is not None else torch.cuda.current_stream(gamma.device)
    b = Budget()
    _check(load().nrt_trace_step_noalloc(C.byref(desc), n_H.data_ptr(), x.data_ptr(),
                                         pos.shape[0], _dp(pos), _dp(ndot), int(ray_capacity),
                                         gamma.data_ptr(), C.byref(b), s.cuda_stream))
    return b.as_dict()


def init_grid(desc, n_H, x, **kw):
    """nrt_init_grid: create a Context (see Context for the keywords)."""
    return Context(desc, n_H, x, **kw)
