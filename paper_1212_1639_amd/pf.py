"""ctypes binding of libpf_mi355x.so (declared in include/pf.h).

Argument marshalling only: every step of the filter runs in the library's
HIP kernels.  torch provides device memory (the workspace and test buffers)
and the HIP stream.  There is no fallback: if the library is missing or no
GPU is visible the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libpf_mi355x.so")

LL_PF, LL_PL, SV_PF, SV_PL = 0, 1, 2, 3
MULTINOMIAL, STRATIFIED, SYSTEMATIC, SORTED_MULTINOMIAL = 0, 1, 2, 3
FP32, FP64 = 0, 1
SEARCH_AUTO, SEARCH_BINARY, SEARCH_CUTPOINT, SEARCH_MERGE = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EDEVICE, EDEGENERATE = 0, -1, -2, -3, -4
FLAG_KEEP_ANCESTORS = 1
FLAG_LOOKBACK_SCAN = 2
FLAG_TEST_SCAN_STALL = 4
N_MOMENTS = {LL_PF: 3, LL_PL: 6, SV_PF: 3, SV_PL: 7}
MODEL_NAMES = {"ll_pf": LL_PF, "ll_pl": LL_PL, "sv_pf": SV_PF, "sv_pl": SV_PL}

# every symbol include/pf.h declares
EXPORTS = ["pf_fields", "pf_workspace_bytes", "pf_create", "pf_step", "pf_loglik", "pf_moments",
           "pf_destroy", "pf_last_error", "pf_batch_create", "pf_batch_update", "pf_batch_step",
           "pf_batch_destroy", "pf_step_batch", "pf_debug_search", "pf_debug_particles",
           "pf_timing_start", "pf_timing_read", "pf_autotune", "pf_autotune_batch",
           "pf_copy_particles_async", "pf_checkpoint_bytes", "pf_checkpoint_save",
           "pf_checkpoint_restore", "pf_batch_bytes", "pf_debug_search_noalloc"]


class PFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pf error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("strategy", ctypes.c_int32),
        ("n_particles", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("items_per_thread", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("x0_mean", ctypes.c_double),
        ("x0_var", ctypes.c_double),
        ("sigma_v2", ctypes.c_double),
        ("sigma_w2", ctypes.c_double),
        ("a_v", ctypes.c_double),
        ("b_v", ctypes.c_double),
        ("a_w", ctypes.c_double),
        ("b_w", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("phi", ctypes.c_double),
        ("sigma2", ctypes.c_double),
        ("prior_mean", ctypes.c_double * 2),
        ("prior_prec", ctypes.c_double * 3),
        ("a_s", ctypes.c_double),
        ("d_s", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        cfgp = ctypes.POINTER(Config)
        L.pf_fields.argtypes = [i32]
        L.pf_fields.restype = ctypes.c_int
        L.pf_workspace_bytes.argtypes = [cfgp]
        L.pf_workspace_bytes.restype = ctypes.c_size_t
        L.pf_create.argtypes = [cfgp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.pf_step.argtypes = [vp, ctypes.POINTER(d), i64]
        L.pf_loglik.argtypes = [vp, ctypes.POINTER(d)]
        L.pf_moments.argtypes = [vp, ctypes.POINTER(d), i32]
        L.pf_destroy.argtypes = [vp]
        L.pf_last_error.restype = ctypes.c_char_p
        L.pf_debug_search.argtypes = [vp, vp, i64, i64, i32, vp, vp]
        L.pf_debug_search_noalloc.argtypes = [vp, vp, i64, i64, i32, vp, vp]
        L.pf_debug_particles.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(i64)]
        L.pf_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, ctypes.POINTER(vp)]
        L.pf_batch_update.argtypes = [vp, ctypes.POINTER(vp), i32]
        L.pf_batch_step.argtypes = [vp, ctypes.POINTER(d), i64]
        L.pf_batch_destroy.argtypes = [vp]
        L.pf_step_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(d)]
        L.pf_timing_start.argtypes = [vp, i64, i64]
        L.pf_copy_particles_async.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.pf_batch_bytes.argtypes = [i32, i32, i64]
        L.pf_batch_bytes.restype = ctypes.c_size_t
        L.pf_checkpoint_bytes.argtypes = [vp]
        L.pf_checkpoint_bytes.restype = ctypes.c_size_t
        L.pf_checkpoint_save.argtypes = [vp, vp, ctypes.c_size_t]
        L.pf_checkpoint_restore.argtypes = [vp, vp, ctypes.c_size_t]
        L.pf_autotune.argtypes = [cfgp, ctypes.POINTER(d), i64, vp, ctypes.POINTER(d)]
        L.pf_autotune_batch.argtypes = [cfgp, i32, ctypes.POINTER(d), i64, vp, ctypes.POINTER(d)]
        L.pf_timing_read.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i64)]
        for name in ("pf_create", "pf_step", "pf_loglik", "pf_moments", "pf_destroy",
                     "pf_batch_create", "pf_batch_update", "pf_batch_step", "pf_batch_destroy",
                     "pf_step_batch",
                     "pf_debug_search", "pf_debug_search_noalloc", "pf_debug_particles",
                     "pf_checkpoint_save",
                     "pf_checkpoint_restore"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise PFError(rc, lib().pf_last_error().decode())


def make_config(model, n, seed, scheme=MULTINOMIAL, precision=FP32, strategy=SEARCH_AUTO,
                items_per_thread=0, flags=0, **params):
    c = Config()
    c.model = MODEL_NAMES.get(model, model) if isinstance(model, str) else model
    c.scheme = scheme
    c.precision = precision
    c.strategy = strategy
    c.n_particles = int(n)
    c.seed = int(seed)
    c.items_per_thread = int(items_per_thread)
    c.flags = int(flags)
    for k, v in params.items():
        if k in ("prior_mean", "prior_prec"):
            arr = getattr(c, k)
            for i, vv in enumerate(v):
                arr[i] = float(vv)
        else:
            setattr(c, k, float(v))
    return c


def workspace_bytes(cfg):
    n = lib().pf_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise PFError(EINVAL, lib().pf_last_error().decode())
    return n


def autotune(cfg, y, stream=None):
    """Tune cfg's items_per_thread, strategy and scan flag in place by timing
    candidates over the host observations y; returns ms per step of the
    winner."""
    y = np.ascontiguousarray(y, dtype=np.float64).ravel()
    ms = ctypes.c_double()
    _check(lib().pf_autotune(ctypes.byref(cfg), y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             y.size, _stream_ptr(stream), ctypes.byref(ms)))
    return ms.value


def autotune_batch(cfgs, y, stream=None):
    """Tune the common items_per_thread and strategy of filters stepped as one
    batch; y is (n_obs, n_filters).  Updates cfgs in place; returns ms per
    step of the winner."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = len(cfgs)
    assert y.ndim == 2 and y.shape[1] == n
    arr = (Config * n)(*cfgs)
    ms = ctypes.c_double()
    _check(lib().pf_autotune_batch(arr, n, y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   y.shape[0], _stream_ptr(stream), ctypes.byref(ms)))
    for k in range(n):
        cfgs[k].items_per_thread = arr[k].items_per_thread
        cfgs[k].strategy = arr[k].strategy
    return ms.value


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Filter:
    """One filter: a handle plus a torch-owned device workspace."""

    def __init__(self, cfg, stream=None, device="cuda"):
        import torch
        self.cfg = cfg
        self.nbytes = workspace_bytes(cfg)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self._h = ctypes.c_void_p()
        _check(lib().pf_create(ctypes.byref(cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                               self.nbytes, _stream_ptr(stream), ctypes.byref(self._h)))

    def step(self, y):
        y = np.ascontiguousarray(np.atleast_1d(y), dtype=np.float64)
        _check(lib().pf_step(self._h, y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), y.size))

    def loglik(self):
        out = ctypes.c_double()
        _check(lib().pf_loglik(self._h, ctypes.byref(out)))
        return out.value

    def moments(self):
        k = N_MOMENTS[self.cfg.model]
        out = (ctypes.c_double * 8)()
        _check(lib().pf_moments(self._h, out, 8))
        return np.array(out[:k])

    def particles(self):
        """(record[F, N], ancestors[N], t) copied to the host."""
        n = self.cfg.n_particles
        F = lib().pf_fields(self.cfg.model)
        dt = np.float64 if self.cfg.precision == FP64 else np.float32
        rec_bytes = F * n * np.dtype(dt).itemsize
        buf = np.empty(rec_bytes + 4 * n, dtype=np.uint8)
        t = ctypes.c_int64()
        _check(lib().pf_debug_particles(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size,
                                        ctypes.byref(t)))
        rec = buf[:rec_bytes].view(dt).reshape(F, n).copy()
        anc = buf[rec_bytes:].view(np.int32).copy()
        return rec, anc, t.value

    def record_shape(self):
        """(fields, N) and numpy dtype of the particle record."""
        F = lib().pf_fields(self.cfg.model)
        dt = np.float64 if self.cfg.precision == FP64 else np.float32
        return (F, self.cfg.n_particles), dt

    def checkpoint(self):
        """Snapshot of the filter's whole state (host bytes, numpy uint8)."""
        nb = lib().pf_checkpoint_bytes(self._h)
        buf = np.empty(nb, dtype=np.uint8)
        _check(lib().pf_checkpoint_save(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        return buf

    def restore(self, snapshot):
        """Replace the filter's state by a snapshot of a filter with the same
        configuration (from checkpoint())."""
        buf = np.ascontiguousarray(snapshot, dtype=np.uint8)
        _check(lib().pf_checkpoint_restore(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))

    def copy_particles_async(self, host, copy_stream):
        """Queue a copy of the current particle record into `host` (a pinned
        CPU torch tensor of the record's shape and dtype) on `copy_stream`;
        the filter keeps stepping while it runs."""
        (F, n), dt = self.record_shape()
        assert host.is_pinned() and not host.is_cuda and host.numel() * host.element_size() >= F * n * np.dtype(dt).itemsize
        _check(lib().pf_copy_particles_async(self._h, ctypes.c_void_p(host.data_ptr()),
                                             host.numel() * host.element_size(),
                                             _stream_ptr(copy_stream)))

    def timing_start(self, max_launches, every=1):
        """Bracket one in `every` of the next cycle-kernel launches with
        events, at most `max_launches` of them."""
        _check(lib().pf_timing_start(self._h, int(max_launches), int(every)))

    def timing_read(self):
        """(summed milliseconds, launches) of the bracketed cycle kernels."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        _check(lib().pf_timing_read(self._h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def close(self):
        if self._h:
            _check(lib().pf_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Filters stepped together (one launch over all their tiles per step, graph-replayed)."""

    def __init__(self, filters, ring=64, capacity=0):
        self.filters = list(filters)
        arr = (ctypes.c_void_p * len(self.filters))(*[f._h.value for f in self.filters])
        self._h = ctypes.c_void_p()
        _check(lib().pf_batch_create(arr, len(self.filters), capacity, ring,
                                     ctypes.byref(self._h)))

    def update(self, filters):
        """Replace the members (filters may join at any stage or leave)."""
        self.filters = list(filters)
        arr = (ctypes.c_void_p * max(1, len(self.filters)))(
            *[f._h.value for f in self.filters])
        _check(lib().pf_batch_update(self._h, arr, len(self.filters)))

    def step(self, y):
        """y: (n_steps, n_filters) observations, or (n_filters,) for one step."""
        if not self.filters:
            return
        y = np.ascontiguousarray(y, dtype=np.float64)
        if y.ndim == 1:
            y = y[None, :]
        assert y.shape[1] == len(self.filters)
        _check(lib().pf_batch_step(self._h, y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   y.shape[0]))

    def close(self):
        if self._h:
            _check(lib().pf_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_search(cdf, u, strategy=SEARCH_MERGE, stream=None):
    """Ancestors min{k : cdf[k] >= u_j} (n-1 if none) for device tensors."""
    import torch
    assert cdf.dtype == torch.float64 and u.dtype == torch.float64 and cdf.is_cuda and u.is_cuda
    cdf = cdf.contiguous()
    u = u.contiguous()
    anc = torch.empty(u.numel(), dtype=torch.int32, device=cdf.device)
    _check(lib().pf_debug_search(ctypes.c_void_p(cdf.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                 cdf.numel(), u.numel(), strategy,
                                 ctypes.c_void_p(anc.data_ptr()), _stream_ptr(stream)))
    return anc
