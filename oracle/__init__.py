"""CPU FP64 oracle for the particle-filter / particle-learning cycle.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package; the
product library never calls it, and it never imports the product package.
It shares no code with the HIP path (see ``pf_oracle.c`` for what each
function follows in McAlinn & Nakatsuma, arXiv:1212.1639).

Parity status of each function (what pins it is in ``tests/test_oracle_*``):
  philox / samplers ........ pinned (rocRAND's engine, KS tests vs scipy)
  CDF / search / cut-point . pinned (Table 1, brute force, closed forms)
  resampling schemes ....... pinned (offspring invariants, exact N<=8 laws,
                             unbiasedness over seeds)
  LL-PF .................... pinned (Kalman filter closed form)
  LL-PL .................... pinned (known-theta limit = Kalman filter;
                             2-D quadrature x Kalman filter; path sums)
  SV-PF .................... pinned (1-D grid filter)
  SV-PL .................... pinned (statistics against least squares on
                             the tracked path; known-parameter limit = 1-D
                             grid filter; unknown parameters: quadrature
                             over (alpha, beta, sigma^2) x grid filters)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LL_PF, LL_PL, SV_PF, SV_PL = 0, 1, 2, 3
MULTINOMIAL, STRATIFIED, SYSTEMATIC, SORTED_MULTINOMIAL = 0, 1, 2, 3
SEARCH_BINARY, SEARCH_CUTPOINT, SEARCH_BRUTE = 0, 1, 2
NMOM = 8
FIELDS = {LL_PF: 1, LL_PL: 5, SV_PF: 1, SV_PL: 7}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math: IEEE round-to-nearest)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
             "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Config(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("search", ctypes.c_int32),
        ("fp32_words", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
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
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.POINTER(ctypes.c_int64)
        u32 = ctypes.POINTER(ctypes.c_uint32)
        _lib.or_philox.argtypes = [u32, u32, u32]
        _lib.or_u32.argtypes = [ctypes.c_uint32]
        _lib.or_u32.restype = ctypes.c_double
        _lib.or_u24.argtypes = [ctypes.c_uint32]
        _lib.or_u24.restype = ctypes.c_double
        _lib.or_box_muller.argtypes = [ctypes.c_double, ctypes.c_double, d]
        _lib.or_gamma_mt.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_int]
        _lib.or_gamma_mt.restype = ctypes.c_double
        _lib.or_cdf.argtypes = [d, ctypes.c_int64, d, d, d]
        _lib.or_search_brute.argtypes = [d, ctypes.c_int64, ctypes.c_double]
        _lib.or_search_brute.restype = ctypes.c_int64
        _lib.or_search_binary.argtypes = [d, ctypes.c_int64, ctypes.c_double]
        _lib.or_search_binary.restype = ctypes.c_int64
        _lib.or_cutpoint_table.argtypes = [d, ctypes.c_int64, i64, i64]
        _lib.or_cutpoint_draw.argtypes = [d, i64, ctypes.c_int64, ctypes.c_double, i64]
        _lib.or_cutpoint_draw.restype = ctypes.c_int64
        _lib.or_resample.argtypes = [d, ctypes.c_int64, d, ctypes.c_int64, ctypes.c_int, i64]
        _lib.or_uniforms.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_int64, d]
        _lib.or_run.argtypes = [ctypes.POINTER(Config), d, ctypes.c_int64, d, d, i64, d, d]
        _lib.or_run.restype = ctypes.c_int
        _lib.or_run_from.argtypes = [ctypes.POINTER(Config), d, ctypes.c_int64, ctypes.c_double,
                                     d, ctypes.c_int64, d, d, i64, d, d]
        _lib.or_run_from.restype = ctypes.c_int
        _lib.or_run_given.argtypes = [ctypes.POINTER(Config), d, ctypes.c_int64, ctypes.c_double,
                                      d, ctypes.c_int64, i64, d, d, i64, d, d]
        _lib.or_run_given.restype = ctypes.c_int
        _lib.or_fields.argtypes = [ctypes.c_int]
        _lib.or_fields.restype = ctypes.c_int
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


# ---------------------------------------------------------------- random words
def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter under a 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox(c, k, o)
    return [int(o[i]) for i in range(4)]


def u32(w):
    return lib().or_u32(w)


def u24(w):
    return lib().or_u24(w)


def box_muller(u1, u2):
    z = (ctypes.c_double * 2)()
    lib().or_box_muller(u1, u2, z)
    return z[0], z[1]


def gamma_mt(a, z0, u0, seed=0, j=0, t=0, g=0, fp32=False):
    return lib().or_gamma_mt(a, z0, u0, seed, j, t, g, int(fp32))


# ---------------------------------------------------------------- resampling
def cdf(logw):
    """Resampling CDF (equation resample.cdf) of log-weights; returns (q, M, S)."""
    logw = np.ascontiguousarray(logw, dtype=np.float64)
    q = np.empty_like(logw)
    M = ctypes.c_double()
    S = ctypes.c_double()
    lib().or_cdf(_dp(logw), logw.size, _dp(q), ctypes.byref(M), ctypes.byref(S))
    return q, M.value, S.value


def search(q, u, method=SEARCH_BINARY):
    """Ancestors (0-based) for uniforms u against CDF q by the given method."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    anc = np.empty(u.size, dtype=np.int64)
    lib().or_resample(_dp(q), q.size, _dp(u), u.size, method, _ip(anc))
    return anc


def cutpoint_table(q):
    """(L, I) of the parallel cut-point search; I holds 0-based indices."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    L = np.empty(q.size, dtype=np.int64)
    I = np.empty(q.size, dtype=np.int64)
    lib().or_cutpoint_table(_dp(q), q.size, _ip(L), _ip(I))
    return L, I


def cutpoint_draw(q, I, u):
    """(ancestor, number of climbs) of one cut-point draw."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    I = np.ascontiguousarray(I, dtype=np.int64)
    c = ctypes.c_int64()
    k = lib().or_cutpoint_draw(_dp(q), _ip(I), q.size, float(u), ctypes.byref(c))
    return k, c.value


def uniforms(scheme, seed, t, n):
    u = np.empty(n, dtype=np.float64)
    lib().or_uniforms(scheme, seed, t, n, _dp(u))
    return u


# ---------------------------------------------------------------- filters
def make_config(model, n, seed, scheme=MULTINOMIAL, search=SEARCH_BINARY, fp32_words=False,
                **params):
    c = Config()
    c.model = model
    c.scheme = scheme
    c.search = search
    c.fp32_words = int(fp32_words)
    c.n = int(n)
    c.seed = int(seed)
    for k, v in params.items():
        if k in ("prior_mean", "prior_prec"):
            arr = getattr(c, k)
            for i, vv in enumerate(v):
                arr[i] = float(vv)
        else:
            setattr(c, k, float(v))
    return c


def run(cfg, y, dump=False, state0=None, t0=0, y_prev=0.0, anc_first=None):
    """Run the oracle filter over observations y.

    With ``state0`` (fields x N, the model's oracle fields) the run starts
    from those particles as the state after step ``t0`` and ``y`` holds the
    observations of steps t0+1, ...; ``y_prev`` is y_{t0} (the weights of
    the first resampling of the models that weight after propagating).
    With ``anc_first`` (N 0-based indices) the first step's resampling is
    replaced by those ancestors; everything else is computed as usual.
    Returns a dict with ``loglik`` (T,), ``moments`` (T, NMOM) and, when
    ``dump`` is set, ``anc`` (T, N), ``state`` (T, F, N) and ``logw`` (T, N).
    """
    y = np.ascontiguousarray(y, dtype=np.float64)
    T = y.size
    N = cfg.n
    F = FIELDS[cfg.model]
    ll = np.zeros(T)
    mom = np.zeros((T, NMOM))
    anc = state = logw = None
    if dump:
        anc = np.zeros((T, N), dtype=np.int64)
        state = np.zeros((T, F, N))
        logw = np.zeros((T, N))
    s0 = None
    if state0 is not None:
        s0 = np.ascontiguousarray(state0, dtype=np.float64).reshape(F, N)
    a0 = None
    if anc_first is not None:
        a0 = np.ascontiguousarray(anc_first, dtype=np.int64)
        assert a0.size == N
    rc = lib().or_run_given(ctypes.byref(cfg), _dp(s0) if s0 is not None else None, int(t0),
                            float(y_prev), _dp(y), T, _ip(a0) if a0 is not None else None,
                            _dp(ll), _dp(mom), _ip(anc) if dump else None,
                            _dp(state) if dump else None, _dp(logw) if dump else None)
    out = {"rc": rc, "loglik": ll, "moments": mom}
    if dump:
        out.update(anc=anc, state=state, logw=logw)
    return out


def sv_posterior(cfg, sums):
    """(L00, L01, L11, m_alpha, m_beta, a, d) from the raw path sums."""
    s = np.ascontiguousarray(sums, dtype=np.float64)
    out = np.empty(7)
    L = lib()
    L.or_sv_posterior.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    L.or_sv_posterior(ctypes.byref(cfg), _dp(s), _dp(out))
    return out


def sv_theta(post, z_g, u_g, z3, z4, seed=0, j=0, t=0, fp32=False):
    """One (alpha, beta, sigma^2) draw from a posterior of ``sv_posterior``."""
    p = np.ascontiguousarray(post, dtype=np.float64)
    th = np.empty(3)
    L = lib()
    L.or_sv_theta.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.or_sv_theta(_dp(p), z_g, u_g, z3, z4, seed, j, t, int(fp32), _dp(th))
    return th


def step_slots(cfg, state0, t0, y_prev, y, slots):
    """One step t0 + 1 from the particles ``state0`` (fields x N, after t0
    steps) for the output slots ``slots`` only: returns (ancestors (k,),
    new fields (F, k)).  ``y_prev`` is y_{t0} (weights of the models that
    weight after propagating), ``y`` is y_{t0+1}.  Same per-slot arithmetic
    as ``run``, for checking outputs at sizes a whole run would take too
    long for."""
    N = cfg.n
    F = FIELDS[cfg.model]
    s0 = np.ascontiguousarray(state0, dtype=np.float64).reshape(F, N)
    sl = np.ascontiguousarray(slots, dtype=np.int64)
    k = sl.size
    anc = np.zeros(k, dtype=np.int64)
    st = np.zeros((F, k))
    L = lib()
    L.or_step_slots.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double),
                                ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    L.or_step_slots.restype = ctypes.c_int
    rc = L.or_step_slots(ctypes.byref(cfg), _dp(s0), int(t0), float(y_prev), float(y), _ip(sl), k,
                         _ip(anc), _dp(st))
    if rc == -2:
        raise ValueError("or_step_slots: bad arguments")
    return anc, st
