"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *generates data*: simulated observation paths of the two
state-space models and the size / arrival mixes of the batched and served
workloads.  It holds none of the filter's arithmetic (no weights, CDF,
resampling or propagation), so both the HIP path and the CPU oracle can be
fed from it without sharing any of the method.

The observation paths draw one (transition, observation) normal pair per
time step in time order, so the first T' observations of a length-T path
equal the path of length T' for the same seed.
"""
from __future__ import annotations

import numpy as np

# Local-level ("stochastic trend with noise") model of Section 4:
#   y_t = x_t + v_t, v_t ~ N(0, sigma_v2);  x_t = x_{t-1} + w_t, w_t ~ N(0, sigma_w2).
LL_TRUTH = dict(sigma_v2=1.0, sigma_w2=0.1, x0=0.0)
# Stochastic volatility: x_t = mu + phi (x_{t-1} - mu) + sigma eta_t, y_t ~ N(0, exp(x_t)).
SV_TRUTH = dict(mu=-1.0, phi=0.95, sigma=0.2)


def local_level(T, seed=0, sigma_v2=1.0, sigma_w2=0.1, x0=0.0):
    """Simulate (y[T], x[T]) of the local-level model from x_0 = x0."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((T, 2))
    x = x0 + np.cumsum(np.sqrt(sigma_w2) * e[:, 0])
    y = x + np.sqrt(sigma_v2) * e[:, 1]
    return y, x


def stochastic_volatility(T, seed=0, mu=-1.0, phi=0.95, sigma=0.2, x0=None):
    """Simulate (y[T], x[T]); x_0 from the stationary law unless given."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((T + 1, 2))
    if x0 is None:
        x0 = mu + sigma / np.sqrt(1.0 - phi * phi) * e[0, 0]
    x = np.empty(T)
    prev = x0
    for t in range(T):
        prev = mu + phi * (prev - mu) + sigma * e[t + 1, 0]
        x[t] = prev
    y = np.exp(0.5 * x) * e[1:, 1]
    return y, x


def batch_sizes(n_filters=256, lo_log2=12, hi_log2=18, seed=0):
    """Particle counts drawn log-uniform in [2^lo_log2, 2^hi_log2]."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_filters)
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def poisson_requests(rate=200.0, duration=30.0, seed=0, lo_log2=10, hi_log2=20,
                     t_lo=50, t_hi=1000):
    """A Poisson arrival stream of filter requests.

    Returns a list of dicts with arrival time (s), model ('ll' or 'sv', 50/50),
    particle count (log-uniform in [2^lo_log2, 2^hi_log2]), T (uniform integer
    in [t_lo, t_hi]) and a request id used as data and filter seed.
    """
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        model = "ll" if rng.random() < 0.5 else "sv"
        n = int(np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * rng.random())))
        T = int(rng.integers(t_lo, t_hi + 1))
        reqs.append(dict(id=rid, arrival=t, model=model, n=n, T=T))
        rid += 1
    return reqs


def random_cdf(n, seed=0, kind="sorted"):
    """A non-decreasing FP64 array in [0, 1] whose last value is 1, for search tests.

    kind: 'sorted' (sorted uniforms), 'cliffs' (a few distinct levels, so
    most neighbours are equal and the array jumps in a few places),
    'flat_runs' (90% of entries repeat their left neighbour), 'step' (zeros
    then ones: a single jump).
    """
    rng = np.random.default_rng(seed)
    if kind == "sorted":
        q = np.sort(rng.random(n))
    elif kind == "cliffs":
        levels = np.sort(rng.random(max(2, n // 1000)))
        q = np.sort(rng.choice(levels, size=n))
    elif kind == "flat_runs":
        q = np.sort(rng.random(n))
        keep = rng.random(n) >= 0.9
        keep[0] = True
        idx = np.maximum.accumulate(np.where(keep, np.arange(n), 0))
        q = q[idx]
    elif kind == "step":
        q = np.zeros(n)
        q[int(rng.integers(0, n)):] = 1.0
    else:
        raise ValueError(kind)
    q[-1] = 1.0
    return q
