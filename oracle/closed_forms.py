"""Exact (or quadrature-exact) references that pin the oracle.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``).

* ``kalman_ll``: the Kalman filter, exact for the linear-Gaussian local-level
  model (Section 2 notes the closed form exists in that case).
* ``ll_pl_exact``: exact marginal likelihood p(y_{1:t}) and posterior means
  of the two variances and of x_t under inverse-gamma priors, by 2-D
  quadrature over (sigma_v^2, sigma_w^2) of Kalman filters; this is what
  particle learning on the Section 4 model estimates.
* ``sv_grid_filter``: point-mass (grid) filter for the stochastic-volatility
  model with known parameters; converges spectrally in the grid size.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def kalman_ll(y, sigma_v2, sigma_w2, m0, C0):
    """Local-level Kalman filter.

    Returns (loglik_increments[T], filtered_mean[T], filtered_var[T]) where
    increment t is log p(y_t | y_{1:t-1}).  sigma_v2 / sigma_w2 may be arrays
    (broadcast over a parameter grid); the returned arrays then carry the
    grid shape after the time axis.
    """
    y = np.asarray(y, dtype=np.float64)
    sv = np.asarray(sigma_v2, dtype=np.float64)
    sw = np.asarray(sigma_w2, dtype=np.float64)
    shape = np.broadcast(sv, sw).shape
    m = np.full(shape, float(m0))
    C = np.full(shape, float(C0))
    T = y.size
    inc = np.empty((T,) + shape)
    mean = np.empty((T,) + shape)
    var = np.empty((T,) + shape)
    for t in range(T):
        R = C + sw
        Q = R + sv
        e = y[t] - m
        inc[t] = -0.5 * np.log(2.0 * np.pi * Q) - 0.5 * e * e / Q
        K = R / Q
        m = m + K * e
        C = R - K * R
        mean[t] = m
        var[t] = C
    return inc, mean, var


def _log_ig_pdf(x, a, b):
    return a * np.log(b) - special.gammaln(a) - (a + 1.0) * np.log(x) - b / x


def ll_pl_exact(y, a_v, b_v, a_w, b_w, m0, C0, grid=400, lo=1e-4, hi=1e2):
    """Exact targets of particle learning on the local-level model.

    Integrates over (sigma_v^2, sigma_w^2) on a log-spaced product grid with
    the trapezoid rule in log-space (integrand includes the Jacobian).
    Returns dict with arrays over t = 1..T:
      loglik_inc[t-1] = log p(y_t | y_{1:t-1}),
      e_v[t-1], e_w[t-1] = E[sigma_v^2 | y_{1:t}], E[sigma_w^2 | y_{1:t}],
      e_x[t-1] = E[x_t | y_{1:t}].
    """
    s = np.linspace(np.log(lo), np.log(hi), grid)
    ds = s[1] - s[0]
    wq = np.full(grid, ds)
    wq[0] = wq[-1] = 0.5 * ds
    SV, SW = np.meshgrid(np.exp(s), np.exp(s), indexing="ij")
    W2 = np.outer(wq, wq)
    logprior = (_log_ig_pdf(SV, a_v, b_v) + np.log(SV) + _log_ig_pdf(SW, a_w, b_w)
                + np.log(SW) + np.log(W2))
    inc, mean, _ = kalman_ll(y, SV, SW, m0, C0)
    cum = np.cumsum(inc, axis=0)
    T = len(y)
    out = {k: np.empty(T) for k in ("loglik", "e_v", "e_w", "e_x")}
    for t in range(T):
        lj = logprior + cum[t]
        mx = lj.max()
        p = np.exp(lj - mx)
        Z = p.sum()
        out["loglik"][t] = mx + np.log(Z)
        out["e_v"][t] = (p * SV).sum() / Z
        out["e_w"][t] = (p * SW).sum() / Z
        out["e_x"][t] = (p * mean[t]).sum() / Z
    lz = np.concatenate([[0.0], out["loglik"]])
    out["loglik_inc"] = np.diff(lz)
    return out


def sv_grid_filter(y, mu, phi, sigma2, x0_mean, x0_var, grid=2001, width=10.0):
    """Point-mass filter for x_t = mu + phi (x_{t-1} - mu) + sigma Z,
    y_t ~ N(0, exp(x_t)).  Returns (loglik_inc[T], filtered_mean[T],
    filtered_var[T])."""
    y = np.asarray(y, dtype=np.float64)
    sd_stat = np.sqrt(sigma2 / (1.0 - phi * phi))
    half = width * max(sd_stat, np.sqrt(x0_var))
    x = np.linspace(mu - half, mu + half, grid)
    dx = x[1] - x[0]
    # transition density matrix K[i, j] = p(x_i | x_j)
    mean_next = mu + phi * (x - mu)
    K = np.exp(-0.5 * (x[:, None] - mean_next[None, :]) ** 2 / sigma2) / np.sqrt(
        2.0 * np.pi * sigma2)
    f = np.exp(-0.5 * (x - x0_mean) ** 2 / x0_var) / np.sqrt(2.0 * np.pi * x0_var)
    T = y.size
    inc = np.empty(T)
    em = np.empty(T)
    ev = np.empty(T)
    for t in range(T):
        pred = K @ f * dx
        lik = np.exp(-0.5 * (np.log(2.0 * np.pi) + x + y[t] * y[t] * np.exp(-x)))
        joint = pred * lik
        Z = joint.sum() * dx
        inc[t] = np.log(Z)
        f = joint / Z
        em[t] = (f * x).sum() * dx
        ev[t] = (f * x * x).sum() * dx - em[t] ** 2
    return inc, em, ev
