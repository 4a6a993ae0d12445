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
* ``sv_pl_exact``: exact marginal likelihood and posterior means of
  (alpha, beta, sigma^2) for the stochastic-volatility model with unknown
  parameters under the conjugate prior, by quadrature over the parameters
  of grid filters; this is what particle learning on that model estimates.
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



def _sv_pl_quadrature(y, prior_mean, lam0, a_s, d_s, x0_mean, x0_var, n_sigma, n_gh, grid,
                      x_lo, x_hi, center, chunk=64):
    """One quadrature pass of sv_pl_exact.  (alpha, beta) nodes: with
    center None, a Gauss-Hermite product rule for the prior's
    N(prior_mean, sigma^2 Lambda0^{-1}) at each sigma^2 node; with center =
    (m, L, R, n), the trapezoid rule on the square [-R, R]^2 of n x n points
    mapped by u -> m + L u, weighted by the prior density and det L."""
    from scipy import stats as _st
    lo = _st.invgamma.ppf(1e-7, a_s, scale=d_s)
    hi = _st.invgamma.ppf(1.0 - 1e-7, a_s, scale=d_s)
    s = np.linspace(np.log(lo), np.log(hi), n_sigma)
    ws = np.full(n_sigma, s[1] - s[0])
    ws[0] = ws[-1] = 0.5 * (s[1] - s[0])
    sig2 = np.exp(s)
    log_ws = np.log(ws) + _log_ig_pdf(sig2, a_s, d_s) + s    # d sigma^2 = sigma^2 ds
    z, wz = special.roots_hermitenorm(n_gh)
    wz = wz / np.sqrt(2.0 * np.pi)
    Z1, Z2 = np.meshgrid(z, z, indexing="ij")
    zz = np.stack([Z1.ravel(), Z2.ravel()])                    # (2, n_gh^2)
    log_wz = np.log(np.outer(wz, wz).ravel())
    b0 = np.asarray(prior_mean, dtype=np.float64)
    cov0 = np.linalg.inv(lam0)
    if center is None:
        ab = b0[None, :, None] + np.sqrt(sig2)[:, None, None] * (np.linalg.cholesky(cov0) @ zz)[None]
        logw = log_ws[:, None] + log_wz[None, :]
    else:
        m, L, R, n_u = center
        u = np.linspace(-R, R, n_u)
        wu = np.full(n_u, u[1] - u[0])
        wu[0] = wu[-1] = 0.5 * (u[1] - u[0])
        U1, U2 = np.meshgrid(u, u, indexing="ij")
        nodes = np.asarray(m, dtype=np.float64)[:, None] + L @ np.stack([U1.ravel(), U2.ravel()])
        ab = np.broadcast_to(nodes[None], (n_sigma,) + nodes.shape)
        d0 = nodes - b0[:, None]
        quad0 = np.einsum("ik,ij,jk->k", d0, lam0, d0)
        # log N(nodes; b0, sigma^2 Lambda0^{-1}) for every sigma^2 node
        log_prior = (-np.log(2.0 * np.pi) - np.log(sig2)[:, None] + 0.5 * np.log(np.linalg.det(lam0))
                     - 0.5 * quad0[None, :] / sig2[:, None])
        log_area = np.log(np.outer(wu, wu).ravel()) + np.log(abs(np.linalg.det(L)))
        logw = log_ws[:, None] + log_area[None, :] + log_prior
    alpha = ab[:, 0, :].ravel()
    beta = ab[:, 1, :].ravel()
    s2 = np.repeat(sig2, ab.shape[2])
    logw = logw.ravel()
    x = np.linspace(x_lo, x_hi, grid)
    dx = x[1] - x[0]
    f0 = np.exp(-0.5 * (x - x0_mean) ** 2 / x0_var) / np.sqrt(2.0 * np.pi * x0_var)
    lik = np.exp(-0.5 * (np.log(2.0 * np.pi) + x[None, :] + y[:, None] ** 2 * np.exp(-x[None, :])))
    logml = np.empty(alpha.size)
    for c0 in range(0, alpha.size, chunk):
        a = alpha[c0:c0 + chunk, None, None]
        b = beta[c0:c0 + chunk, None, None]
        v = s2[c0:c0 + chunk, None, None]
        # K[k, i, j] = p(x_i | x_j, theta_k)
        K = np.exp(-0.5 * (x[None, :, None] - a - b * x[None, None, :]) ** 2 / v) / np.sqrt(
            2.0 * np.pi * v)
        f = np.broadcast_to(f0, (K.shape[0], grid)).copy()
        acc = np.zeros(K.shape[0])
        for t in range(y.size):
            joint = np.matmul(K, f[:, :, None])[:, :, 0] * dx * lik[t][None, :]
            Zt = joint.sum(axis=1) * dx
            acc += np.log(Zt)
            f = joint / Zt[:, None]
        logml[c0:c0 + chunk] = acc
    lj = logw + logml
    mx = lj.max()
    p = np.exp(lj - mx)
    Zs = p.sum()
    p /= Zs
    th = np.stack([alpha, beta])
    mean = th @ p
    cov = (th - mean[:, None]) * p @ (th - mean[:, None]).T
    return {"loglik": mx + np.log(Zs), "e_alpha": mean[0], "e_beta": mean[1],
            "e_sigma2": p @ s2, "cov_ab": cov}


def sv_pl_exact(y, prior_mean, prior_prec, a_s, d_s, x0_mean, x0_var, n_sigma=16, n_gh=8,
                grid=201, x_lo=-5.0, x_hi=3.0, reach=7.0, n_box=17):
    """Exact targets of stochastic-volatility particle learning with unknown
    (alpha, beta, sigma^2): x_t = alpha + beta x_{t-1} + sigma Z,
    y_t ~ N(0, exp(x_t)), x_0 ~ N(x0_mean, x0_var), prior
    (alpha, beta) | sigma^2 ~ N(prior_mean, sigma^2 Lambda0^{-1}) with
    Lambda0 = [[p0, p1], [p1, p2]], sigma^2 ~ IG(a_s, d_s).

    p(y_{1:T}) = int p(y_{1:T} | theta) p(theta) d theta by quadrature: the
    trapezoid rule in log sigma^2 over the prior's central mass and a
    rule for (alpha, beta), with a point-mass filter on a fixed grid of x
    for every node.  A first pass (Gauss-Hermite on the prior) finds the
    posterior mean and covariance of (alpha, beta), which the data make much
    narrower than the prior; the second integrates by the trapezoid rule
    over that posterior's +-`reach` standard-deviation box in its own
    (Cholesky) coordinates, n_box points a side.  Returns dict with loglik
    (log p(y_{1:T})) and the posterior means e_alpha, e_beta, e_sigma2."""
    y = np.asarray(y, dtype=np.float64)
    p0, p1, p2 = prior_prec
    lam0 = np.array([[p0, p1], [p1, p2]], dtype=np.float64)
    args = (y, prior_mean, lam0, a_s, d_s, x0_mean, x0_var, n_sigma, n_gh, grid, x_lo, x_hi)
    first = _sv_pl_quadrature(*args, center=None)
    m = np.array([first["e_alpha"], first["e_beta"]])
    L = np.linalg.cholesky(first["cov_ab"])
    return _sv_pl_quadrature(*args, center=(m, L, reach, n_box))
