"""Pins of the oracle's resampling schemes (Section 3.1; sorted multinomial
from exponential spacings).

Offspring invariants, the exact law of the ancestor vector at N <= 8 by
enumeration, unbiasedness E[offspring_i] = N w_i over many seeds, and the
order-statistic law of the sorted multinomial uniforms.
"""
import math
import itertools

import numpy as np
import pytest
from scipy import stats

SCHEMES = ["multinomial", "stratified", "systematic", "sorted_multinomial"]


def _scheme(orc, name):
    return {"multinomial": orc.MULTINOMIAL, "stratified": orc.STRATIFIED,
            "systematic": orc.SYSTEMATIC, "sorted_multinomial": orc.SORTED_MULTINOMIAL}[name]


def _weights(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.exponential(size=n)
    if n > 1:
        w[rng.integers(0, n)] = 0.0  # a zero weight is never chosen
    return w / w.sum()


def _draw(orc, scheme, q, seed, t=1):
    u = orc.uniforms(_scheme(orc, scheme), seed, t, q.size)
    return orc.search(q, u)


def _q(w):
    q = np.cumsum(w)
    q[-1] = 1.0
    return q


@pytest.mark.parametrize("scheme", SCHEMES)
def test_offspring_invariants(orc, scheme):
    for seed in range(200):
        n = 1 + seed % 37
        w = _weights(n, seed)
        q = _q(w)
        anc = _draw(orc, scheme, q, seed)
        o = np.bincount(anc, minlength=n)
        assert o.sum() == n
        assert np.all(o[w == 0] == 0)
        if scheme != "multinomial":
            assert np.all(np.diff(anc) >= 0)  # sorted uniforms give sorted ancestors
        if scheme == "systematic":
            nw = n * np.diff(np.concatenate([[0.0], q]))
            assert np.all(o >= np.floor(nw - 1e-9)) and np.all(o <= np.ceil(nw + 1e-9))


def _exact_law(scheme, q):
    """Exact probability of every ancestor vector (dict tuple -> prob)."""
    n = q.size
    edges = np.concatenate([[0.0], q])
    if scheme == "multinomial":
        w = np.diff(edges)
        return {v: float(np.prod(w[list(v)])) for v in itertools.product(range(n), repeat=n)}
    if scheme == "sorted_multinomial":
        # non-decreasing vectors only, each with the multinomial probability
        # of its offspring counts
        w = np.diff(edges)
        law = {}
        for v in itertools.combinations_with_replacement(range(n), n):
            o = np.bincount(v, minlength=n)
            coef = math.factorial(n) / np.prod([math.factorial(int(k)) for k in o])
            law[v] = float(coef * np.prod(w ** o))
        return law
    if scheme == "stratified":
        per = []
        for j in range(n):
            lo, hi = j / n, (j + 1) / n
            p = np.clip(np.minimum(edges[1:], hi) - np.maximum(edges[:-1], lo), 0, None) * n
            per.append(p)
        return {v: float(np.prod([per[j][v[j]] for j in range(n)]))
                for v in itertools.product(range(n), repeat=n)}
    # systematic: the vector is piecewise constant in the one offset U;
    # breakpoints are where (j + U)/n crosses a CDF value
    bps = sorted({0.0, 1.0} | {n * qi - j for qi in q for j in range(n)
                               if 0.0 < n * qi - j < 1.0})
    law = {}
    for a, b in zip(bps[:-1], bps[1:]):
        U = 0.5 * (a + b)
        v = tuple(int(min(np.searchsorted(q, (j + U) / n, side="left"), n - 1))
                  for j in range(n))
        law[v] = law.get(v, 0.0) + (b - a)
    return law


@pytest.mark.parametrize("scheme", SCHEMES)
def test_exact_ancestor_law_small_n(orc, scheme):
    n = 4
    w = np.array([0.1, 0.45, 0.05, 0.4])
    q = _q(w)
    law = _exact_law(scheme, q)
    assert sum(law.values()) == pytest.approx(1.0, abs=1e-12)
    S = 40000
    counts = {}
    for seed in range(S):
        v = tuple(int(a) for a in _draw(orc, scheme, q, seed))
        counts[v] = counts.get(v, 0) + 1
    # every observed vector is possible
    assert all(law.get(v, 0.0) > 0 for v in counts)
    keys = [v for v, p in law.items() if p * S >= 5]
    obs = np.array([counts.get(v, 0) for v in keys], dtype=float)
    exp = np.array([law[v] * S for v in keys])
    rest_obs = S - obs.sum()
    rest_exp = S - exp.sum()
    if rest_exp >= 5:
        obs = np.append(obs, rest_obs)
        exp = np.append(exp, rest_exp)
    else:
        exp = exp * obs.sum() / exp.sum()
    chi2 = ((obs - exp) ** 2 / exp).sum()
    p = stats.chi2.sf(chi2, df=max(len(obs) - 1, 1))
    assert p > 1e-4, (scheme, chi2, len(obs))


def test_systematic_is_deterministic_in_offset(orc):
    # the oracle's systematic draw at a given offset equals the enumeration
    n = 6
    w = _weights(n, 9)
    q = _q(w)
    for seed in range(300):
        u = orc.uniforms(orc.SYSTEMATIC, seed, 1, n)
        U = u[0] * n
        assert np.allclose(u, (np.arange(n) + U) / n, rtol=0, atol=1e-15)
        v = orc.search(q, u)
        brute = [min([k for k in range(n) if q[k] >= x] or [n - 1]) for x in u]
        assert list(v) == brute


@pytest.mark.parametrize("scheme", SCHEMES)
def test_unbiased_offspring(orc, scheme):
    n = 16
    w = _weights(n, 4)
    q = _q(w)
    S = 20000
    tot = np.zeros(n)
    for seed in range(S):
        tot += np.bincount(_draw(orc, scheme, q, seed, t=3), minlength=n)
    mean = tot / S
    se = np.sqrt(n * w * (1 - w) / S) + 1e-12
    z = np.abs(mean - n * w) / se
    assert np.all(z < 4.5), (scheme, z.max())


def test_sorted_multinomial_uniforms_are_order_statistics(orc):
    # u_j is the (j+1)-th smallest of N i.i.d. uniforms: Beta(j + 1, N - j)
    n, S = 12, 3000
    us = np.array([orc.uniforms(orc.SORTED_MULTINOMIAL, seed, 2, n) for seed in range(S)])
    assert np.all(np.diff(us, axis=1) > 0) and np.all(us > 0) and np.all(us < 1)
    for j in (0, 5, 11):
        assert stats.kstest(us[:, j], stats.beta(j + 1, n - j).cdf).pvalue > 1e-4
    # the spacings' ratios are independent of the scale: gaps have the law of
    # a uniform spacing, Beta(1, N)
    assert stats.kstest(us[:, 7] - us[:, 6], stats.beta(1, n).cdf).pvalue > 1e-4
