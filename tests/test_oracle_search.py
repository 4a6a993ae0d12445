"""Pins of the oracle's CDF and inverse-CDF search (Section 3).

The worked example of Table 1, the definition of a cut-point, the three
properties of L_j listed in Section 3.2, and brute force on random CDFs.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1212_1639_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_cutpoint.json")


@pytest.fixture(scope="module")
def table1():
    with open(GOLD) as f:
        return json.load(f)


def test_table1_L_and_cutpoints(orc, table1):
    q = np.array(table1["q"])
    L, I = orc.cutpoint_table(q)
    assert list(L) == table1["L"]
    inc = [bool(L[0] > 0)] + [bool(L[j] > L[j - 1]) for j in range(1, 10)]
    assert inc == table1["L_increases"]
    assert list(I + 1) == table1["I_definition"]
    # the definition of a cut-point, written as a brute-force minimum
    N = q.size
    brute = [min(i for i in range(N) if q[i] > (k - 1) / N) + 1 for k in range(1, N + 1)]
    assert brute == table1["I_definition"]


def test_table1_resampled_indices(orc, table1):
    q = np.array(table1["q"])
    u = np.array(table1["u"])
    _, I = orc.cutpoint_table(q)
    N = q.size
    assert [math.ceil(N * v) for v in u] == table1["ceil_Nu"]
    assert [int(I[c - 1]) + 1 for c in table1["ceil_Nu"]] == table1["I_at_ceil_Nu"]
    climbs = []
    for v in u:
        _, c = orc.cutpoint_draw(q, I, v)
        climbs.append(c)
    assert max(climbs) == table1["max_climbs"]
    for method in (orc.SEARCH_BINARY, orc.SEARCH_CUTPOINT, orc.SEARCH_BRUTE):
        assert list(orc.search(q, u, method) + 1) == table1["resampled"]


@pytest.mark.parametrize("kind", ["sorted", "cliffs", "flat_runs", "step"])
@pytest.mark.parametrize("n", [1, 2, 7, 64, 1000, 4099])
def test_search_methods_agree_with_brute(orc, kind, n):
    q = inputs.random_cdf(n, seed=n, kind=kind)
    rng = np.random.default_rng(n + 1)
    u = rng.random(2 * n + 5)
    # exact ties with CDF values inside (0, 1], and the ends of (0, 1]; the
    # uniforms of the cut-point method live on the open interval (0, 1)
    pos = q[q > 0][:5]
    u[: pos.size] = pos
    u[-1] = 1.0
    u[-2] = 1e-300
    brute = np.array([min([k for k in range(n) if q[k] >= v] or [n - 1]) for v in u])
    for method in (orc.SEARCH_BINARY, orc.SEARCH_CUTPOINT, orc.SEARCH_BRUTE):
        assert np.array_equal(orc.search(q, u, method), brute)
    # searchsorted 'left' is the same inverse CDF
    assert np.array_equal(np.minimum(np.searchsorted(q, u, side="left"), n - 1), brute)


@pytest.mark.parametrize("kind", ["sorted", "cliffs", "flat_runs", "step"])
def test_L_properties_and_table(orc, kind):
    n = 513
    q = inputs.random_cdf(n, seed=3, kind=kind)
    L, I = orc.cutpoint_table(q)
    # property 1: 0 = L_0 < L_1 <= ... <= L_N = N (L_1 > 0 needs q(1) > 0)
    assert np.all(np.diff(L) >= 0) and L[-1] == n and L[0] >= 0
    # properties 2 and 3: entries L_{j-1}+1..L_j hold j; j with L_{j-1} = L_j owns none
    prev = 0
    for j in range(n):
        for k in range(prev + 1, L[j] + 1):
            assert I[k - 1] == j
        prev = L[j]
    # the table is the definition I_k = min{i : q_i > (k-1)/N}
    for k in range(1, n + 1):
        idx = np.nonzero(q > (k - 1) / n)[0]
        assert I[k - 1] == (idx[0] if idx.size else n - 1)


def test_cdf_normaliser_against_exact_sum(orc):
    rng = np.random.default_rng(5)
    lw = rng.normal(size=10007) * 30.0 - 500.0
    q, M, S = orc.cdf(lw)
    assert M == lw.max()
    assert S == pytest.approx(math.fsum(np.exp(lw - M)), rel=1e-13)
    assert q[-1] == 1.0 and np.all(np.diff(q) >= 0)
    pref = np.cumsum(np.exp(lw - M))
    assert np.allclose(q[:-1], pref[:-1] / S, rtol=1e-12, atol=0)
