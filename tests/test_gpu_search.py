"""GPU parity of the inverse-CDF search (Section 3.2) through the C-ABI
test surface pf_debug_search: bit-exact ancestors against the oracle, for
every strategy, given the same FP64 CDF and uniforms."""
import json
import os

import numpy as np
import pytest

from paper_1212_1639_amd import inputs

pytestmark = pytest.mark.gpu

STRATS = ["binary", "cutpoint", "merge"]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_1639_amd import pf
    pf.lib()
    return torch.device("cuda:0")


def _strategy(pf, name):
    return {"binary": pf.SEARCH_BINARY, "cutpoint": pf.SEARCH_CUTPOINT,
            "merge": pf.SEARCH_MERGE}[name]


def _gpu_search(dev, q, u, strat):
    import torch
    from paper_1212_1639_amd import pf
    print(f"pf_debug_search n={q.size} m={u.size} strategy={strat}", flush=True)
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    ud = torch.from_numpy(np.ascontiguousarray(u)).to(dev)
    return pf.debug_search(qd, ud, _strategy(pf, strat)).cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("strat", STRATS)
def test_table1(dev, orc, strat):
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_cutpoint.json")) as f:
        t1 = json.load(f)
    q, u = np.array(t1["q"]), np.array(t1["u"])
    got = _gpu_search(dev, q, u, strat)
    assert list(got + 1) == t1["resampled"]
    assert np.array_equal(got, orc.search(q, u))


@pytest.mark.parametrize("strat", STRATS)
@pytest.mark.parametrize("kind", ["sorted", "cliffs", "flat_runs", "step"])
@pytest.mark.parametrize("n,m,sorted_u", [(1, 5, False), (3, 1, True), (1000, 1000, False),
                                           (4099, 4099, True), (70001, 123457, True),
                                           (70001, 5000, False)])
def test_random_cdfs(dev, orc, strat, kind, n, m, sorted_u):
    q = inputs.random_cdf(n, seed=n + m, kind=kind)
    rng = np.random.default_rng(m)
    u = rng.random(m)
    if sorted_u:
        u = np.sort(u)
    pos = q[q > 0][: min(m, 7)]  # exact ties with CDF values
    u[: pos.size] = pos
    if sorted_u:
        u = np.sort(u)
    want = orc.search(q, u)
    got = _gpu_search(dev, q, u, strat)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])


def test_stratified_uniforms_large(dev, orc):
    # the stratified uniforms of a 2^22-particle step against a flat CDF:
    # sampled slots are checked one by one with the oracle's bisection
    n = 1 << 22
    q = inputs.random_cdf(n, seed=5, kind="sorted")
    u = (np.arange(n) + np.random.default_rng(1).random(n)) / n
    res = {s: _gpu_search(dev, q, u, s) for s in ("binary", "merge", "cutpoint")}
    assert np.array_equal(res["binary"], res["merge"])
    assert np.array_equal(res["binary"], res["cutpoint"])
    idx = np.random.default_rng(2).integers(0, n, size=4000)
    want = orc.search(q, u[idx])
    assert np.array_equal(res["binary"][idx], want)
    assert np.all(np.diff(res["merge"]) >= 0)


def test_rejects_decreasing_cdf(dev):
    import torch
    from paper_1212_1639_amd import pf
    q = torch.tensor([0.1, 0.5, 0.4, 1.0], dtype=torch.float64, device=dev)
    u = torch.tensor([0.2], dtype=torch.float64, device=dev)
    with pytest.raises(pf.PFError, match="decreasing"):
        pf.debug_search(q, u, pf.SEARCH_BINARY)


def test_empty_uniforms(dev):
    import torch
    from paper_1212_1639_amd import pf
    q = torch.tensor([0.5, 1.0], dtype=torch.float64, device=dev)
    u = torch.empty(0, dtype=torch.float64, device=dev)
    assert pf.debug_search(q, u, pf.SEARCH_MERGE).numel() == 0


def test_merge_over_a_long_flat_run(dev):
    """Section 3.2's worst case for a merge of sorted uniforms: two heavy
    entries at the ends of a CDF that is flat for 2^22 - 2 entries between
    them, so the tile of uniforms that straddles the jump brackets the
    whole CDF.  The merge bisects per uniform in a bracket wider than 16
    LDS windows: the answers equal searchsorted-left and the call stays
    fast."""
    import time
    import torch
    from paper_1212_1639_amd import pf
    n = 1 << 22
    q = np.full(n, 0.5)
    q[-1] = 1.0
    u = (np.arange(n) + 0.5) / n
    qd = torch.tensor(q, dtype=torch.float64, device=dev)
    ud = torch.tensor(u, dtype=torch.float64, device=dev)
    pf.debug_search(qd, ud, pf.SEARCH_MERGE)   # warm-up
    t0 = time.perf_counter()
    got = pf.debug_search(qd, ud, pf.SEARCH_MERGE).cpu().numpy()
    dt = time.perf_counter() - t0
    want = np.searchsorted(q, u, side="left")
    np.testing.assert_array_equal(got, np.minimum(want, n - 1))
    print(f"merge over a flat run of {n - 2}: {1e3 * dt:.2f} ms", flush=True)
    assert dt < 0.05
