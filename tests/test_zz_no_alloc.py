"""GPU test of the search entry point that allocates nothing
(pf_debug_search_noalloc): on two calls in a row, the second with a smaller
input, every strategy returns exactly what pf_debug_search returns on the
same CDF and uniforms; the static array's previous contents (a raised check
flag, a larger table) do not leak into a later call; sizes beyond the
static table are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_1639_amd import pf
    pf.lib()
    return torch.device("cuda:0")


def _cdf(n, seed):
    from paper_1212_1639_amd import inputs
    return inputs.random_cdf(n, seed=seed)


def _noalloc(q, u, strategy):
    import torch
    from paper_1212_1639_amd import pf
    anc = torch.empty(u.numel(), dtype=torch.int32, device=q.device)
    rc = pf.lib().pf_debug_search_noalloc(
        ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(u.data_ptr()), q.numel(), u.numel(),
        strategy, ctypes.c_void_p(anc.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, anc


@pytest.mark.parametrize("strategy", ["binary", "cutpoint", "merge"])
def test_noalloc_equals_search_on_two_calls(dev, strategy):
    import torch
    from paper_1212_1639_amd import pf
    st = {"binary": pf.SEARCH_BINARY, "cutpoint": pf.SEARCH_CUTPOINT,
          "merge": pf.SEARCH_MERGE}[strategy]
    for call, (n, m) in enumerate([(1 << 20, 300000), (5000, 3001)]):
        print(f"noalloc {strategy} call {call} n={n} m={m}", flush=True)
        q = torch.tensor(_cdf(n, seed=10 + call), dtype=torch.float64, device=dev)
        rng = np.random.default_rng(call)
        u_np = np.sort(rng.random(m)) if strategy == "merge" else rng.random(m)
        u = torch.tensor(1.0 - u_np * 0.999999, dtype=torch.float64, device=dev)
        if strategy == "merge":
            u = torch.flip(u, [0]).contiguous()
        want = pf.debug_search(q, u, st)
        rc, got = _noalloc(q, u, st)
        assert rc == pf.OK, pf.lib().pf_last_error()
        assert torch.equal(got, want)


def test_noalloc_flag_and_limits(dev):
    import torch
    from paper_1212_1639_amd import pf
    q_bad = torch.tensor([0.1, 0.5, 0.4, 1.0], dtype=torch.float64, device=dev)
    u = torch.tensor([0.2, 0.45, 0.9], dtype=torch.float64, device=dev)
    rc, _ = _noalloc(q_bad, u, pf.SEARCH_CUTPOINT)
    assert rc == pf.EINVAL and b"decreasing" in pf.lib().pf_last_error()
    # the raised flag is cleared by the next call
    q = torch.tensor([0.1, 0.4, 0.5, 1.0], dtype=torch.float64, device=dev)
    rc, got = _noalloc(q, u, pf.SEARCH_CUTPOINT)
    assert rc == pf.OK
    assert got.tolist() == [1, 2, 3]
    # the static table holds 2^20 entries; the other strategies take any n
    big = torch.linspace(1.0 / ((1 << 20) + 1), 1.0, (1 << 20) + 1, dtype=torch.float64,
                         device=dev)
    rc, _ = _noalloc(big, u, pf.SEARCH_CUTPOINT)
    assert rc == pf.EINVAL and b"2^20" in pf.lib().pf_last_error()
    rc, got = _noalloc(big, u, pf.SEARCH_BINARY)
    assert rc == pf.OK
    assert torch.equal(got, pf.debug_search(big, u, pf.SEARCH_BINARY))
