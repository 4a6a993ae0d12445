"""GPU test of the continuous-batching server: requests of both models and
uneven N and T arrive over time, are admitted by memory footprint and share
batched launches; every request's log-likelihood and moments must be the
same as when the request is run alone (bit-identical: the batched cycle is
the single-filter cycle, and the tile scan is deterministic)."""
import numpy as np
import pytest

from tests import _cases as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_1639_amd import pf as mod
    mod.lib()
    return mod


def _groups(pf):
    return {"ll": dict(model="ll_pl", scheme=pf.STRATIFIED, params=C.PARAMS["ll_pl"]),
            "sv": dict(model="sv_pl", scheme=pf.SYSTEMATIC, params=C.PARAMS["sv_pl"])}


def _reqs(k, rate, seed=0):
    from paper_1212_1639_amd import inputs
    from paper_1212_1639_amd.serve import Request, stream_requests
    specs = inputs.poisson_requests(rate=rate, duration=k / rate, seed=seed, lo_log2=8,
                                    hi_log2=15, t_lo=5, t_hi=60)
    return stream_requests(specs, lambda T, s: inputs.local_level(T, seed=s)[0],
                           lambda T, s: inputs.stochastic_volatility(T, seed=s)[0])


@pytest.mark.parametrize("budget_mb", [4096, 8])
def test_served_equals_alone(pf, budget_mb):
    import torch
    from paper_1212_1639_amd.serve import GpuBackend, Server
    reqs = _reqs(40, rate=400.0)
    print(f"serve {len(reqs)} requests, budget {budget_mb} MiB", flush=True)
    be = GpuBackend(_groups(pf), capacity=64)
    srv = Server(be, budget_bytes=budget_mb << 20)
    st = srv.run(reqs, realtime=True)
    be.close()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["max_bytes_in_use"] <= budget_mb << 20
    assert st["step_latency_ms"]["p50"] > 0
    grp = _groups(pf)
    for r in st["done"]:
        g = grp[r.model]
        cfg = pf.make_config(g["model"], r.n, r.id, scheme=g["scheme"], precision=pf.FP32,
                             items_per_thread=4, **g["params"])
        f = pf.Filter(cfg, stream=torch.cuda.current_stream())
        f.step(r.y)
        ll, mom = f.loglik(), f.moments()
        f.close()
        assert ll == r.result["loglik"], (r.id, ll, r.result["loglik"])
        np.testing.assert_array_equal(mom, r.result["moments"])


def test_served_fp64_matches_the_oracle(pf, orc):
    """Served in double precision (both models, uneven N and T, batched with
    continuous admission): every request's log-likelihood and moments match
    the CPU oracle run alone on the same random streams (log-likelihood to
    1e-9, moments to 1e-8), which anchors the served form to the oracle."""
    from paper_1212_1639_amd import inputs
    from paper_1212_1639_amd.serve import GpuBackend, Server, stream_requests
    specs = inputs.poisson_requests(rate=400.0, duration=16 / 400.0, seed=4, lo_log2=8,
                                    hi_log2=13, t_lo=5, t_hi=30)
    reqs = stream_requests(specs, lambda T, s: inputs.local_level(T, seed=s)[0],
                           lambda T, s: inputs.stochastic_volatility(T, seed=s)[0])
    print(f"serve fp64 {len(reqs)} requests", flush=True)
    groups = _groups(pf)
    groups["sv"]["items_per_thread"] = 2
    be = GpuBackend(groups, capacity=32, precision=pf.FP64)
    st = Server(be, budget_bytes=1 << 30).run(reqs, realtime=True)
    be.close()
    assert st["completed"] == len(reqs)
    name = {"ll": "ll_pl", "sv": "sv_pl"}
    scheme = {"ll": "stratified", "sv": "systematic"}
    for r in st["done"]:
        ocfg = C.oracle_config(orc, name[r.model], r.n, r.id, scheme[r.model], fp32=False)
        ref = orc.run(ocfg, r.y)
        assert ref["rc"] == 0
        mom = r.result["moments"]
        # a particle-learning filter weighs one observation ahead: the served
        # result covers all T observations, as the oracle's run does
        assert abs(r.result["loglik"] - ref["loglik"].sum()) < 1e-9 * max(1.0, abs(ref["loglik"].sum())), r.id
        np.testing.assert_allclose(mom, ref["moments"][-1, :mom.size], rtol=1e-8, atol=1e-10)


def test_preempted_requests_give_the_same_results(pf):
    """Requests pre-empted mid-run (saved to host memory, their device
    memory freed, restored when admitted again) end with the same results,
    bit for bit, as in a run without pre-emption."""
    from paper_1212_1639_amd.serve import GpuBackend, Server
    reqs = _reqs(24, rate=400.0, seed=2)
    print(f"serve with pre-emption, {len(reqs)} requests", flush=True)
    out = []
    for policy in (None, lambda tick, ids: ids[:2] if tick % 9 == 4 else []):
        be = GpuBackend(_groups(pf), capacity=32)
        st = Server(be, budget_bytes=1 << 30).run(reqs, realtime=False, preempt=policy)
        be.close()
        assert st["completed"] == len(reqs)
        out.append({r.id: r.result for r in st["done"]})
        if policy is not None:
            assert st["preempted"] > 0
    for rid, res in out[0].items():
        assert out[1][rid]["loglik"] == res["loglik"], rid
        np.testing.assert_array_equal(out[1][rid]["moments"], res["moments"])
