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
