"""GPU tests of the autotuner and the kernel-timing hook.

The autotuner only chooses the tile size, search strategy and CDF scan; the
random draws are indexed by particle slot, so a tuned double-precision
filter must still match the oracle (ancestors bit-exact, records to 1e-9),
and a tuned batch must equal its members stepped alone."""
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


@pytest.mark.parametrize("model,n,scheme", [("ll_pf", 1024, "multinomial"),
                                            ("sv_pl", 5000, "systematic"),
                                            ("ll_pl", 70000, "stratified")])
def test_tuned_fp64_filter_matches_oracle(pf, orc, model, n, scheme):
    print(f"autotune fp64 {model} n={n} {scheme}", flush=True)
    T = 12
    y = C.data(model, T)
    cfg = C.pf_config(pf, model, n, 5, scheme, fp32=False)
    ms = pf.autotune(cfg, C.data(model, 6, seed=1))
    assert ms > 0
    assert cfg.items_per_thread in (1, 2, 4, 8)
    assert cfg.strategy in (pf.SEARCH_BINARY, pf.SEARCH_CUTPOINT, pf.SEARCH_MERGE,
                            pf.SEARCH_AUTO)
    # the cached choice comes back unchanged
    again = C.pf_config(pf, model, n, 5, scheme, fp32=False)
    pf.autotune(again, C.data(model, 6, seed=1))
    assert (again.items_per_thread, again.strategy, again.flags) == \
        (cfg.items_per_thread, cfg.strategy, cfg.flags)
    ocfg = C.oracle_config(orc, model, n, 5, scheme, fp32=False)
    ref = orc.run(ocfg, y, dump=True)
    f = pf.Filter(cfg)
    f.step(y)
    rec, anc, tt = f.particles()
    ll = f.loglik()
    assert abs(ll - ref["loglik"].sum()) < 1e-9 * max(1.0, abs(ll))
    np.testing.assert_array_equal(anc, ref["anc"][tt - 1])
    np.testing.assert_allclose(rec, C.oracle_to_record(orc, model, ocfg, ref["state"][tt - 1]),
                               rtol=1e-9, atol=1e-11)
    f.close()


def test_tuned_batch_equals_alone(pf):
    sizes = [4096, 30000, 1000, 70000]
    T = 8
    y = np.stack([C.data("ll_pl", T, seed=f) for f in range(len(sizes))], axis=1)
    cfgs = [C.pf_config(pf, "ll_pl", n, 20 + k, "stratified", fp32=True)
            for k, n in enumerate(sizes)]
    ms = pf.autotune_batch(cfgs, y[:5])
    assert ms > 0
    ipts = {c.items_per_thread for c in cfgs}
    assert len(ipts) == 1 and ipts.pop() in (1, 2, 4, 8)
    together = [pf.Filter(c) for c in cfgs]
    alone = [pf.Filter(c) for c in cfgs]
    b = pf.Batch(together)
    b.step(y)
    for k, f in enumerate(alone):
        f.step(y[:, k])
    for fa, fb in zip(alone, together):
        ra, aa, ta = fa.particles()
        rb, ab_, tb = fb.particles()
        assert ta == tb and fa.loglik() == fb.loglik()
        np.testing.assert_array_equal(ra, rb)
    b.close()
    for f in alone + together:
        f.close()


def test_autotune_errors(pf):
    cfg = C.pf_config(pf, "ll_pl", 1000, 1, "stratified", fp32=True)
    with pytest.raises(pf.PFError, match="n_obs >= 3"):
        pf.autotune(cfg, np.zeros(2))
    with pytest.raises(pf.PFError, match="not finite"):
        pf.autotune(cfg, np.array([0.0, np.nan, 1.0]))
    bad = C.pf_config(pf, "ll_pl", 0, 1, "stratified", fp32=True)
    with pytest.raises(pf.PFError):
        pf.autotune(bad, np.zeros(4))
    look = C.pf_config(pf, "ll_pl", 1000, 1, "stratified", fp32=True, lookback=True)
    with pytest.raises(pf.PFError, match="tile scan"):
        pf.autotune_batch([look], np.zeros((4, 1)))


def test_kernel_timing(pf):
    cfg = C.pf_config(pf, "ll_pl", 1 << 16, 1, "stratified", fp32=True, keep_ancestors=False)
    f = pf.Filter(cfg)
    y = C.data("ll_pl", 30)
    f.timing_start(20)
    f.step(y[:25])          # more launches than armed: only the first 20 are timed
    ms, k = f.timing_read()
    assert k == 20 and ms > 0
    ms2, k2 = f.timing_read()   # disarmed after a read
    assert k2 == 0 and ms2 == 0
    f.timing_start(100, every=4)
    f.step(y[:25])          # launches 0, 4, ..., 24
    ms3, k3 = f.timing_read()
    assert k3 == 7 and ms3 > 0
    with pytest.raises(pf.PFError):
        f.timing_start(0)
    with pytest.raises(pf.PFError):
        f.timing_start(10, every=0)
    f.close()
