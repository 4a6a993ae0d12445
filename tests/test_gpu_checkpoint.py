"""GPU tests of filter snapshots (pf_checkpoint_save / pf_checkpoint_restore):
a filter saved after t0 steps, destroyed, and restored into a new handle of
the same configuration continues exactly as the uninterrupted filter does:
the same ancestors, particles, log-likelihood and moments bit for bit (the
cycle of Section 3.2 is a function of the particles, the latest CDF and the
step's counter-based draws, all of which the snapshot holds)."""
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


def _strategy(pf, name):
    return {"auto": pf.SEARCH_AUTO, "binary": pf.SEARCH_BINARY, "cutpoint": pf.SEARCH_CUTPOINT,
            "merge": pf.SEARCH_MERGE}[name]


CASES = [
    # model, n, scheme, strategy, items_per_thread, precision fp32, T, t0
    ("ll_pf", 1024, "multinomial", "auto", 0, False, 12, 5),      # fused tile scan, LDS cut-point
    ("ll_pl", 3000, "stratified", "merge", 1, False, 12, 6),      # pending observation
    ("ll_pl", 1 << 16, "stratified", "auto", 4, True, 10, 4),
    ("sv_pl", 20000, "systematic", "merge", 2, True, 10, 3),
    ("sv_pf", 9001, "multinomial", "cutpoint", 2, False, 10, 4),  # cut-point table in memory
    ("ll_pf", 50000, "stratified", "merge", 4, False, 8, 1),      # separate tile-scan launch
]


@pytest.mark.parametrize("model,n,scheme,strat,ipt,fp32,T,t0", CASES)
def test_restored_filter_continues_bit_for_bit(pf, model, n, scheme, strat, ipt, fp32, T, t0):
    print(f"checkpoint {model} n={n} {scheme} {strat} ipt={ipt} fp32={fp32} t0={t0}", flush=True)
    y = C.data(model, T)

    def cfg():
        return C.pf_config(pf, model, n, 13, scheme, fp32=fp32, strategy=_strategy(pf, strat),
                           ipt=ipt)

    ref = pf.Filter(cfg())
    ref.step(y)
    want_ll = ref.loglik()
    want_mom = ref.moments()
    want_rec, want_anc, want_t = ref.particles()
    ref.close()

    a = pf.Filter(cfg())
    a.step(y[:t0])
    snap = a.checkpoint()
    a.close()
    b = pf.Filter(cfg())
    b.step(y[:1])           # some unrelated state of its own, replaced by the restore
    b.restore(snap)
    b.step(y[t0:])
    assert b.loglik() == want_ll
    np.testing.assert_array_equal(b.moments(), want_mom)
    rec, anc, t = b.particles()
    assert t == want_t
    np.testing.assert_array_equal(anc, want_anc)
    np.testing.assert_array_equal(rec, want_rec)
    # the same snapshot rewinds a filter that has moved on (moments first:
    # for particle learning they complete the latest propagation, as above)
    b.restore(snap)
    b.step(y[t0:])
    assert b.loglik() == want_ll
    np.testing.assert_array_equal(b.moments(), want_mom)
    np.testing.assert_array_equal(b.particles()[0], want_rec)
    b.close()


def test_snapshot_taken_between_moments_and_steps(pf):
    # a particle-learning filter whose pending propagation was flushed by
    # pf_moments before the snapshot
    y = C.data("ll_pl", 16)
    cfg = lambda: C.pf_config(pf, "ll_pl", 5000, 3, "stratified", fp32=False)  # noqa: E731
    ref = pf.Filter(cfg())
    for t in range(16):
        ref.step(y[t])
        if t == 6:
            ref.moments()
    a = pf.Filter(cfg())
    a.step(y[:7])
    a.moments()
    snap = a.checkpoint()
    a.close()
    b = pf.Filter(cfg())
    b.restore(snap)
    b.step(y[7:])
    assert b.loglik() == ref.loglik()
    np.testing.assert_array_equal(b.moments(), ref.moments())
    ref.close()
    b.close()


def test_restore_refuses_other_configurations(pf):
    y = C.data("ll_pf", 4)
    a = pf.Filter(C.pf_config(pf, "ll_pf", 2000, 1, "stratified", fp32=False))
    a.step(y)
    snap = a.checkpoint()
    for other in (C.pf_config(pf, "ll_pf", 2001, 1, "stratified", fp32=False),
                  C.pf_config(pf, "ll_pf", 2000, 2, "stratified", fp32=False),
                  C.pf_config(pf, "ll_pf", 2000, 1, "systematic", fp32=False),
                  C.pf_config(pf, "ll_pf", 2000, 1, "stratified", fp32=True)):
        o = pf.Filter(other)
        with pytest.raises(pf.PFError) as e:
            o.restore(snap)
        assert e.value.code == pf.EINVAL
        o.close()
    with pytest.raises(pf.PFError):
        a.restore(snap[:-1])
    bad = snap.copy()
    bad[:8] = 0
    with pytest.raises(pf.PFError):
        a.restore(bad)
    # a refused restore leaves the filter as it was
    ll = a.loglik()
    a.restore(snap)
    assert a.loglik() == ll
    a.close()
