"""GPU tests of the batched step: many filters of uneven N advanced by one
persistent launch per step from a replayed HIP graph.  Every filter's
results must equal the same filter stepped alone, bit for bit (same kernel
body, same tiling, same fixed-order scan), across graph replays separated by
eager work, ring wrap-around and filters that join at different stages; an
FP64 batch must also match the oracle."""
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


def _make(pf, model, sizes, scheme, fp32, ipt=1, seed0=100):
    return [pf.Filter(C.pf_config(pf, model, n, seed0 + k, scheme, fp32, ipt=ipt))
            for k, n in enumerate(sizes)]


def _data(model, nf, T):
    return np.stack([C.data(model, T, seed=f) for f in range(nf)], axis=1)  # (T, nf)


def _state(f):
    rec, anc, t = f.particles()
    return f.loglik(), rec, anc, t


@pytest.mark.parametrize("model,scheme,fp32", [("ll_pl", "stratified", True),
                                                ("sv_pl", "systematic", True),
                                                ("ll_pf", "multinomial", False),
                                                ("sv_pf", "stratified", True)])
def test_batch_equals_alone(pf, model, scheme, fp32):
    # multinomial members above 512 particles (one tile of 1 item per
    # thread: the LDS window) use the cut-point table in device memory,
    # which the batch builds in its scan launch
    sizes = [700, 3000, 256, 5001, 1]
    print(f"batch vs alone {model} sizes={sizes}", flush=True)
    T = 12
    y = _data(model, len(sizes), T)
    alone = _make(pf, model, sizes, scheme, fp32)
    together = _make(pf, model, sizes, scheme, fp32)
    batch = pf.Batch(together, ring=4)
    # chunks of different sizes (ring wrap-around), eager reads in between
    done = 0
    for chunk in (1, 3, 5, 2, 1):
        batch.step(y[done:done + chunk])
        for k, f in enumerate(alone):
            f.step(y[done:done + chunk, k])
        done += chunk
        for fa, fb in zip(alone, together):
            la, ra, aa, ta = _state(fa)
            lb, rb, ab_, tb = _state(fb)
            assert ta == tb and la == lb, (done, la, lb)
            np.testing.assert_array_equal(ra, rb)
            np.testing.assert_array_equal(aa, ab_)
    for fa, fb in zip(alone, together):
        np.testing.assert_array_equal(fa.moments(), fb.moments())
    batch.close()
    for f in alone + together:
        f.close()


def test_filters_join_at_different_stages(pf):
    # particle learning runs one observation behind; filters stepped alone
    # before joining the batch carry their own stage into it
    sizes = [2000, 1500, 800]
    T = 10
    y = _data("ll_pl", 3, T)
    alone = _make(pf, "ll_pl", sizes, "stratified", True)
    together = _make(pf, "ll_pl", sizes, "stratified", True)
    head = [0, 3, 1]
    for k in range(3):
        if head[k]:
            alone[k].step(y[: head[k], k])
            together[k].step(y[: head[k], k])
    # then each continues with its own next observations, in lockstep
    steps = 5
    yb = np.stack([y[head[k]:head[k] + steps, k] for k in range(3)], axis=1)
    batch = pf.Batch(together)
    batch.step(yb)
    for k in range(3):
        alone[k].step(yb[:, k])
    for fa, fb in zip(alone, together):
        la, ra, aa, ta = _state(fa)
        lb, rb, ab_, tb = _state(fb)
        assert ta == tb and la == lb
        np.testing.assert_array_equal(ra, rb)
    batch.close()
    for f in alone + together:
        f.close()


def test_fp64_batch_matches_oracle(pf, orc):
    sizes = [1024, 3000, 777]
    T = 15
    y = _data("sv_pl", len(sizes), T)
    fs = _make(pf, "sv_pl", sizes, "systematic", fp32=False, ipt=1, seed0=7)
    batch = pf.Batch(fs)
    batch.step(y)
    for k, (f, n) in enumerate(zip(fs, sizes)):
        ocfg = C.oracle_config(orc, "sv_pl", n, 7 + k, "systematic", fp32=False)
        ref = orc.run(ocfg, y[:, k], dump=True)
        ll, rec, anc, t = _state(f)
        assert t == T
        assert abs(ll - ref["loglik"].sum()) < 1e-9 * abs(ll)
        np.testing.assert_array_equal(anc, ref["anc"][-1])
        np.testing.assert_allclose(rec, C.oracle_to_record(orc, "sv_pl", ocfg, ref["state"][-1]),
                                   rtol=1e-9, atol=1e-11)
    batch.close()
    for f in fs:
        f.close()


def test_one_shot_step_batch(pf):
    import ctypes
    sizes = [500, 1200]
    y = _data("ll_pf", 2, 3)
    a = _make(pf, "ll_pf", sizes, "multinomial", False)
    b = _make(pf, "ll_pf", sizes, "multinomial", False)
    arr = (ctypes.c_void_p * 2)(*[f._h.value for f in b])
    for s in range(3):
        row = np.ascontiguousarray(y[s])
        pf._check(pf.lib().pf_step_batch(arr, 2, row.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        for k in range(2):
            a[k].step(y[s, k])
    for fa, fb in zip(a, b):
        assert fa.loglik() == fb.loglik()
    for f in a + b:
        f.close()


def test_batch_errors(pf):
    f1 = pf.Filter(C.pf_config(pf, "ll_pl", 1000, 1, "stratified", True))
    f2 = pf.Filter(C.pf_config(pf, "sv_pl", 1000, 1, "systematic", True))
    f3 = pf.Filter(C.pf_config(pf, "ll_pl", 1000, 1, "stratified", True, lookback=True))
    with pytest.raises(pf.PFError, match="one model"):
        pf.Batch([f1, f2])
    with pytest.raises(pf.PFError, match="twice"):
        pf.Batch([f1, f1])
    with pytest.raises(pf.PFError, match="tile scan"):
        pf.Batch([f1, f3])
    f4 = pf.Filter(C.pf_config(pf, "ll_pl", 3000, 1, "stratified", False, ipt=4))
    f5 = pf.Filter(C.pf_config(pf, "ll_pl", 3000, 2, "sorted_multinomial", False, ipt=4))
    with pytest.raises(pf.PFError, match="stepped alone"):
        pf.Batch([f4, f5])
    b = pf.Batch([f1])
    with pytest.raises(pf.PFError, match="not finite"):
        b.step(np.array([[np.inf]]))
    b.close()
    for f in (f1, f2, f3, f4, f5):
        f.close()


@pytest.mark.parametrize("n,ipt", [(4097 * 256 + 5, 1), (8193 * 1024 - 77, 4)])
def test_large_filter_alone_batched_alone(pf, n, ipt):
    # a filter of more than 4096 tiles (stepped alone its tile scan runs as
    # three chunked launches; in a batch one work-group does the same
    # arithmetic) stepped alone, then in a batch, then alone again, equals
    # the same filter stepped alone throughout: results and the whole
    # snapshot (CDF tables, chunk prefixes, totals) byte for byte
    sizes = [n, 3000]
    T = 7
    y = _data("ll_pl", 2, T)
    print(f"alone / batched / alone sizes={sizes} ipt={ipt}", flush=True)
    ref = _make(pf, "ll_pl", sizes[:1], "stratified", True, ipt=ipt)[0]
    f, g = _make(pf, "ll_pl", sizes, "stratified", True, ipt=ipt)
    snaps = []
    ref.step(y[:5, 0])
    snaps.append(ref.checkpoint())
    ref.step(y[5:, 0])
    snaps.append(ref.checkpoint())
    f.step(y[:3, 0])
    g.step(y[:3, 1])
    batch = pf.Batch([f, g])
    batch.step(y[3:5])
    batch.close()
    got = [f.checkpoint()]
    f.step(y[5:, 0])
    got.append(f.checkpoint())
    for a, b in zip(snaps, got):
        assert a.size == b.size
        diff = np.flatnonzero(a != b)
        assert diff.size == 0, f"snapshots differ at {diff.size} bytes from offset {diff[0]}"
    la, ra, aa, ta = _state(ref)
    lb, rb, ab_, tb = _state(f)
    assert ta == tb and la == lb
    np.testing.assert_array_equal(aa, ab_)
    np.testing.assert_array_equal(ra, rb)
    for h in (ref, f, g):
        h.close()
