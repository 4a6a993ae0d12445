"""GPU parity of the whole cycle (weights, CDF, resampling, propagation)
through the C-ABI, against the CPU oracle on the same random streams.

Double precision: ancestors bit-exact at every step and every particle's
record within a relative 1e-9 (transcendental functions and summation
order differ by ulps).  Single precision: the target tolerances
|d loglik| <= 1e-3 T and filtered moments within 1e-4 relative (relative to
max(|m|, posterior sd)) against the double-precision oracle driven by the
same random words."""
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


SV_PL_FP64_IPT4_OFF = pytest.mark.skip(
    reason="double-precision SV-PL with 4 items per thread is switched off: it gave wrong "
           "weights from the first resampling on (and its one sorted-multinomial run faulted "
           "the GPU); the cause has not been found, and the library refuses the configuration")

CASES = [
    # model, n, scheme, strategy, items_per_thread, T, scan
    ("ll_pf", 1024, "multinomial", "auto", 0, 100, "tiles"),   # the 1024-particle FP64 workload
    ("ll_pf", 1500, "multinomial", "cutpoint", 4, 20, "tiles"),
    ("ll_pf", 3000, "stratified", "merge", 1, 20, "tiles"),
    ("ll_pf", 3000, "multinomial", "binary", 1, 20, "tiles"),
    ("ll_pf", 700, "systematic", "merge", 1, 20, "tiles"),
    ("ll_pf", 9001, "stratified", "merge", 2, 12, "tiles"),
    ("ll_pl", 3000, "stratified", "merge", 1, 20, "tiles"),
    ("ll_pl", 1500, "multinomial", "auto", 4, 20, "tiles"),
    ("ll_pl", 2049, "systematic", "binary", 2, 20, "tiles"),
    ("sv_pf", 3000, "systematic", "merge", 1, 20, "tiles"),
    ("sv_pf", 1000, "multinomial", "cutpoint", 4, 20, "tiles"),
    ("sv_pl", 3000, "systematic", "merge", 1, 20, "tiles"),
    ("sv_pl", 1777, "stratified", "binary", 2, 20, "tiles"),
    ("sv_pl", 513, "multinomial", "auto", 1, 20, "tiles"),
    ("sv_pl", 20000, "systematic", "merge", 8, 10, "tiles"),
    ("ll_pf", 3000, "stratified", "merge", 1, 20, "lookback"),
    ("ll_pl", 2049, "systematic", "binary", 2, 20, "lookback"),
    ("sv_pl", 3000, "systematic", "merge", 1, 20, "lookback"),
    ("sv_pf", 9001, "stratified", "merge", 8, 12, "lookback"),
    # the tile scan run by the cycle kernel's last work-group (at most 16
    # tiles, here with N a multiple of the tile) and, one particle more, by
    # the separate scan kernel
    ("ll_pl", 16 * 1024, "stratified", "merge", 4, 8, "tiles"),
    ("ll_pl", 16 * 1024 + 1, "stratified", "merge", 4, 8, "tiles"),
    ("sv_pl", 16 * 1024, "systematic", "merge", 8, 8, "tiles"),
    ("ll_pf", 16 * 1024, "stratified", "merge", 4, 8, "tiles"),
    ("sv_pf", 16 * 1024 + 3, "systematic", "merge", 4, 8, "tiles"),
    # the cut-point method with its table in device memory (multinomial
    # above one LDS window): built after each weighting, then a bounded climb
    ("ll_pf", 3000, "multinomial", "cutpoint", 1, 20, "tiles"),
    ("ll_pl", 20000, "multinomial", "auto", 4, 12, "tiles"),
    ("sv_pf", 16 * 1024 + 1, "multinomial", "cutpoint", 4, 8, "tiles"),
    ("sv_pl", 5000, "multinomial", "auto", 2, 12, "tiles"),
    ("ll_pf", 9000, "multinomial", "cutpoint", 8, 10, "tiles"),
    # more than 4096 tiles: the tile scan runs in chunks (three launches)
    ("ll_pf", 4096 * 256 + 300, "stratified", "merge", 1, 4, "tiles"),
    ("sv_pf", 4096 * 256 + 1, "systematic", "merge", 1, 3, "tiles"),
    ("ll_pl", 4097 * 256, "stratified", "merge", 1, 3, "tiles"),
    # double-precision SV-PL at 4 items per thread: switched off (refused)
    pytest.param("sv_pl", 16 * 1024, "systematic", "merge", 4, 8, "tiles", marks=SV_PL_FP64_IPT4_OFF),
    pytest.param("sv_pl", 8 * 1024, "systematic", "merge", 4, 8, "lookback", marks=SV_PL_FP64_IPT4_OFF),
    # sorted multinomial (order statistics from exponential spacings); its
    # first GPU run faulted in the fourth case, in the switched-off double-
    # precision SV-PL kernel of 4 items per thread, which stays refused
    ("ll_pf", 3000, "sorted_multinomial", "merge", 1, 20, "tiles"),
    ("ll_pf", 700, "sorted_multinomial", "auto", 1, 12, "tiles"),
    ("ll_pl", 2049, "sorted_multinomial", "auto", 2, 20, "tiles"),
    pytest.param("sv_pl", 5000, "sorted_multinomial", "merge", 4, 12, "tiles", marks=SV_PL_FP64_IPT4_OFF),
    ("sv_pl", 5000, "sorted_multinomial", "merge", 2, 12, "tiles"),
    ("sv_pf", 20000, "sorted_multinomial", "binary", 8, 8, "tiles"),
    ("ll_pl", 100000, "sorted_multinomial", "merge", 4, 6, "tiles"),
    ("ll_pf", 4096 * 256 + 300, "sorted_multinomial", "merge", 1, 3, "tiles"),
]


@pytest.mark.parametrize("model,n,scheme,strat,ipt,T,scan", CASES)
def test_fp64_stepwise_parity(pf, orc, model, n, scheme, strat, ipt, T, scan):
    print(f"fp64 parity {model} n={n} {scheme} {strat} ipt={ipt} T={T} scan={scan}", flush=True)
    y = C.data(model, T)
    seed = 7
    ocfg = C.oracle_config(orc, model, n, seed, scheme, fp32=False)
    ref = orc.run(ocfg, y, dump=True)
    assert ref["rc"] == 0
    cfg = C.pf_config(pf, model, n, seed, scheme, fp32=False, strategy=_strategy(pf, strat),
                      ipt=ipt, lookback=(scan == "lookback"))
    f = pf.Filter(cfg)
    lag = 1 if model == "ll_pl" else 0
    for t in range(1, T + 1):
        f.step(y[t - 1])
        rec, anc, tt = f.particles()
        assert tt == t - lag
        ll = f.loglik()
        assert abs(ll - ref["loglik"][:t].sum()) < 1e-9 * max(1.0, abs(ll)), (t, ll)
        if tt == 0:
            continue
        want_anc = ref["anc"][tt - 1]
        bad = np.nonzero(anc != want_anc)[0]
        assert bad.size == 0, (t, bad[:5], anc[bad[:5]], want_anc[bad[:5]])
        want = C.oracle_to_record(orc, model, ocfg, ref["state"][tt - 1])
        np.testing.assert_allclose(rec, want, rtol=1e-9, atol=1e-11)
    mom = f.moments()
    k = mom.size
    np.testing.assert_allclose(mom, ref["moments"][-1, :k], rtol=1e-8, atol=1e-10)
    f.close()


def _rel_err(a, b, sd):
    return np.abs(a - b) / np.maximum(np.abs(b), sd)


FP32_MODELS = [("ll_pl", "stratified"), ("ll_pf", "stratified"), ("sv_pl", "systematic"),
               ("sv_pf", "systematic"),
               ("ll_pl", "sorted_multinomial")]


@pytest.mark.parametrize("model,scheme", FP32_MODELS)
def test_fp32_one_step_from_common_state(pf, orc, model, scheme):
    """Single precision against the double-precision oracle over one cycle
    started from the same particles (the GPU's own state after t0 steps):
    ancestors equal to the oracle's own resampling except for the rare
    slots whose uniform falls within rounding of a CDF value (at most
    1e-3 N); on the GPU's ancestors (the oracle's run_given), filtered
    moments within 1e-4 relative (to max(|m|, sd) for the state) and the
    step's log-likelihood increment within 1e-3.  (A flipped slot takes a
    neighbouring CDF entry, an unrelated particle, so moments against the
    oracle's own resampling would measure the flip count.)"""
    n, t0 = 1 << 18, 40
    print(f"fp32 one step {model} n={n} {scheme} t0={t0}", flush=True)
    y = C.data(model, t0 + 2)
    cfg = C.pf_config(pf, model, n, 3, scheme, fp32=True)
    f = pf.Filter(cfg)
    f.step(y[:t0])
    ll_a = f.loglik()
    if model == "ll_pl":
        # scores y_{t0+1} on z_{t0}; the particles are still z_{t0}
        f.step(y[t0:t0 + 1])
        ll_inc = f.loglik() - ll_a
        rec0, _, tt = f.particles()
        mom = f.moments()          # propagates with y_{t0+1}
    else:
        rec0, _, tt = f.particles()
        f.step(y[t0:t0 + 1])
        ll_inc = f.loglik() - ll_a
        mom = f.moments()
    assert tt == t0
    rec1, anc1, tt1 = f.particles()
    f.close()
    assert tt1 == t0 + 1
    ocfg = C.oracle_config(orc, model, n, 3, scheme, fp32=True)
    state0 = C.record_to_oracle(model, rec0, t0)
    ref = orc.run(ocfg, y[t0:t0 + 1], dump=True, state0=state0, t0=t0, y_prev=y[t0 - 1])
    given = orc.run(ocfg, y[t0:t0 + 1], dump=True, state0=state0, t0=t0, y_prev=y[t0 - 1],
                    anc_first=anc1)
    want = given["moments"][0, : mom.size]
    sd = np.sqrt(want[1])
    assert _rel_err(mom[0], want[0], sd) <= 1e-4, (mom, want)
    assert abs(mom[1] - want[1]) <= 1e-4 * want[1]
    for i in range(2, mom.size):
        assert abs(mom[i] - want[i]) <= 1e-4 * abs(want[i]), (i, mom[i], want[i])
    assert abs(ll_inc - given["loglik"][0]) <= 1e-3, (ll_inc, given["loglik"][0])
    flips = np.count_nonzero(anc1 != ref["anc"][0])
    print("ancestor flips", flips, "of", n)
    assert flips <= 1e-3 * n
    want_rec = C.oracle_to_record(orc, model, ocfg, given["state"][0]) if model != "sv_pl" else None
    if want_rec is not None:
        close = np.isclose(rec1, want_rec, rtol=1e-4, atol=1e-5)
        assert np.count_nonzero(~close) <= 1e-4 * n * rec1.shape[0]


@pytest.mark.parametrize("model,scheme", FP32_MODELS)
def test_fp32_trajectory(pf, orc, model, scheme):
    """Whole single-precision runs against the double-precision oracle:
    |d loglik| <= 1e-3 T.  A single-precision run and the oracle's run
    decorrelate after their first ancestor flips, so one pair differs by
    Monte Carlo noise (s.d. about 0.02-0.05 at N = 2^16, T = 100, i.e. the
    bound is only about two standard deviations); the arithmetic's effect is
    therefore measured on the means over 8 seeds (standard error about
    0.015).  The filtered means are held to 5% of the filtered standard
    deviation, again on the seed means."""
    n, T, seeds = 1 << 16, 100, range(3, 11)
    print(f"fp32 trajectory {model} n={n} {scheme} T={T} seeds={list(seeds)}", flush=True)
    y = C.data(model, T)
    ll_gpu, ll_or, m_gpu, m_or, sd = [], [], [], [], []
    for seed in seeds:
        ref = orc.run(C.oracle_config(orc, model, n, seed, scheme, fp32=True), y)
        f = pf.Filter(C.pf_config(pf, model, n, seed, scheme, fp32=True, keep_ancestors=False))
        f.step(y)
        ll_gpu.append(f.loglik())
        mom = f.moments()
        f.close()
        ll_or.append(ref["loglik"].sum())
        m_gpu.append(mom[0])
        m_or.append(ref["moments"][-1, 0])
        sd.append(np.sqrt(ref["moments"][-1, 1]))
    d_ll = np.mean(ll_gpu) - np.mean(ll_or)
    d_m = np.mean(m_gpu) - np.mean(m_or)
    print("loglik means", np.mean(ll_gpu), np.mean(ll_or), "per seed", np.subtract(ll_gpu, ll_or))
    assert abs(d_ll) <= 1e-3 * T, (d_ll, ll_gpu, ll_or)
    assert abs(d_m) <= 0.05 * np.mean(sd), (d_m, m_gpu, m_or)


def test_ll_pl_call_pattern_does_not_change_results(pf):
    # the cycle weights y_{t+1} before it propagates with y_t; stepping one
    # observation at a time, in blocks, or with moments read in between must
    # give the same filter
    y = C.data("ll_pl", 40)
    outs = []
    for pattern in ("all", "single", "moments_between"):
        cfg = C.pf_config(pf, "ll_pl", 5000, 11, "stratified", fp32=False)
        f = pf.Filter(cfg)
        if pattern == "all":
            f.step(y)
        else:
            for t in range(40):
                f.step(y[t])
                if pattern == "moments_between" and t % 7 == 3:
                    f.moments()
        ll = f.loglik()
        mom = f.moments()
        rec, anc, tt = f.particles()
        f.close()
        outs.append((ll, mom, rec, tt))
    for ll, mom, rec, tt in outs[1:]:
        assert tt == outs[0][3] == 40
        assert abs(ll - outs[0][0]) < 1e-10
        np.testing.assert_allclose(mom, outs[0][1], rtol=1e-10)
        np.testing.assert_array_equal(rec, outs[0][2])


@pytest.mark.parametrize("scan", ["tiles", "lookback"])
def test_repeat_runs(pf, scan):
    # the tile scan folds the tiles in a fixed order: runs are bit-identical;
    # the look-back's association depends on timing (differences of ulps)
    y = C.data("sv_pl", 30)
    res = []
    for _ in range(2):
        cfg = C.pf_config(pf, "sv_pl", 100000, 5, "systematic", fp32=True,
                          lookback=(scan == "lookback"))
        f = pf.Filter(cfg)
        f.step(y)
        res.append((f.loglik(), f.particles()[0]))
        f.close()
    if scan == "tiles":
        assert res[0][0] == res[1][0]
        np.testing.assert_array_equal(res[0][1], res[1][1])
    else:
        assert abs(res[0][0] - res[1][0]) < 1e-9


def test_cutpoint_table_with_dominant_particles(pf, orc):
    """The cut-point search in device memory when a few particles carry
    almost all the weight (Section 3.2's worst case for the table: one
    particle owns a long run of entries, filled by its whole work-group):
    an outlying observation, then ordinary ones; ancestors bit-exact and
    records within 1e-9 of the oracle at every step."""
    n, T = 60000, 8
    print(f"cut-point table, dominant particles n={n}", flush=True)
    y = C.data("ll_pf", T).copy()
    y[2] += 6.0   # a jump of 6 observation s.d.: few particles keep weight
    ocfg = C.oracle_config(orc, "ll_pf", n, 21, "multinomial", fp32=False)
    ref = orc.run(ocfg, y, dump=True)
    assert ref["rc"] == 0
    f = pf.Filter(C.pf_config(pf, "ll_pf", n, 21, "multinomial", fp32=False,
                              strategy=pf.SEARCH_CUTPOINT, ipt=4))
    for t in range(1, T + 1):
        f.step(y[t - 1])
        rec, anc, tt = f.particles()
        assert tt == t
        np.testing.assert_array_equal(anc, ref["anc"][t - 1])
        np.testing.assert_allclose(rec, ref["state"][t - 1], rtol=1e-9, atol=1e-11)
        ll = f.loglik()
        assert abs(ll - ref["loglik"][:t].sum()) < 1e-9 * max(1.0, abs(ll))
    # the step after the jump resamples from a few ancestors
    assert np.unique(ref["anc"][3]).size < n // 10
    f.close()


def test_errors(pf):
    cfg = C.pf_config(pf, "ll_pf", 1000, 1, "multinomial", fp32=False)
    f = pf.Filter(cfg)
    with pytest.raises(pf.PFError, match="not finite"):
        f.step([1.0, float("nan")])
    f.step([0.5])
    # an observation so far away that every weight underflows to zero
    f.step([1e200])
    with pytest.raises(pf.PFError) as e:
        f.loglik()
    assert e.value.code == pf.EDEGENERATE
    f.close()


@pytest.mark.parametrize("model,scheme", [("ll_pl", "stratified"), ("ll_pf", "stratified"),
                                          ("sv_pl", "systematic"), ("sv_pf", "systematic")])
def test_fp32_common_state_every_step(pf, orc, model, scheme):
    """Single precision against the double-precision oracle at every step of
    a run.  Before each cycle the oracle is handed the GPU's own particles;
    it then runs that cycle twice on the same random words: once with its
    own resampling, to count the slots whose ancestor differs (a uniform
    within rounding of a CDF value: at most 1e-3 N), and once with the GPU's
    ancestors, so that the single-precision propagation, weights and
    moments are held to its arithmetic on exactly the same particles:
    filtered moments within 1e-4 relative (to max(|m|, sd) for the state's
    mean) and the step's log-likelihood increment within 1e-3."""
    n, t_first, T = 1 << 16, 2, 30
    print(f"fp32 every step {model} n={n} {scheme} T={T}", flush=True)
    y = C.data(model, T + 1)
    f = pf.Filter(C.pf_config(pf, model, n, 5, scheme, fp32=True))
    ocfg = C.oracle_config(orc, model, n, 5, scheme, fp32=True)
    f.step(y[:t_first])
    ll_prev = f.loglik()
    worst_m, worst_ll, flips = 0.0, 0.0, 0
    for t0 in range(t_first, T):
        if model == "ll_pl":
            # the call weighs y_{t0+1} on z_{t0}; moments() then propagates
            f.step(y[t0:t0 + 1])
            rec0, _, tt = f.particles()
        else:
            rec0, _, tt = f.particles()
            f.step(y[t0:t0 + 1])
        ll = f.loglik()
        ll_inc, ll_prev = ll - ll_prev, ll
        mom = f.moments()
        _, anc1, _ = f.particles()
        assert tt == t0
        state0 = C.record_to_oracle(model, rec0, t0)
        own = orc.run(ocfg, y[t0:t0 + 1], dump=True, state0=state0, t0=t0, y_prev=y[t0 - 1])
        same = orc.run(ocfg, y[t0:t0 + 1], state0=state0, t0=t0, y_prev=y[t0 - 1],
                       anc_first=anc1)
        want = same["moments"][0, : mom.size]
        sd = np.sqrt(want[1])
        errs = [_rel_err(mom[0], want[0], sd), abs(mom[1] - want[1]) / want[1]]
        errs += [abs(mom[i] - want[i]) / abs(want[i]) for i in range(2, mom.size)]
        worst_m = max(worst_m, max(errs))
        worst_ll = max(worst_ll, abs(ll_inc - same["loglik"][0]))
        flips = max(flips, int(np.count_nonzero(anc1 != own["anc"][0])))
        assert max(errs) <= 1e-4, (t0, mom, want)
        assert abs(ll_inc - same["loglik"][0]) <= 1e-3, (t0, ll_inc, same["loglik"][0])
        assert flips <= 1e-3 * n, (t0, flips)
    print(f"worst moment error {worst_m:.2e}, worst increment error {worst_ll:.2e}, "
          f"most ancestor flips {flips}")
    f.close()


def test_fp32_full_size_trajectory_ll_pl(pf):
    """The full local-level particle-learning configuration in single
    precision (N = 2^20, T = 500, stratified) against the oracle's run on the
    same data and random words (values written by tests/golden/make_fullrun.py
    from the oracle): |d loglik| <= 1e-3 T over the whole run and at every
    50th step (scaled to the steps so far).  At this N one run's Monte Carlo
    s.d. is about 0.004, far inside the bound, so one seed suffices."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ll_pl_2p20_t500.json")
    with open(path) as fh:
        gold = json.load(fh)
    n, T = gold["n"], gold["T"]
    print(f"fp32 full-size trajectory ll_pl n={n} T={T}", flush=True)
    y = C.data("ll_pl", T, seed=gold["data_seed"])
    f = pf.Filter(C.pf_config(pf, "ll_pl", n, gold["filter_seed"], "stratified", fp32=True,
                              keep_ancestors=False))
    cum_or = np.cumsum(gold["loglik_steps"])
    done = 0
    for t in gold["moment_steps"]:
        f.step(y[done:t + 1])
        done = t + 1
        ll = f.loglik()
        assert abs(ll - cum_or[t]) <= 1e-3 * (t + 1), (t, ll, cum_or[t])
    d_ll = f.loglik() - cum_or[-1]
    print(f"loglik {f.loglik():.4f} oracle {cum_or[-1]:.4f} difference {d_ll:.4f}")
    assert abs(d_ll) <= 1e-3 * T
    f.close()


@pytest.mark.parametrize("n,lookback", [(8 * 1024, True), (4 * 1024, False)])
def test_scan_wait_gives_up_and_reports(pf, n, lookback):
    """The tile scans that run inside the cycle kernel wait for other tiles'
    sums with a bound: forced to wait for words no tile writes (a test
    flag), the look-back (8 tiles) and the last work-group's scan (4 tiles)
    give up, the launches end, and the next read reports PF_EDEVICE."""
    print(f"scan stall n={n} lookback={lookback}", flush=True)
    y = C.data("ll_pf", 3)
    cfg = C.pf_config(pf, "ll_pf", n, 1, "stratified", fp32=False, ipt=4, lookback=lookback)
    cfg.flags |= pf.FLAG_TEST_SCAN_STALL
    f = pf.Filter(cfg)
    f.step(y)
    with pytest.raises(pf.PFError) as e:
        f.loglik()
    assert e.value.code == pf.EDEVICE and "stopped waiting" in str(e.value)
    f.close()
    # the same filter without the flag is unaffected
    cfg.flags &= ~pf.FLAG_TEST_SCAN_STALL
    g = pf.Filter(cfg)
    g.step(y)
    assert np.isfinite(g.loglik())
    g.close()
