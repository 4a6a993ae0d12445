"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the paper's
timing protocol (mean of the five runs closest to the median, Section 4),
the pooled oracle baseline and the gating of counter figures on the kernel
sources they were taken with."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_median5_protocol():
    # ten runs, median (11 + 12) / 2 = 11.5; distances 0.5 (11, 12), 1.5
    # (10, 13), 2.5 (9), 3.5 (8): the five closest are 9 .. 13
    xs = [70.0, 1.0, 8.0, 13.0, 9.0, 10.0, 11.0, 12.0, 30.0, 50.0]
    assert np.median(xs) == 11.5
    assert bench._median5(xs) == pytest.approx((9 + 10 + 11 + 12 + 13) / 5)
    # outliers on either side do not move it
    assert bench._median5([5.0] * 6 + [1e9, -1e9, 1e9, -1e9]) == 5.0
    assert bench._median5([2.0, 4.0, 6.0, 8.0, 10.0]) == pytest.approx(6.0)


def test_oracle_pool_rate_counts_every_particle_step():
    import oracle
    cfgs = [(oracle.make_config(oracle.LL_PF, n, s, scheme=oracle.STRATIFIED, sigma_v2=1.0,
                                sigma_w2=0.1, x0_var=10.0), np.linspace(-1, 1, 7))
            for s, n in enumerate([64, 128, 256, 32, 512])]
    rate, workers, done = bench.oracle_pool_rate(iter(cfgs), budget_s=30.0)
    assert done == len(cfgs)
    assert 1 <= workers <= 16
    assert rate > 0
    # a zero budget submits nothing
    rate0, _, done0 = bench.oracle_pool_rate(iter(cfgs), budget_s=0.0)
    assert done0 == 0 and rate0 == 0.0


def test_counter_figures_follow_the_kernel_sources(monkeypatch):
    h = bench.kernel_sources_hash()
    assert len(h) == 16
    monkeypatch.setitem(bench.TRAFFIC, "probe", dict(fetch_kib=1.0, write_kib=2.0, sources=h))
    assert bench.traffic_bytes("probe") == pytest.approx((1.0 * bench.FETCH_SCALE
                                                          + 2.0 * bench.WRITE_SCALE) * 1024)
    monkeypatch.setitem(bench.TRAFFIC, "probe", dict(fetch_kib=1.0, write_kib=2.0,
                                                     sources="0" * 16))
    assert bench.traffic_bytes("probe") is None
    assert bench.traffic_bytes("no such workload") is None
    monkeypatch.setitem(bench.VALU_ISSUE, "probe", dict(share=0.5, valu_per_particle=10,
                                                        sources="0" * 16))
    assert bench.valu_issue("probe") is None
