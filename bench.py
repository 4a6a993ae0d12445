"""Benchmark of the fused particle-filter cycle on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one full cycle of the filter (weights, CDF scan, resampling,
propagation with the particle-learning statistics) over all particles of
one filter, launched through the C-ABI.  Prints ONE JSON line: whole-job
particle-steps/s, the roofline of the cycle kernel (algorithmic bytes per
launch over its average duration, from HIP events on the filter's stream;
HBM traffic and the share of SIMD cycles its vector instructions occupy,
from counter runs of the same kernel sources), the per-step latency of one
filter driven one observation at a time (plain launches and a one-filter
graph replay), and the CPU oracle timed on a bounded sample of the same
workload (one filter per host core for the batched and served workloads).

Workloads (all synthetic; data simulated from the model):
  sv_pl_2p26  particle learning, stochastic volatility, unknown
              (alpha, beta, sigma^2), N = 2^26, T = 1000, systematic, FP32
              (default; the line also carries the batched-vs-plain figures
              of ll_pl_batch256 under "batched")
  ll_pl_2p20  particle learning, local-level model, unknown variances under
              IG(2, 1) priors, N = 2^20, T = 500, stratified, FP32
  ll_pf_1024  bootstrap filter, local-level model, known variances,
              N = 1024, T = 100, multinomial, FP64
  served_mix  a Poisson stream (200 requests/s for 30 s) of filter requests,
              half local-level, half stochastic-volatility particle learning,
              N log-uniform in [2^10, 2^20], T uniform in [50, 1000], served
              with continuous batching under a memory budget (80% of free
              device memory, or --serve-budget-gb); reports p50/p99 per-step
              latency and aggregate particle-steps/s
  paper_table2  the paper's experiment (Section 4): particle learning on the
              local-level model, IG(5, 4) / IG(5, 0.4) priors, T = 100,
              multinomial, the particle record copied to host memory
              after every cycle, N = 2^10 .. 2^23, single and double precision, 10 runs
              per size (mean of the 5 closest to the median; --steps sets
              the run count), plus the phase breakdown at 131,072
  ll_pl_batch256  256 independent local-level particle-learning filters, each
              with its own seed and data, N drawn log-uniform in [2^12, 2^18],
              T = 200, stratified, FP32; stepped together (one launch over
              all their tiles per step, replayed from a HIP graph) and, for comparison,
              one after the other ("plain")
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_EVERY = 8

# HBM bytes per full cycle of the dominant kernel, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE runs (KiB per dispatch) scaled by the counters' reading for a
# 1 GiB device copy (fetch x 2.0, write x 1.0).  Valid only for the kernel
# sources they were taken with (hash of the three files below); otherwise
# the bench reports null.
COUNTER_SOURCES = ("pf_kernels.hip", "pf_models.hpp", "pf_internal.h")
TRAFFIC = {
    "ll_pl_2p20": dict(fetch_kib=14073.86, write_kib=24964.15, sources="de01866dfaa5de0e"),
    "sv_pl_2p26": dict(fetch_kib=981842.78, write_kib=1990648.57, sources="de01866dfaa5de0e"),
    # one batched step: k_step_batch + k_scan_batch
    "ll_pl_batch256": dict(fetch_kib=238748.0, write_kib=442723.26, sources="de01866dfaa5de0e"),
}
# Share of the SIMD cycles the cycle kernel's vector instructions occupy
# (SQ_INSTS_VALU x 4 cycles per wave instruction over the kernel's clock
# cycles x 1024 SIMDs), from a counter run of the same kernel sources.
VALU_ISSUE = {
    "ll_pl_2p20": dict(share=0.52, valu_per_particle=648, sources="de01866dfaa5de0e"),
    "sv_pl_2p26": dict(share=0.95, valu_per_particle=566, sources="de01866dfaa5de0e"),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, "paper_1212_1639_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def valu_issue(workload):
    v = VALU_ISSUE.get(workload)
    if v is None or v["sources"] != kernel_sources_hash():
        return None
    return {"share": v["share"], "valu_per_particle": v["valu_per_particle"]}


def traffic_bytes(workload):
    t = TRAFFIC.get(workload)
    if t is None or t["sources"] != kernel_sources_hash():
        return None
    return (t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE) * 1024.0
METRIC = "particle-steps/sec @1 MI355X (batched vs plain), %HBM peak; p50/p99 step latency"

WORKLOADS = {
    "ll_pl_2p20": dict(model="ll_pl", n=1 << 20, T=500, scheme="stratified", fp32=True,
                       params=dict(x0_mean=0.0, x0_var=10.0, a_v=2.0, b_v=1.0, a_w=2.0, b_w=1.0),
                       # record x, b_v, b_w, sigma_v2, sigma_w2 (4 B each), read + written;
                       # in-tile CDF prefix written then read (4 B each)
                       bytes_per_particle=2 * 20 + 8),
    "sv_pl_2p26": dict(model="sv_pl", n=1 << 26, T=1000, scheme="systematic", fp32=True,
                       params=dict(x0_mean=-1.0, x0_var=0.04 / (1 - 0.95**2),
                                   prior_mean=[-0.05, 0.95], prior_prec=[1.0, 0.0, 1.0],
                                   a_s=2.0, d_s=0.04),
                       # the scope table's figure: a record of x + 7 statistics
                       # (4 B each) read + written, one weight passed across the
                       # scan (written then read)
                       bytes_per_particle=2 * 32 + 8,
                       # what this record layout moves: x + 5 per-particle
                       # statistics (the shape and L00 are per filter)
                       record_bytes_per_particle=2 * 24 + 8),
    # (a latency-bound filter of one to four tiles: its tile size and search
    # are chosen by pf_autotune on the run's own observations)
    "ll_pf_1024": dict(model="ll_pf", n=1024, T=100, scheme="multinomial", fp32=False,
                       params=dict(x0_mean=0.0, x0_var=10.0, sigma_v2=1.0, sigma_w2=0.1),
                       bytes_per_particle=2 * 8 + 16, autotune=True),
    "served_mix": dict(model="mix", n=None, T=None, scheme="mixed", fp32=True, served=True,
                       rate=200.0, duration=30.0, bytes_per_particle=None),
    # the paper's experiment (Section 4, Tables 2 and 3): particle learning on
    # the local-level model with IG(5, 4) and IG(5, 0.4) priors, T = 100, the
    # particles stored to host memory every step, 10 runs per size
    "paper_table2": dict(model="ll_pl", n=None, T=100, scheme="multinomial", fp32=True, paper=True,
                         params=dict(x0_mean=0.0, x0_var=10.0, a_v=5.0, b_v=4.0, a_w=5.0, b_w=0.4),
                         sizes=[1024, 4096, 16384, 131072, 1048576, 8388608], runs=10,
                         bytes_per_particle=2 * 20 + 8),
    "ll_pl_batch256": dict(model="ll_pl", n=None, T=200, scheme="stratified", fp32=True,
                           filters=256, params=dict(x0_mean=0.0, x0_var=10.0, a_v=2.0, b_v=1.0,
                                                    a_w=2.0, b_w=1.0),
                           bytes_per_particle=2 * 20 + 8),
}


def run_served(args, w, pf, torch):
    """The served workload: continuous batching of a Poisson request stream."""
    from paper_1212_1639_amd import inputs
    from paper_1212_1639_amd.serve import GpuBackend, Server, stream_requests
    duration = args.serve_seconds or w["duration"]
    specs = inputs.poisson_requests(rate=w["rate"], duration=duration, seed=0)
    reqs = stream_requests(specs, lambda T, s: inputs.local_level(T, seed=s)[0],
                           lambda T, s: inputs.stochastic_volatility(T, seed=s)[0])
    groups = {"ll": dict(model="ll_pl", scheme=pf.STRATIFIED,
                         params=WORKLOADS["ll_pl_2p20"]["params"]),
              "sv": dict(model="sv_pl", scheme=pf.SYSTEMATIC,
                         params=WORKLOADS["sv_pl_2p26"]["params"])}
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.serve_budget_gb * 2**30) if args.serve_budget_gb else int(0.8 * free)
    be = GpuBackend(groups, capacity=1024)
    srv = Server(be, budget_bytes=budget)
    st = srv.run(reqs, realtime=True)
    be.close()
    out = {
        "metric": METRIC,
        "value": st["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": st["ticks"],
        "warmup": 0,
        "ms_per_step": st["wall_s"] * 1e3 / max(1, st["ticks"]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "rate_per_s": w["rate"], "duration_s": duration,
                   "requests": st["requests"], "budget_bytes": budget, "form": "served"},
        "served": {k: st[k] for k in ("completed", "rejected", "ticks", "wall_s",
                                      "particle_steps", "step_latency_ms", "queue_delay_ms",
                                      "max_bytes_in_use")},
    }
    if not args.no_cpu_baseline:
        # the oracle on the requests in arrival order, each over its first
        # SERVE_CPU_OBS observations, one request per host core, about 15 s
        import oracle
        models = {"ll": (oracle.LL_PL, oracle.STRATIFIED), "sv": (oracle.SV_PL, oracle.SYSTEMATIC)}
        jobs = ((oracle.make_config(models[r.model][0], r.n, r.id, scheme=models[r.model][1],
                                    fp32_words=True, **groups[r.model]["params"]),
                 r.y[:SERVE_CPU_OBS]) for r in reqs)
        rate, workers, done = oracle_pool_rate(jobs)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"first {done} requests in arrival order, first "
                                         f"{SERVE_CPU_OBS} observations each, one request per "
                                         f"worker thread (FP64 C oracle)"}
    print(json.dumps(out), flush=True)


SERVE_CPU_OBS = 20


# The paper's GPU(sp) / GPU(dp) times in ms (Table 2; GTX 580) and the
# breakdown at 131,072 particles (Table 3): context only, other hardware.
PAPER_TABLE2_MS = {"sp": {1024: 17, 4096: 21, 16384: 51, 131072: 216, 1048576: 1527,
                          8388608: 11878},
                   "dp": {1024: 20, 4096: 25, 16384: 130, 131072: 429}}


def _median5(xs):
    """Mean of the five values closest to the median (the paper's protocol)."""
    xs = np.asarray(xs, dtype=np.float64)
    med = np.median(xs)
    return float(np.mean(xs[np.argsort(np.abs(xs - med))[:5]]))


def run_paper(args, w, pf, torch):
    """The paper's experiment: whole particle-learning runs (initialise, T
    cycles, the particles copied to host memory after every cycle), 10 runs
    per size, mean of the 5 closest to the median; single and double
    precision; and the phase breakdown at 131,072."""
    from paper_1212_1639_amd import inputs
    T = w["T"]
    y = inputs.local_level(T, seed=0)[0]
    stream = torch.cuda.Stream()
    runs = args.steps or w["runs"]
    sizes = [n for n in w["sizes"] if not args.paper_max_n or n <= args.paper_max_n]
    table = {"sp": {}, "dp": {}}
    for prec, key in ((pf.FP32, "sp"), (pf.FP64, "dp")):
        for n in sizes:
            def cfg(seed):
                return pf.make_config(w["model"], n, seed, scheme=pf.MULTINOMIAL, precision=prec,
                                      **w["params"])
            times = []
            for r in range(runs + 1):           # run 0 warms up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f = pf.Filter(cfg(r + 1), stream=stream)
                for t in range(T):
                    f.step(y[t])
                    f.particles()               # store: record to host memory
                torch.cuda.synchronize()
                if r:
                    times.append(time.perf_counter() - t0)
                f.close()
            table[key][n] = _median5(times) * 1e3 if len(times) >= 5 else float(np.mean(times)) * 1e3
            print(f"paper_table2 {key} N={n}: {table[key][n]:.2f} ms", file=sys.stderr, flush=True)
    # phase breakdown at 131,072 particles, single precision
    n = 131072
    breakdown = {}
    if n in sizes:
        c = pf.make_config(w["model"], n, 1, scheme=pf.MULTINOMIAL, precision=pf.FP32,
                           **w["params"])
        ph = {"initialize": [], "cycles": [], "cycles_and_store": [], "cycle_kernel": []}
        for r in range(runs + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = pf.Filter(c, stream=stream)
            stream.synchronize()
            t1 = time.perf_counter()
            f.step(y)
            stream.synchronize()
            t2 = time.perf_counter()
            f.close()
            f = pf.Filter(c, stream=stream)
            stream.synchronize()
            t3 = time.perf_counter()
            for t in range(T):
                f.step(y[t])
                f.particles()
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            f.close()
            # the fused cycle kernel alone (resampling, propagation, weights
            # and the in-tile CDF), every launch bracketed by events
            f = pf.Filter(c, stream=stream)
            f.timing_start(T, 1)
            f.step(y)
            stream.synchronize()
            kern_ms, _ = f.timing_read()
            f.close()
            if r:
                ph["initialize"].append(t1 - t0)
                ph["cycles"].append(t2 - t1)
                ph["cycles_and_store"].append(t4 - t3)
                ph["cycle_kernel"].append(kern_ms * 1e-3)
        breakdown = {k: _median5(v) * 1e3 for k, v in ph.items()}
        breakdown["store"] = breakdown["cycles_and_store"] - breakdown["cycles"]
        # the rest of the cycles: the CDF's tile scan, the cut-point table
        # (multinomial above one LDS window) and the gaps between launches
        breakdown["cdf_scan_cut_table_and_gaps"] = breakdown["cycles"] - breakdown["cycle_kernel"]
    # the multinomial cycle with the paper's cut-point search (the library's
    # default: its table in LDS up to 2048 particles, in device memory above)
    # against bisection per slot and against sorted multinomial (the same
    # law, its uniforms formed in order from exponential spacings, searched
    # by the merge at 2 items per thread), and stratified resampling with the
    # merge search for reference: device time per cycle, no store
    search_ms = {}
    for n in [m for m in (131072, 1048576, 8388608) if m in sizes]:
        row = {}
        for name, scheme, strat in (("cutpoint", pf.MULTINOMIAL, pf.SEARCH_CUTPOINT),
                                    ("bisection", pf.MULTINOMIAL, pf.SEARCH_BINARY),
                                    ("sorted_merge", pf.SORTED_MULTINOMIAL, pf.SEARCH_MERGE),
                                    ("stratified_merge", pf.STRATIFIED, pf.SEARCH_MERGE)):
            c = pf.make_config(w["model"], n, 1, scheme=scheme, precision=pf.FP32, strategy=strat,
                               **w["params"])
            f = pf.Filter(c, stream=stream)
            f.step(y[:3])                       # warm-up (the first call only weighs)
            stream.synchronize()
            t0 = time.perf_counter()
            f.step(y[3:])
            stream.synchronize()
            row[name] = (time.perf_counter() - t0) * 1e3 / (T - 3)
            f.close()
        search_ms[str(n)] = {k: round(v, 4) for k, v in row.items()}
        print(f"paper_table2 multinomial cycle N={n}: {search_ms[str(n)]}", file=sys.stderr,
              flush=True)
    nmax = max(table["sp"])
    value = nmax * T / (table["sp"][nmax] * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": T,
        "warmup": 1,
        "ms_per_step": table["sp"][nmax] / T,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "model": w["model"], "T": T, "scheme": "multinomial",
                   "priors": "IG(5,4), IG(5,0.4)", "runs": runs, "form": "plain",
                   "store": "particle record to host memory after every cycle (synchronous)"},
        "table2_ms": {k: {str(n): round(v, 3) for n, v in d.items()} for k, d in table.items()},
        "table3_131072_ms": {k: round(v, 3) for k, v in breakdown.items()},
        "multinomial_cycle_ms": search_ms,
        "paper_gpu_ms_context": {k: {str(n): v for n, v in d.items()}
                                 for k, d in PAPER_TABLE2_MS.items()},
    }
    print(json.dumps(out), flush=True)


def measure_batch(args, w, pf, torch, K, W, tune=True):
    """Batched vs plain stepping of many filters of uneven N: the batch's
    common tile size and search chosen by the library's autotuner (when
    `tune`), then K full cycles of the batch (one launch over all tiles per
    step, replayed from a HIP graph) and the same K cycles with every filter
    stepped alone, one after the other.  The first observation of each
    filter (which only weighs) is stepped before the timed region."""
    from paper_1212_1639_amd import inputs
    nf = w["filters"]
    sizes = inputs.batch_sizes(nf, 12, 18, seed=0)
    T = max(K + 1, W, 3)
    y = np.stack([inputs.local_level(T, seed=f)[0] for f in range(nf)], axis=1)  # (T, nf)
    stream = torch.cuda.Stream()

    def configs():
        return [pf.make_config(w["model"], int(n), f, scheme=pf.STRATIFIED, precision=pf.FP32,
                               items_per_thread=args.items_per_thread, **w["params"])
                for f, n in enumerate(sizes)]

    cfgs = configs()
    tuned = None
    if tune and not args.items_per_thread:
        n_obs = min(T, 8)
        tuned_ms = pf.autotune_batch(cfgs, y[:n_obs], stream=stream)
        tuned = {"items_per_thread": int(cfgs[0].items_per_thread),
                 "strategy": int(cfgs[0].strategy), "tuning_ms_per_step": tuned_ms}

    def filters():
        return [pf.Filter(c, stream=stream) for c in cfgs]

    if W > 0:
        warm = filters()
        b = pf.Batch(warm)
        b.step(y[:W])
        torch.cuda.synchronize()
        b.close()
        for f in warm:
            f.close()
    fs = filters()
    b = pf.Batch(fs, ring=min(K, 256))
    b.step(y[:1])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    b.step(y[1:K + 1])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    lls = [f.loglik() for f in fs]
    b.close()
    for f in fs:
        f.close()
    # plain: the same filters, each stepped alone, one after the other
    ps = filters()
    for k, f in enumerate(ps):
        f.step(y[:1, k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, f in enumerate(ps):
        f.step(y[1:K + 1, k])
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    lls_plain = [f.loglik() for f in ps]
    for f in ps:
        f.close()
    total = int(sizes.sum())
    step_s = ev_ms * 1e-3 / K
    bytes_step = w["bytes_per_particle"] * total
    achieved = bytes_step / step_s / 1e9
    return {
        "value": total * K / wall,
        "ms_per_step": wall * 1e3 / K,
        "config": {"workload": "ll_pl_batch256", "model": w["model"], "filters": nf,
                   "total_particles": total, "n_min": int(sizes.min()), "n_max": int(sizes.max()),
                   "T": w["T"], "scheme": w["scheme"], "form": "batched",
                   "items_per_thread": int(cfgs[0].items_per_thread),
                   "strategy": int(cfgs[0].strategy), "autotuned": tuned is not None},
        "autotune": tuned,
        "plain": {"value": total * K / wall_plain, "ms_per_step": wall_plain * 1e3 / K},
        "batched_over_plain": wall_plain / wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes("ll_pl_batch256"),
                     "kernel": "k_step_batch + k_scan_batch", "kernel_avg_us": step_s * 1e6,
                     "algorithmic_bytes_per_launch": bytes_step},
        "batched_equals_plain_loglik": bool(np.array_equal(np.array(lls), np.array(lls_plain))),
        "sizes": sizes,
        "y": y,
    }


def run_batch(args, w, pf, torch):
    """The batched workload on its own line."""
    K = args.steps or w["T"]
    W = args.warmup
    r = measure_batch(args, w, pf, torch, K, W)
    sizes, y = r.pop("sizes"), r.pop("y")
    out = {"metric": METRIC, "value": r["value"], "unit": "particle-steps/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    out.update({k: v for k, v in r.items() if k not in ("value", "ms_per_step")})
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(w, sizes, y, K)
    print(json.dumps(out), flush=True)


def batch_cpu_baseline(w, sizes, y, K):
    """The oracle on the filters of the batched workload in order, one filter
    per host core, for about 15 s."""
    import oracle
    jobs = ((oracle.make_config(oracle.LL_PL, int(n), f, scheme=oracle.STRATIFIED,
                                fp32_words=True, **w["params"]), y[1:K + 1, f])
            for f, n in enumerate(sizes))
    rate, workers, done = oracle_pool_rate(jobs)
    return {"value": rate, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"first {done} of {len(sizes)} filters, {K} steps each, one filter per "
                      f"worker thread (FP64 C oracle)", "host": host_info()}


def data(w, T):
    from paper_1212_1639_amd import inputs
    if w["model"].startswith("ll"):
        return inputs.local_level(T, seed=0)[0]
    return inputs.stochastic_volatility(T, seed=0)[0]


def host_info():
    """Host cores (all, and those this process may run on) and CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model}


def synthetic_state(w, n, seed=12345):
    """Particles after one step, drawn from the model with its true
    parameters, in the oracle's field layout: the CPU baseline starts from
    them so that it times full cycles (resample, propagate, weigh) and not
    the initial draw.  numpy draws; none of the filter's arithmetic."""
    from paper_1212_1639_amd import inputs
    rng = np.random.default_rng(seed)
    m = w["model"]
    if m == "sv_pl":
        tr = inputs.SV_TRUTH
        x0 = tr["mu"] + tr["sigma"] / np.sqrt(1 - tr["phi"] ** 2) * rng.standard_normal(n)
        x1 = tr["mu"] + tr["phi"] * (x0 - tr["mu"]) + tr["sigma"] * rng.standard_normal(n)
        # (x, n, S1, S11, Sy, S1y, Syy): the path sums of one transition
        return np.stack([x1, np.ones(n), x0, x0 * x0, x1, x0 * x1, x1 * x1])
    if m == "ll_pl":
        p = w["params"]
        x = p["x0_mean"] + np.sqrt(p["x0_var"]) * rng.standard_normal(n)
        bv = np.full(n, p["b_v"])
        bw = np.full(n, p["b_w"])
        return np.stack([x, bv, bw, bv / rng.gamma(p["a_v"], size=n),
                         bw / rng.gamma(p["a_w"], size=n)])
    p = w["params"]
    return (p["x0_mean"] + np.sqrt(p["x0_var"]) * rng.standard_normal(n))[None, :]


def cpu_baseline(w, y, budget_s=15.0):
    """The oracle as it stands, sequential (1 thread), timed over full cycles
    of the same workload from a particle state after step 1 (its
    initialisation left out): about `budget_s` seconds of steps."""
    import oracle
    model = {"ll_pf": oracle.LL_PF, "ll_pl": oracle.LL_PL, "sv_pf": oracle.SV_PF,
             "sv_pl": oracle.SV_PL}[w["model"]]
    scheme = {"multinomial": oracle.MULTINOMIAL, "stratified": oracle.STRATIFIED,
              "systematic": oracle.SYSTEMATIC}[w["scheme"]]
    n = w["n"]
    cfg = oracle.make_config(model, n, 1, scheme=scheme, fp32_words=w["fp32"], **w["params"])
    s0 = synthetic_state(w, n)
    oracle.lib()
    steps, done, dt = 1, 0, 0.0
    t_all = time.perf_counter()
    while done < len(y) - 1:
        k = min(steps, len(y) - 1 - done)
        t0 = time.perf_counter()
        oracle.run(cfg, y[1 + done:1 + done + k], state0=s0, t0=1 + done, y_prev=y[done])
        dt += time.perf_counter() - t0
        done += k
        left = budget_s - (time.perf_counter() - t_all)
        if left < dt / done:
            break
        # the next batch of steps fits the rest of the budget
        steps = max(1, int(left / (dt / done)))
    return {"value": n * done / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} full cycles at N={n} (sequential FP64 C oracle from a synthetic "
                      f"particle state after step 1, its initialisation not timed)",
            "host": host_info()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: the workload's T)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sv_pl_2p26", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="sv_pl_2p26: leave out the batched-vs-plain figures of ll_pl_batch256")
    ap.add_argument("--items-per-thread", type=int, default=0)
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="served_mix: device memory budget (default 80%% of free memory)")
    ap.add_argument("--serve-seconds", type=float, default=0.0,
                    help="served_mix: length of the arrival window (default 30 s)")
    ap.add_argument("--paper-max-n", type=int, default=0,
                    help="paper_table2: largest N to run (default all, up to 2^23)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the filter, copy MIB mebibytes device to device (a plain "
                         "copy kernel of known size, to scale the profiler's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs each filter on one GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1212_1639_amd import pf

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps or 3)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": nbytes,
                          "copies": max(1, args.steps or 3)}), flush=True)
        return

    w = WORKLOADS[args.workload]
    if w.get("served"):
        torch.cuda.set_device(0)
        run_served(args, w, pf, torch)
        return
    if w.get("filters"):
        torch.cuda.set_device(0)
        run_batch(args, w, pf, torch)
        return
    if w.get("paper"):
        torch.cuda.set_device(0)
        run_paper(args, w, pf, torch)
        return
    K = args.steps or w["T"]
    W = args.warmup
    y = data(w, max(K + 1, W, 2))
    scheme = {"multinomial": pf.MULTINOMIAL, "stratified": pf.STRATIFIED,
              "systematic": pf.SYSTEMATIC}[w["scheme"]]
    cfg = pf.make_config(w["model"], w["n"], 1, scheme=scheme,
                         precision=pf.FP32 if w["fp32"] else pf.FP64,
                         items_per_thread=args.items_per_thread, **w["params"])
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    tuned = None
    if w.get("autotune") and not args.items_per_thread:
        pf.autotune(cfg, y[:K + 1], stream=stream)
        tuned = {"items_per_thread": cfg.items_per_thread, "strategy": cfg.strategy,
                 "lookback_scan": bool(cfg.flags & pf.FLAG_LOOKBACK_SCAN)}

    if W > 0:
        warm = pf.Filter(cfg, stream=stream)
        warm.step(y[:W])
        warm.loglik()
        warm.close()
        del warm

    f = pf.Filter(cfg, stream=stream)
    # the first observation only weighs (particle learning on the local-level
    # model) or has nothing to resample (the other models): it is stepped
    # before the timed region, so that every timed step is a full cycle
    f.step(y[:1])
    # one cycle launch in TIMING_EVERY is bracketed by a pair of HIP events
    # on the filter's stream (the events' own cost then stays out of the
    # other launches and of the throughput)
    f.timing_start(K, TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.step(y[1:K + 1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kern_ms, launches = f.timing_read()
    loglik = f.loglik()
    mom = f.moments()
    f.close()

    n = w["n"]
    value = n * K / wall
    # the cycle kernel's average duration over the bracketed launches
    kern_s = kern_ms * 1e-3 / max(1, launches)
    bytes_launch = w["bytes_per_particle"] * n
    achieved = bytes_launch / kern_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes(args.workload),
            "kernel": "k_step", "kernel_avg_us": kern_s * 1e6, "kernel_launches_timed": launches,
            "bytes_per_particle": w["bytes_per_particle"],
            "algorithmic_bytes_per_launch": bytes_launch,
            "valu_issue": valu_issue(args.workload)}
    rb = w.get("record_bytes_per_particle")
    if rb:
        # the bytes this record layout moves (two statistics are per filter)
        roof["record_bytes_per_particle"] = rb
        roof["record_frac"] = rb * n / kern_s / 1e9 / HBM_PEAK_GBS
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w["fp32"] else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "model": w["model"], "n_particles": n,
                   "T": w["T"], "scheme": w["scheme"], "form": "plain",
                   "timed": "full cycles only (resample, propagate, weigh)"},
        "roofline": roof,
        "loglik": loglik,
        "moments": [float(v) for v in mom],
    }
    if tuned is not None:
        out["config"]["autotuned"] = tuned
    out["latency"] = step_latency(pf, cfg, y, stream, torch, min(K, LATENCY_STEPS))
    if args.workload == "sv_pl_2p26" and not args.no_batch:
        wb = WORKLOADS["ll_pl_batch256"]
        r = measure_batch(args, wb, pf, torch, K, min(W, 5))
        r.pop("sizes")
        r.pop("y")
        out["batched"] = r
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, y)
    print(json.dumps(out), flush=True)


LATENCY_STEPS = 200


def step_latency(pf, cfg, y, stream, torch, steps):
    """Per-step latency of one filter driven one observation at a time (host
    clock from the call to the stream's completion), outside the timed
    region: plain launches (`pf_step`) and a one-filter batch (the captured
    graph replayed per step).  The first two steps of each (initialisation,
    first weighting) are left out."""
    res = {"steps": max(0, steps - 2)}
    for form in ("plain", "graph"):
        if form == "graph" and cfg.flags & pf.FLAG_LOOKBACK_SCAN:
            # a batch steps its members with the tile scan: the one-filter
            # graph runs the same filter with it
            c = pf.Config.from_buffer_copy(cfg)
            c.flags &= ~pf.FLAG_LOOKBACK_SCAN
            f = pf.Filter(c, stream=stream)
            res["graph_scan"] = "tiles"
        else:
            f = pf.Filter(cfg, stream=stream)
        b = pf.Batch([f]) if form == "graph" else None
        lat = []
        for k in range(steps):
            t0 = time.perf_counter()
            if b is None:
                f.step(y[k:k + 1])
            else:
                b.step(y[k:k + 1, None])
            stream.synchronize()
            lat.append(time.perf_counter() - t0)
        if b is not None:
            b.close()
        f.close()
        lat = np.asarray(lat[2:]) * 1e3
        res[form] = ({"p50_ms": float(np.percentile(lat, 50)),
                      "p99_ms": float(np.percentile(lat, 99))} if lat.size else None)
    return res


def oracle_pool_rate(jobs, budget_s=15.0):
    """The oracle on independent filters spread over the host's cores, one
    filter per worker thread (the C oracle releases the interpreter lock
    and keeps no global state).  `jobs` yields (cfg, y) pairs; submission
    stops once `budget_s` of wall time has passed.  Returns (particle-steps
    per second, workers, filters completed)."""
    import concurrent.futures as cf
    import oracle
    oracle.lib()
    workers = max(1, min(16, os.cpu_count() or 1))
    done_ps, done = 0, 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        pending = set()
        it = iter(jobs)
        exhausted = False
        while True:
            while not exhausted and len(pending) < workers and time.perf_counter() - t0 < budget_s:
                try:
                    cfg, yy = next(it)
                except StopIteration:
                    exhausted = True
                    break
                pending.add(ex.submit(lambda c=cfg, v=yy: (oracle.run(c, v), c.n * v.size)[1]))
            if not pending:
                break
            fin, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
            for fu in fin:
                done_ps += fu.result()
                done += 1
    return done_ps / (time.perf_counter() - t0), workers, done


if __name__ == "__main__":
    main()
