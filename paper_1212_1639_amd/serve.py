"""Continuous-batching server for particle filters.

Requests (a model, a particle count N, an observation sequence of length T)
arrive over time.  Each tick the server
  1. queues the requests that have arrived,
  2. admits queued requests in arrival order while their device footprint
     (pf_workspace_bytes, plus what their model's batch allocates for
     itself, pf_batch_bytes) fits the memory budget and a batch slot is
     free; with backfill, a request that does not fit lets later, smaller
     ones past it; pre-empted requests (below) come back first,
  3. advances every resident filter by one observation: one batch per model
     (pf_batch_update + pf_batch_step), so filters that joined at different
     times share each launch,
  4. retires the filters that have consumed their whole sequence (reads the
     log-likelihood and moments, frees the workspace).
Filters keep their particles and statistics in device memory from admission
to retirement, unless a pre-emption policy (a callable given to run) picks
them: a pre-empted filter is saved to host memory (pf_checkpoint_save),
its device memory freed, and it rejoins the queue ahead of new arrivals;
when it is admitted again it continues from the snapshot
(pf_checkpoint_restore) exactly as if it had not been interrupted.  Per-step latency is the interval between two consecutive
step completions of one filter (device events, one per tick); queueing delay
is admission time minus arrival time (host clock).

The scheduling logic is independent of the device: `GpuBackend` drives the
C-ABI library; tests substitute a fake backend that records what each filter
was fed.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    model: str              # 'll' (local-level PL) or 'sv' (stochastic-volatility PL)
    n: int                  # particles
    y: np.ndarray           # observations, length T
    result: dict = field(default=None)

    @property
    def T(self):
        return int(self.y.size)


def stream_requests(specs, ll_data, sv_data):
    """Turn arrival specs (inputs.poisson_requests) into requests with data."""
    out = []
    for s in specs:
        y = ll_data(s["T"], s["id"]) if s["model"] == "ll" else sv_data(s["T"], s["id"])
        out.append(Request(id=s["id"], arrival=s["arrival"], model=s["model"], n=s["n"], y=y))
    return out


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


class Server:
    def __init__(self, backend, budget_bytes, capacity=1024, backfill=True):
        self.be = backend
        self.budget = int(budget_bytes)
        self.capacity = int(capacity)
        self.backfill = backfill
        self.used = 0             # workspaces of resident filters
        self.queue = collections.deque()
        self.active = {}          # id -> dict(req, handle, idx, bytes, group)
        self.rejected = []
        self.max_used = 0
        self.admitted_order = []
        self.suspended = {}       # id -> (snapshot, idx) of pre-empted filters
        self.preempted = []       # ids in the order they were pre-empted
        # per model group: tiles of the members (an upper bound), and the most
        # the group's batch has had to hold (its tile map never shrinks)
        self.group_tiles = collections.Counter()
        self.group_peak = {}

    # ------------------------------------------------------------ accounting
    def _batch_bytes(self, peaks):
        return sum(self.be.group_bytes(t) for t in peaks.values())

    def in_use(self):
        """Device bytes the server holds: resident workspaces plus every
        model group's batch buffers."""
        return self.used + self._batch_bytes(self.group_peak)

    def _fits(self, req, nbytes):
        peaks = dict(self.group_peak)
        g = req.model
        peaks[g] = max(peaks.get(g, 0), self.group_tiles[g] + self.be.tiles_bound(req))
        return self.used + nbytes + self._batch_bytes(peaks) <= self.budget

    def _never_fits(self, req, nbytes):
        # batch buffers are never released, so a request that does not fit
        # with no filter resident never will
        peaks = dict(self.group_peak)
        g = req.model
        peaks[g] = max(peaks.get(g, 0), self.be.tiles_bound(req))
        return nbytes + self._batch_bytes(peaks) > self.budget

    def _charge(self, req, nbytes, sign):
        g = req.model
        self.used += sign * nbytes
        self.group_tiles[g] += sign * self.be.tiles_bound(req)
        self.group_peak[g] = max(self.group_peak.get(g, 0), self.group_tiles[g])
        self.max_used = max(self.max_used, self.in_use())

    # ------------------------------------------------------------ admission
    def _admit(self, now):
        admitted = []
        kept = collections.deque()
        blocked = False
        while self.queue:
            req = self.queue.popleft()
            if blocked and not self.backfill:
                kept.append(req)
                continue
            nbytes = self.be.footprint(req)
            if nbytes is None:                 # malformed request
                self.rejected.append(req)
                continue
            per_group = sum(1 for a in self.active.values() if a["group"] == req.model)
            if self._fits(req, nbytes) and per_group < self.capacity:
                idx = 0
                if req.id in self.suspended:
                    snap, idx = self.suspended.pop(req.id)
                    h = self.be.resume(req, snap)
                else:
                    h = self.be.create(req)
                self._charge(req, nbytes, +1)
                self.active[req.id] = dict(req=req, handle=h, idx=idx, bytes=nbytes,
                                           group=req.model, admitted=now, last_done=None)
                self.admitted_order.append(req.id)
                admitted.append(req.id)
            else:
                if self._never_fits(req, nbytes):
                    self.rejected.append(req)   # can never fit
                    continue
                kept.append(req)
                blocked = True
        self.queue = kept
        return admitted

    # ------------------------------------------------------------ main loop
    def run(self, requests, realtime=True, max_ticks=None, preempt=None):
        """Serve `requests` (sorted by arrival).  Returns a stats dict.

        preempt: optional policy, called after every tick as
        preempt(tick, resident_ids) -> ids to pre-empt (save to host, free,
        re-queue ahead of new arrivals)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        sim_now = 0.0
        ticks = 0
        queue_delays = []
        step_lat = []
        particle_steps = 0
        tick_log = []   # (event, [(group, [ids])])
        done = []
        members = {}    # group -> list of ids in the batch
        while pending or self.queue or self.active:
            now = clock() if realtime else sim_now
            while pending and pending[0].arrival <= now:
                self.queue.append(pending.popleft())
            if not self.active and not self.queue and pending:
                # idle until the next arrival
                if realtime:
                    time.sleep(max(0.0, pending[0].arrival - now))
                else:
                    sim_now = pending[0].arrival
                continue
            for rid in self._admit(now):
                if self.active[rid]["idx"] == 0:
                    queue_delays.append(now - self.active[rid]["req"].arrival)
            # one step for every resident filter, one batch per model
            groups = collections.defaultdict(list)
            for rid, a in self.active.items():
                groups[a["group"]].append(rid)
            stepped = []
            for g, ids in groups.items():
                if members.get(g) != ids:
                    self.be.set_members(g, [self.active[i]["handle"] for i in ids])
                    members[g] = list(ids)
                ys = np.array([self.active[i]["req"].y[self.active[i]["idx"]] for i in ids])
                self.be.step(g, ys)
                for i in ids:
                    self.active[i]["idx"] += 1
                    particle_steps += self.active[i]["req"].n
                stepped.append((g, ids))
            for g in list(members):
                if g not in groups and members[g]:
                    self.be.set_members(g, [])
                    members[g] = []
            ev = self.be.mark()
            tick_log.append((ev, [i for _, ids in stepped for i in ids]))
            ticks += 1
            # retire finished filters
            finished = [rid for rid, a in self.active.items() if a["idx"] >= a["req"].T]
            if finished:
                for g in list(members):
                    keep = [i for i in members[g] if i not in finished]
                    if keep != members[g]:
                        self.be.set_members(g, [self.active[i]["handle"] for i in keep])
                        members[g] = keep
                for rid in finished:
                    a = self.active.pop(rid)
                    a["req"].result = self.be.finish(a["handle"])
                    self._charge(a["req"], a["bytes"], -1)
                    done.append(a["req"])
            # pre-emption: save, free, and queue ahead of new arrivals
            victims = [i for i in (preempt(ticks, list(self.active)) if preempt else [])
                       if i in self.active]
            if victims:
                for g in list(members):
                    keep = [i for i in members[g] if i not in victims]
                    if keep != members[g]:
                        self.be.set_members(g, [self.active[i]["handle"] for i in keep])
                        members[g] = keep
                for rid in reversed(victims):
                    a = self.active.pop(rid)
                    self.suspended[rid] = (self.be.suspend(a["handle"]), a["idx"])
                    self._charge(a["req"], a["bytes"], -1)
                    self.preempted.append(rid)
                    self.queue.appendleft(a["req"])
            if not realtime:
                sim_now += self.be.tick_seconds
            if max_ticks and ticks >= max_ticks:
                break
        self.be.drain()
        wall = (time.perf_counter() - t0)
        # per-step latency: gaps between consecutive step completions of a filter
        times = self.be.times([ev for ev, _ in tick_log])
        last = {}
        for (ev, ids), tt in zip(tick_log, times):
            for i in ids:
                if i in last:
                    step_lat.append(tt - last[i])
                last[i] = tt
        return {
            "requests": len(requests), "completed": len(done), "rejected": len(self.rejected),
            "ticks": ticks, "wall_s": wall, "particle_steps": particle_steps,
            "particle_steps_per_s": particle_steps / wall if wall > 0 else float("nan"),
            "step_latency_ms": {"p50": 1e3 * percentile(step_lat, 50),
                                "p99": 1e3 * percentile(step_lat, 99)},
            "queue_delay_ms": {"p50": 1e3 * percentile(queue_delays, 50),
                               "p99": 1e3 * percentile(queue_delays, 99)},
            "max_bytes_in_use": self.max_used, "budget_bytes": self.budget,
            "preempted": len(self.preempted),
            "done": done,
        }


class GpuBackend:
    """Filters and batches of the C-ABI library on one GPU stream."""

    tick_seconds = 0.0

    RING = 8

    def __init__(self, params, capacity=1024, items_per_thread=4, stream=None, precision=None):
        """params: group -> dict(model, scheme, params[, precision,
        items_per_thread]); a group's precision defaults to `precision`
        (FP32 if None) and its tile size to items_per_thread."""
        import torch
        from paper_1212_1639_amd import pf
        self.pf = pf
        self.torch = torch
        self.params = params
        self.capacity = capacity
        self.ipt = items_per_thread
        self.precision = pf.FP32 if precision is None else precision
        self.stream = stream or torch.cuda.Stream()
        self.batches = {}
        self.events = []
        self.t0 = torch.cuda.Event(enable_timing=True)
        self.t0.record(self.stream)

    def _cfg(self, req):
        p = self.params[req.model]
        return self.pf.make_config(p["model"], req.n, req.id, scheme=p["scheme"],
                                   precision=p.get("precision", self.precision),
                                   items_per_thread=p.get("items_per_thread", self.ipt),
                                   **p["params"])

    def tiles_bound(self, req):
        # a tile holds at least 256 particles (one item per thread)
        return -(-int(req.n) // 256)

    def group_bytes(self, tiles):
        return self.pf.lib().pf_batch_bytes(self.capacity, self.RING, int(tiles))

    def suspend(self, handle):
        snap = handle.checkpoint()
        handle.close()
        return snap

    def resume(self, req, snap):
        h = self.create(req)
        h.restore(snap)
        return h

    def footprint(self, req):
        if req.model not in self.params or req.n < 1 or req.T < 1 or not np.all(np.isfinite(req.y)):
            return None
        try:
            return self.pf.workspace_bytes(self._cfg(req))
        except self.pf.PFError:
            return None

    def create(self, req):
        return self.pf.Filter(self._cfg(req), stream=self.stream)

    def set_members(self, group, handles):
        b = self.batches.get(group)
        if b is None:
            if not handles:
                return
            b = self.pf.Batch(handles, ring=self.RING, capacity=self.capacity)
            self.batches[group] = b
        else:
            b.update(handles)

    def step(self, group, ys):
        self.batches[group].step(ys)

    def mark(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def finish(self, handle):
        ll = handle.loglik()
        mom = handle.moments()
        handle.close()
        return {"loglik": ll, "moments": mom}

    def drain(self):
        self.torch.cuda.synchronize()

    def times(self, events):
        return [self.t0.elapsed_time(ev) * 1e-3 for ev in events]

    def close(self):
        for b in self.batches.values():
            b.close()
        self.batches = {}
