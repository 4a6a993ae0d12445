"""Scheduler tests of the continuous-batching server on the CPU, with a
fake device that records what every resident filter is fed: each request
must see exactly its own observations in order whatever the mix, admission
must respect the memory budget (FIFO, optional backfill), malformed
requests are rejected, and nothing is lost."""
import numpy as np
import pytest

from paper_1212_1639_amd import inputs
from paper_1212_1639_amd.serve import Request, Server


class FakeFilter:
    def __init__(self, req):
        self.req = req
        self.fed = []


class FakeBackend:
    tick_seconds = 0.001

    def __init__(self, bytes_per_particle=64):
        self.bpp = bytes_per_particle
        self.members = {}
        self.created = []
        self.suspended = []
        self.resumed = []
        self.ticks = 0

    def footprint(self, req):
        if req.model not in ("ll", "sv") or req.n < 1 or req.T < 1 or not np.all(np.isfinite(req.y)):
            return None
        return req.n * self.bpp

    def create(self, req):
        f = FakeFilter(req)
        self.created.append(req.id)
        return f

    def tiles_bound(self, req):
        return -(-req.n // 256)

    def group_bytes(self, tiles):
        return self.batch_base + 8 * tiles if tiles or self.batch_base else 0

    batch_base = 0

    def suspend(self, h):
        self.suspended.append(h.req.id)
        return list(h.fed)

    def resume(self, req, snap):
        f = FakeFilter(req)
        f.fed = list(snap)
        self.resumed.append(req.id)
        return f

    def set_members(self, group, handles):
        self.members[group] = list(handles)

    def step(self, group, ys):
        hs = self.members[group]
        assert len(hs) == len(ys)
        for h, y in zip(hs, ys):
            h.fed.append(float(y))

    def mark(self):
        self.ticks += 1
        return self.ticks

    def finish(self, h):
        return {"fed": np.array(h.fed)}

    def drain(self):
        pass

    def times(self, events):
        return [e * self.tick_seconds for e in events]


def _requests(k=60, seed=0, rate=2000.0):
    specs = inputs.poisson_requests(rate=rate, duration=k / rate, seed=seed, lo_log2=4, hi_log2=10,
                                    t_lo=3, t_hi=40)
    rng = np.random.default_rng(seed)
    return [Request(id=s["id"], arrival=s["arrival"], model=s["model"], n=s["n"],
                    y=rng.normal(size=s["T"])) for s in specs]


def test_every_request_sees_its_own_observations():
    reqs = _requests()
    be = FakeBackend()
    srv = Server(be, budget_bytes=10 ** 12)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    for r in st["done"]:
        np.testing.assert_array_equal(r.result["fed"], r.y)
    assert st["particle_steps"] == sum(r.n * r.T for r in reqs)


@pytest.mark.parametrize("backfill", [False, True])
def test_budget_is_respected_and_waits_happen(backfill):
    reqs = _requests(k=80, seed=3)
    be = FakeBackend()
    budget = 3 * 1024 * 64   # room for about three of the largest filters
    srv = Server(be, budget_bytes=budget, backfill=backfill)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == len(reqs)
    assert st["max_bytes_in_use"] <= budget
    assert st["queue_delay_ms"]["p99"] > 0  # some requests had to wait
    for r in st["done"]:
        np.testing.assert_array_equal(r.result["fed"], r.y)
    if not backfill:
        # without backfill admission follows arrival order exactly
        order = srv.admitted_order
        arrival = {r.id: (r.arrival, r.id) for r in reqs}
        assert order == sorted(order, key=lambda i: arrival[i])


def test_backfill_lets_small_requests_past_a_big_one():
    y = np.zeros(5)
    reqs = [Request(0, 0.0, "ll", 1000, y), Request(1, 0.0, "ll", 900, y),
            Request(2, 0.0, "sv", 10, y)]
    be = FakeBackend(bytes_per_particle=1)
    srv = Server(be, budget_bytes=1200, backfill=True)
    srv.run(reqs, realtime=False)
    # 0 is admitted, 1 does not fit beside it, 2 does and goes first
    assert srv.admitted_order == [0, 2, 1]
    srv = Server(FakeBackend(bytes_per_particle=1), budget_bytes=1200, backfill=False)
    srv.run(reqs, realtime=False)
    assert srv.admitted_order == [0, 1, 2]


def test_malformed_requests_are_rejected():
    good = Request(0, 0.0, "ll", 100, np.zeros(4))
    bad = [Request(1, 0.0, "ll", 0, np.zeros(4)),          # no particles
           Request(2, 0.0, "xx", 100, np.zeros(4)),        # unknown model
           Request(3, 0.0, "sv", 100, np.array([0.0, np.nan])),  # non-finite data
           Request(4, 0.0, "sv", 100, np.zeros(0)),        # no observations
           Request(5, 0.0, "ll", 10 ** 9, np.zeros(4))]    # larger than the budget
    srv = Server(FakeBackend(), budget_bytes=10 ** 8)
    st = srv.run([good] + bad, realtime=False)
    assert st["completed"] == 1 and st["rejected"] == len(bad)
    np.testing.assert_array_equal(st["done"][0].result["fed"], good.y)


def test_capacity_bounds_resident_filters():
    y = np.zeros(3)
    reqs = [Request(i, 0.0, "ll", 10, y) for i in range(10)]
    be = FakeBackend()
    srv = Server(be, budget_bytes=10 ** 9, capacity=4)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == 10
    assert max(len(v) for v in be.members.values()) <= 4


def test_batch_buffers_are_charged_to_the_budget():
    # every model group's batch holds buffers of its own (here 10,000 bytes
    # plus 8 per tile): admission leaves room for them, and the bytes in use
    # count them
    reqs = _requests(k=80, seed=5)
    be = FakeBackend()
    be.batch_base = 10_000
    budget = 3 * 1024 * 64
    srv = Server(be, budget_bytes=budget)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == len(reqs)
    assert st["max_bytes_in_use"] <= budget
    assert srv.in_use() >= 2 * 10_000   # both groups' buffers stay allocated
    for r in st["done"]:
        np.testing.assert_array_equal(r.result["fed"], r.y)
    # a request that would fit alone but not beside the batch buffers is rejected
    big = Request(99, 0.0, "ll", budget // 64, np.zeros(3))
    srv = Server(be, budget_bytes=budget)
    srv.group_peak = {"ll": 0, "sv": 0}
    st = srv.run([big], realtime=False)
    assert st["rejected"] == 1


def test_preempted_requests_resume_where_they_stopped():
    reqs = _requests(k=50, seed=7)
    be = FakeBackend()
    srv = Server(be, budget_bytes=10 ** 12)
    picks = {3: 2, 7: 1, 12: 3}     # tick -> how many residents to pre-empt

    def policy(tick, ids):
        return ids[:picks.get(tick, 0)]

    st = srv.run(reqs, realtime=False, preempt=policy)
    assert st["completed"] == len(reqs) and st["preempted"] == 6
    assert sorted(be.suspended) == sorted(be.resumed) == sorted(srv.preempted)
    for r in st["done"]:
        np.testing.assert_array_equal(r.result["fed"], r.y)
    assert st["particle_steps"] == sum(r.n * r.T for r in reqs)
