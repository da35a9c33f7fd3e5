"""Scheduler of the serving loop, driven by a fake executor on the CPU:
admission under the byte budget with LRU eviction, at most one in-flight
step per simulation, continuous batching (requests arriving during a launch
go into the next launch, which may start before the first one ends), and the
latency/throughput accounting."""
import collections
import time

import numpy as np
import pytest

from paper_2208_11630_amd import serve


class FakeExecutor(serve.Executor):
    def __init__(self, sizes, cost_per_cell=1e-9, fail_sim=None):
        self.sizes = sizes
        self.res = set()
        self.log = []            # (event, payload)
        self.cost = cost_per_cell
        self.inflight = {}       # handle -> (end time, sims)
        self.active_sims = collections.Counter()
        self.max_overlap = 0
        self.overlapping_launches = 0
        self.next = 0
        self.evicted_at = {}

    def cells_of(self, s):
        return self.sizes[s] ** 3

    def bytes_of(self, s):
        return 80 * self.cells_of(s)

    def is_resident(self, s):
        return s in self.res

    def make_resident(self, s):
        assert s not in self.res
        self.res.add(s)
        self.log.append(("admit", s))

    def evict(self, s):
        assert s in self.res
        assert self.active_sims[s] == 0, "evicted a simulation with a step in flight"
        self.res.discard(s)
        self.log.append(("evict", s))
        self.evicted_at.setdefault(s, []).append(time.perf_counter())

    def launch(self, sims):
        for s in sims:
            assert s in self.res, "launched a non-resident simulation"
            self.active_sims[s] += 1
            assert self.active_sims[s] == 1, "two steps of one simulation in flight"
        if self.inflight:
            self.overlapping_launches += 1
        h = self.next
        self.next += 1
        self.inflight[h] = (time.perf_counter() + self.cost * sum(self.cells_of(s) for s in sims), list(sims))
        self.max_overlap = max(self.max_overlap, len(self.inflight))
        self.log.append(("launch", tuple(sims)))
        return h

    def done(self, h):
        return time.perf_counter() >= self.inflight[h][0]

    def finish(self, h):
        _, sims = self.inflight.pop(h)
        for s in sims:
            self.active_sims[s] -= 1


def test_all_requests_served_once_in_order_per_sim():
    sizes = [32, 48, 64, 32, 80]
    ex = FakeExecutor(sizes)
    srv = serve.Server(ex, budget_bytes=10 ** 12)
    arr = serve.poisson_arrivals(rate=4000, duration=0.05, nsims=len(sizes), seed=1)
    st = srv.run(arr)
    assert len(st.requests) == len(arr)
    assert all(not np.isnan(r.t_done) and r.t_done >= r.t_launch >= r.t_arrival for r in st.requests)
    # per simulation, requests complete in arrival order (one step in flight at a time)
    by = collections.defaultdict(list)
    for r in st.requests:
        by[r.sim].append(r)
    for rs in by.values():
        done = [r.t_done for r in sorted(rs, key=lambda r: r.t_arrival)]
        assert done == sorted(done)
    s = st.summary()
    assert s["completed"] == len(arr) and s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_respected_with_lru_eviction():
    sizes = [64] * 10                       # 80 B * 64^3 = 21 MB each
    ex = FakeExecutor(sizes)
    budget = 3 * 80 * 64 ** 3 + 10           # room for three
    srv = serve.Server(ex, budget_bytes=budget)
    arr = [(0.0001 * k, k % 10) for k in range(60)]
    st = srv.run(arr)
    assert st.summary()["completed"] == 60
    assert st.evictions > 0
    # replay the log: resident bytes never exceed the budget
    res = set()
    for ev, x in ex.log:
        if ev == "admit":
            res.add(x)
        elif ev == "evict":
            res.discard(x)
        assert sum(80 * 64 ** 3 for _ in res) <= budget


def test_no_eviction_of_a_simulation_with_waiting_requests():
    """Under a budget of three simulations and a stream cycling over ten, no
    simulation is evicted between the moment the loop takes in one of its
    requests and that request's launch (its state would only have to come
    back), and the launches take resident simulations before waiting for
    admissions."""
    sizes = [64] * 10
    ex = FakeExecutor(sizes, cost_per_cell=4e-9)
    srv = serve.Server(ex, budget_bytes=3 * 80 * 64 ** 3 + 10)
    rng = np.random.default_rng(3)
    arr = [(0.0002 * k, int(x)) for k, x in enumerate(rng.integers(0, 10, size=200))]
    st = srv.run(arr)
    assert st.summary()["completed"] == 200
    assert st.evictions > 0
    for r in st.requests:
        for t in ex.evicted_at.get(r.sim, []):
            assert r.t_arrival <= r.t_seen <= r.t_launch
            assert not (r.t_seen < t < r.t_launch), (r.sim, r.t_seen, t, r.t_launch)


def test_restore_returns_to_the_same_residency():
    """restore() brings back exactly the listed simulations in that LRU order
    after a run that changed the residency, within the budget."""
    sizes = [64] * 10
    ex = FakeExecutor(sizes)
    srv = serve.Server(ex, budget_bytes=4 * 80 * 64 ** 3 + 10)
    srv.stats = serve.Stats()
    for s in (2, 7, 4, 9):
        srv._admit(s, set())
    snap = list(srv.lru)
    st = srv.run([(0.0001 * k, k % 10) for k in range(40)])
    assert st.evictions > 0 and set(srv.lru) != set(snap)
    srv.restore(snap)
    assert list(srv.lru) == snap and ex.res == set(snap)
    assert srv.used == sum(ex.bytes_of(s) for s in snap) <= srv.budget


def test_request_larger_than_budget_is_refused_not_hung():
    sizes = [32, 256]
    ex = FakeExecutor(sizes)
    srv = serve.Server(ex, budget_bytes=80 * 128 ** 3)
    st = srv.run([(0.0, 0), (0.0, 1)])
    assert st.refused > 0
    done = [r for r in st.requests if not np.isnan(r.t_done)]
    assert [r.sim for r in done] == [0]


def test_continuous_batching_overlaps_launches():
    sizes = [64] * 40
    ex = FakeExecutor(sizes, cost_per_cell=2e-8)  # ~5 ms per 64^3 step: launches overlap arrivals
    srv = serve.Server(ex, budget_bytes=10 ** 12, max_inflight=2)
    arr = serve.poisson_arrivals(rate=3000, duration=0.1, nsims=40, seed=2)
    st = srv.run(arr)
    assert st.summary()["completed"] == len(arr)
    assert ex.max_overlap == 2 and ex.overlapping_launches > 0
    assert st.summary()["mean_batch"] > 1.0


def test_poisson_arrivals_statistics():
    arr = serve.poisson_arrivals(rate=2000.0, duration=2.0, nsims=100, seed=4)
    assert abs(len(arr) - 4000) < 4 * np.sqrt(4000)
    t = np.array([a[0] for a in arr])
    assert np.all(np.diff(t) >= 0) and t.min() >= 0 and t.max() <= 2.0
    gaps = np.diff(t)
    assert abs(gaps.mean() * 2000.0 - 1.0) < 0.1


def test_pinned_pool_recycles_exact_sizes_and_respects_its_cap():
    """Host bookkeeping of the pinned pool (plain host tensors stand in for
    pinned ones): buffers come from large chunks, are recycled by exact size,
    and get() refuses once the chunk cap is reached."""
    import torch

    class HostTorch:
        uint8 = torch.uint8

        @staticmethod
        def empty(n, dtype, pin_memory):
            return torch.empty(n, dtype=dtype)

    p = serve.PinnedPool(HostTorch, chunk_bytes=1 << 20, cap_bytes=2 << 20)
    a = p.get(300_000)
    b = p.get(300_000)
    assert a.numel() == b.numel() == 300_000
    assert b.data_ptr() - a.data_ptr() == 303_104          # 4 KiB-aligned carving
    c = p.get(500_000)                                       # does not fit the first chunk
    assert len(p.chunks) == 2 and c.data_ptr() == p.chunks[1].data_ptr()
    p.put(a)
    assert p.get(300_000).data_ptr() == a.data_ptr()        # recycled, same size
    assert p.get(600_000) is None                            # would need a third chunk
    assert p.get(2 << 20) is None                            # larger than a chunk


class FailingExecutor(FakeExecutor):
    """Raises at the launch that carries `raise_sim`; reports `bad_sim` as
    failed when its step completes."""

    def __init__(self, sizes, raise_sim, bad_sim):
        super().__init__(sizes)
        self.raise_sim, self.bad_sim = raise_sim, bad_sim

    def launch(self, sims):
        if self.raise_sim in sims:
            raise RuntimeError("device error")
        return super().launch(sims)

    def finish(self, h):
        sims = self.inflight[h][1]
        super().finish(h)
        return {self.bad_sim} & set(sims)


def test_failures_stay_local_and_quarantine_the_sim():
    sizes = [16] * 6
    ex = FailingExecutor(sizes, raise_sim=1, bad_sim=4)
    srv = serve.Server(ex, budget_bytes=10 ** 9, max_inflight=2, max_cells_per_launch=16 ** 3)
    arrivals = [(0.0005 * i, i % 6) for i in range(60)]
    stats = srv.run(arrivals)
    by_sim = collections.defaultdict(list)
    for r in stats.requests:
        by_sim[r.sim].append(r)
    for s in (0, 2, 3, 5):
        assert all(r.error is None and not np.isnan(r.t_done) for r in by_sim[s]), s
    assert all(r.error and "launch raised RuntimeError" in r.error for r in by_sim[1])
    assert all(np.isnan(r.t_done) for r in by_sim[1])
    # sim 4: its first step fails when it completes, every later request at once
    assert all(r.error == "step failed" for r in by_sim[4])
    assert sum(1 for ev, p in ex.log if ev == "launch" and 4 in p) == 1
    assert stats.failed == len(by_sim[1]) + len(by_sim[4]) == 20
    assert srv.quarantined.keys() == {1, 4}
    summ = stats.summary()
    assert summ["completed"] == 40 and summ["failed"] == 20


class SlowCopyExecutor(FakeExecutor):
    """Admissions whose copies take `copy_s` to land: a simulation is
    resident at once but in place (ready) only after its copy."""

    def __init__(self, sizes, copy_s, cost_per_cell):
        super().__init__(sizes, cost_per_cell=cost_per_cell)
        self.copy_s = copy_s
        self.landed = {}
        self.admits_under_launch = 0
        self.max_copies = 0

    def make_resident(self, s):
        super().make_resident(s)
        now = time.perf_counter()
        self.landed[s] = now + self.copy_s
        if self.inflight:
            self.admits_under_launch += 1
        self.max_copies = max(self.max_copies, sum(1 for t in self.landed.values() if t > now))

    def evict(self, s):
        super().evict(s)
        self.landed.pop(s, None)

    def is_ready(self, s):
        return s in self.res and time.perf_counter() >= self.landed.get(s, 0.0)

    def launch(self, sims):
        for s in sims:
            assert self.is_ready(s), "launched a simulation whose copy had not landed"
        return super().launch(sims)


def test_admission_copies_overlap_the_launches():
    """With the launch slot busy the loop still starts admission copies
    (at most `max_admitting` in flight), and a launch takes a simulation only
    once its copy has landed."""
    sizes = [64] * 30
    ex = SlowCopyExecutor(sizes, copy_s=2e-3, cost_per_cell=2e-8)   # ~5 ms per 64^3 step
    srv = serve.Server(ex, budget_bytes=10 ** 12, max_inflight=1, max_cells_per_launch=2 * 64 ** 3,
                       max_admitting=4)
    arr = [(0.0, k % 30) for k in range(90)]
    st = srv.run(arr)
    assert st.summary()["completed"] == 90
    assert ex.admits_under_launch > 0
    assert ex.max_copies <= 4
