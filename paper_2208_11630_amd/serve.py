"""Serving loop: step requests for many resident simulations.

Requests ``(sim, arrival time)`` ask for one step of one simulation.  The
server keeps simulation states on the device within an HBM byte budget
(admitting a simulation evicts least-recently-used idle ones to host memory),
allows at most one in-flight step per simulation, and batches whatever is
ready: all ready requests go into one batched launch (one persistent kernel
over their blocks), and requests that arrive while launches are running are
admitted into the next launch, which may start on a second stream while the
first still runs (continuous batching).  Latency is arrival -> completion of
the step; throughput is cells updated per second.

The device side is an ``Executor``; ``GpuExecutor`` drives libhydro through
the Python binding, and tests drive the scheduler with a fake executor.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    sim: int
    t_arrival: float
    t_launch: float = math.nan
    t_done: float = math.nan
    error: Optional[str] = None   # set when the request failed (it then has no t_done)
    t_seen: float = math.nan      # when the loop took it in (at or after t_arrival)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Executor:
    """What the server needs from the device."""

    def bytes_of(self, sim: int) -> int: ...
    def cells_of(self, sim: int) -> int: ...
    def is_resident(self, sim: int) -> bool: ...
    def is_ready(self, sim: int) -> bool:
        """Resident with its state in place (an admission copy may still be
        in flight after make_resident returns)."""
        return self.is_resident(sim)
    def make_resident(self, sim: int) -> None: ...
    def evict(self, sim: int) -> None: ...
    def settle(self) -> None:
        """Wait for admission and eviction copies in flight and recycle their
        staging memory."""
    def launch(self, sims: Sequence[int]): ...
    def done(self, handle) -> bool: ...
    def finish(self, handle):
        """Complete a launch; may return the sims whose step failed (e.g. a
        nonphysical state): their requests fail and they take no more."""
        ...


@dataclass
class Stats:
    requests: List[Request] = field(default_factory=list)
    launches: int = 0
    cells: int = 0
    evictions: int = 0
    admissions: int = 0
    refused: int = 0
    failed: int = 0
    wall: float = 0.0

    def summary(self) -> Dict:
        lat = np.array([r.latency for r in self.requests if not math.isnan(r.t_done)])
        out = {"completed": int(lat.size), "launches": self.launches, "evictions": self.evictions,
               "admissions": self.admissions, "refused": self.refused, "failed": self.failed,
               "wall_s": self.wall,
               "cell_updates_per_s": self.cells / self.wall if self.wall > 0 else 0.0,
               "requests_per_s": lat.size / self.wall if self.wall > 0 else 0.0}
        if lat.size:
            out.update({"p50_ms": float(np.percentile(lat, 50) * 1e3),
                        "p99_ms": float(np.percentile(lat, 99) * 1e3),
                        "mean_ms": float(lat.mean() * 1e3),
                        "mean_batch": lat.size / max(self.launches, 1)})
        return out


class Server:
    """Admission, continuous batching and completion tracking (host side).

    Failures stay local: a launch that raises fails the requests it carried
    and nothing else; a sim that the executor reports as failed (or whose
    launch raised) is quarantined, and its later requests fail at once."""

    def __init__(self, executor: Executor, budget_bytes: int, max_inflight: int = 2,
                 max_cells_per_launch: Optional[int] = None, clock=time.perf_counter, max_admitting: int = 16):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.max_cells = max_cells_per_launch
        self.max_admitting = max_admitting
        self.clock = clock
        self.used = 0
        self.lru: "collections.OrderedDict[int, None]" = collections.OrderedDict()  # resident, oldest first
        self.busy: set = set()
        self.quarantined: Dict[int, str] = {}

    # -- residency ------------------------------------------------------------
    def _admit(self, sim: int, pinned: set, waiting=()) -> bool:
        """Make sim resident, evicting least-recently-used idle simulations:
        never one with a step in flight, one pinned for the launch being
        formed, or one with requests waiting (`waiting`), whose state would
        only have to come back."""
        if self.ex.is_resident(sim):
            self.lru.move_to_end(sim)
            return True
        need = self.ex.bytes_of(sim)
        if need > self.budget:
            return False
        victims = []
        free = self.budget - self.used
        for s in self.lru:
            if free >= need:
                break
            if s in self.busy or s in pinned or s in waiting:
                continue
            victims.append(s)
            free += self.ex.bytes_of(s)
        if free < need:
            return False
        for s in victims:
            self.ex.evict(s)
            del self.lru[s]
            self.used -= self.ex.bytes_of(s)
            self.stats.evictions += 1
        self.ex.make_resident(sim)
        self.lru[sim] = None
        self.used += need
        self.stats.admissions += 1
        return True

    def restore(self, sims: Sequence[int]) -> None:
        """Make exactly `sims` resident, in that LRU order (evicting every other
        simulation), so that several measured runs start from the same
        residency.  Admissions alternate with the evictions that make room
        for them, and the executor settles its copies every few admissions,
        so host staging memory stays bounded."""
        self.stats = Stats()
        keep = set(sims)
        extra = [s for s in self.lru if s not in keep]
        missing = [s for s in sims if not self.ex.is_resident(s)]

        def drop(v):
            self.ex.evict(v)
            del self.lru[v]
            self.used -= self.ex.bytes_of(v)

        for k, s in enumerate(missing):
            need = self.ex.bytes_of(s)
            while self.budget - self.used < need and extra:
                drop(extra.pop(0))
            if not self._admit(s, set()):
                raise RuntimeError(f"simulation {s} does not fit the budget")
            if k % 8 == 7:
                self.ex.settle()
        for v in extra:
            drop(v)
        self.ex.settle()
        for s in sims:
            self.lru.move_to_end(s)
        self.stats = Stats()

    # -- the loop ---------------------------------------------------------------
    def run(self, arrivals: Sequence[tuple], until_done: bool = True, horizon: Optional[float] = None) -> Stats:
        """Serve arrivals [(t_offset_seconds, sim), ...] sorted by time."""
        self.stats = Stats()
        arrivals = sorted(arrivals)
        pending: "collections.OrderedDict[int, collections.deque]" = collections.OrderedDict()
        inflight: List = []  # (handle, [requests], [sims])
        t0 = self.clock()
        i = 0
        n = len(arrivals)
        # simulations with requests waiting whose state is not on the device,
        # oldest request first, and those whose admission copy is in flight
        to_admit: "collections.OrderedDict[int, None]" = collections.OrderedDict()
        copying: set = set()

        def ingest() -> float:
            # take in every request due by now
            nonlocal i
            now = self.clock() - t0
            while i < n and arrivals[i][0] <= now:
                t, s = arrivals[i]
                r = Request(s, t0 + t, t_seen=t0 + now)
                self.stats.requests.append(r)
                pending.setdefault(s, collections.deque()).append(r)
                if not self.ex.is_resident(s):
                    to_admit[s] = None
                i += 1
            return now

        while True:
            now = ingest()
            # completions
            still = []
            for h, reqs, sims in inflight:
                if self.ex.done(h):
                    try:
                        bad = set(self.ex.finish(h) or ())
                        why = "step failed"
                    except Exception as e:  # the whole launch is lost
                        bad, why = set(sims), f"finish raised {type(e).__name__}: {e}"
                    tdone = self.clock()
                    for r in reqs:
                        if r.sim in bad:
                            self._fail(r, why)
                        else:
                            r.t_done = tdone
                    for s in sims:
                        self.busy.discard(s)
                        if s in bad:
                            self.quarantined[s] = why
                else:
                    still.append((h, reqs, sims))
            inflight = still
            # requests of quarantined sims fail at once
            if self.quarantined:
                for s in [s for s in pending if s in self.quarantined]:
                    for r in pending.pop(s):
                        self._fail(r, self.quarantined[s])
            # admissions: keep up to `max_admitting` state copies in flight
            # whether or not a launch slot is free, so the copies overlap the
            # launches; requests that came due meanwhile count as waiting
            # before any eviction is decided
            copying = {s for s in copying if self.ex.is_resident(s) and not self.ex.is_ready(s)}
            if to_admit and len(copying) < self.max_admitting:
                ingest()
                for s in list(to_admit):
                    if len(copying) >= self.max_admitting:
                        break
                    if s not in pending or s in self.quarantined or self.ex.is_resident(s):
                        # requests gone (or about to fail), or on the device already
                        del to_admit[s]
                        continue
                    if self.ex.bytes_of(s) > self.budget:
                        # can never be resident: refuse its requests (left incomplete)
                        self.stats.refused += len(pending.pop(s))
                        del to_admit[s]
                        continue
                    if not self._admit(s, set(), pending):
                        break  # wait for memory to free up
                    del to_admit[s]
                    if not self.ex.is_ready(s):  # (first touch: in place at once)
                        copying.add(s)
            # the next launch: the waiting simulations whose state is on the
            # device and in place, oldest request first, up to the cell cap
            if len(inflight) < self.max_inflight:
                chosen, reqs, cells = [], [], 0
                for s in list(pending.keys()):
                    if s in self.busy or s in self.quarantined or not self.ex.is_ready(s):
                        continue
                    c = self.ex.cells_of(s)
                    if self.max_cells and chosen and cells + c > self.max_cells:
                        break
                    self.lru.move_to_end(s)
                    chosen.append(s)
                    cells += c
                    q = pending[s]
                    reqs.append(q.popleft())
                    if not q:
                        del pending[s]
                if chosen:
                    try:
                        h = self.ex.launch(chosen)
                    except Exception as e:
                        why = f"launch raised {type(e).__name__}: {e}"
                        for r in reqs:
                            self._fail(r, why)
                        for s_ in chosen:
                            self.quarantined[s_] = why
                        continue
                    tl = self.clock()
                    for r in reqs:
                        r.t_launch = tl
                    for s in chosen:
                        self.busy.add(s)
                    inflight.append((h, reqs, chosen))
                    self.stats.launches += 1
                    self.stats.cells += cells
                    continue
            if i >= n and not inflight and not pending:
                break
            if horizon is not None and now > horizon and not until_done:
                break
            # idle: wait a little for an arrival or a completion
            if not inflight and not copying and i < n:
                dt = arrivals[i][0] - (self.clock() - t0)
                if dt > 2e-4:
                    time.sleep(min(dt, 1e-3))
            else:
                time.sleep(2e-5)
        self.stats.wall = self.clock() - t0
        return self.stats

    def _fail(self, r: Request, why: str) -> None:
        r.error = why
        self.stats.failed += 1


def poisson_arrivals(rate: float, duration: float, nsims: int, seed: int = 4) -> List[tuple]:
    """Poisson arrivals at `rate` per second for `duration` seconds, targets
    uniform over the simulations."""
    rng = np.random.default_rng(seed)
    n = rng.poisson(rate * duration)
    t = np.sort(rng.uniform(0.0, duration, size=n))
    s = rng.integers(0, nsims, size=n)
    return list(zip(t.tolist(), s.tolist()))


class PinnedPool:
    """Pinned host buffers for evicted states, carved from a few large pinned
    chunks and recycled per exact size (the served sizes take a handful of
    values), so the pinned footprint tracks the evicted bytes instead of
    growing with every eviction.  get() returns None once `cap_bytes` of
    chunks are in use (the caller then falls back to pageable memory)."""

    def __init__(self, torch, chunk_bytes: int = 4 << 30, cap_bytes: int = 96 << 30):
        self.torch = torch
        self.chunk_bytes = int(chunk_bytes)
        self.cap_bytes = int(cap_bytes)
        self.chunks: List = []
        self.free: Dict[int, List] = collections.defaultdict(list)
        self.spare: List = []          # reserved chunks not carved yet
        self.off = 0

    def reserve(self, nbytes: int) -> None:
        """Pin up to `nbytes` (within the cap) up front, so that serving does
        not page-lock host memory on its critical path."""
        while (len(self.chunks) + len(self.spare)) * self.chunk_bytes < min(int(nbytes), self.cap_bytes):
            self.spare.append(self.torch.empty(self.chunk_bytes, dtype=self.torch.uint8, pin_memory=True))

    def get(self, nbytes: int):
        lst = self.free.get(nbytes)
        if lst:
            return lst.pop()
        size = (nbytes + 4095) // 4096 * 4096
        if size > self.chunk_bytes:
            return None
        if not self.chunks or self.off + size > self.chunk_bytes:
            if self.spare:
                self.chunks.append(self.spare.pop())
            elif (len(self.chunks) + 1) * self.chunk_bytes > self.cap_bytes:
                return None
            else:
                try:
                    self.chunks.append(self.torch.empty(self.chunk_bytes, dtype=self.torch.uint8, pin_memory=True))
                except RuntimeError:  # the host refuses more page-locked memory: cap the pool here
                    self.cap_bytes = len(self.chunks) * self.chunk_bytes
                    return None
            self.off = 0
        buf = self.chunks[-1][self.off:self.off + nbytes]
        self.off += size
        return buf

    def put(self, buf) -> None:
        self.free[buf.numel()].append(buf)


class GpuExecutor(Executor):
    """Simulations as libhydro grids on the device.

    A resident simulation holds one state buffer (40 B per cell); each launch
    lends its members an output buffer for the step in flight (from torch's
    caching allocator, so no device allocation after warm-up), and on
    completion the output becomes the state and the old buffer is returned.
    Evicted states go to pinned host memory and come back through
    asynchronous copies on a copy stream of their own, overlapped with the
    steps of resident simulations; a simulation joins a launch once its
    state is in place.  The initial state of simulation s (cubic L^3, 16^3
    blocks, periodic) is drawn on the device on first admission
    (``ics.served_state_device``).  Each launch is one batched step on the
    next of `nstreams` streams."""

    def __init__(self, sizes: Sequence[int], cfl: float = 0.8, nstreams: int = 2, device: str = "cuda",
                 seed: int = 3, nxb: int = 16):
        import torch

        from . import hydro

        self.torch = torch
        self.hydro = hydro
        self.sizes = list(sizes)
        self.cfl = cfl
        self.seed = seed
        self.nxb = nxb
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(nstreams)]
        self.copy_stream = torch.cuda.Stream(device=device)   # admissions, host -> device
        self.evict_stream = torch.cuda.Stream(device=device)  # evictions, device -> host
        self.next_stream = 0
        self.state: Dict[int, "torch.Tensor"] = {}
        self.grid: Dict[int, "hydro.Grid"] = {}
        self.host: Dict[int, tuple] = {}       # evicted: (host tensor, event of its copy or None, pool buffer)
        self.incoming: Dict[int, tuple] = {}   # admission copies in flight: (event, pool buffer)
        self.pool = PinnedPool(torch)
        self.steps_done = collections.Counter()
        self.host_s = collections.Counter()    # host seconds spent in each executor call
        self.moved = collections.Counter()     # state bytes copied "in" (host -> device) and "out"

    def shape_of(self, sim: int):
        nb = self.sizes[sim] // self.nxb
        return (nb ** 3, 5, self.nxb, self.nxb, self.nxb)

    def cells_of(self, sim: int) -> int:
        return self.sizes[sim] ** 3

    def bytes_of(self, sim: int) -> int:
        return 40 * self.cells_of(sim) + 256

    def is_resident(self, sim: int) -> bool:
        return sim in self.state

    def is_ready(self, sim: int) -> bool:
        if sim not in self.state:
            return False
        inc = self.incoming.get(sim)
        if inc is None:
            return True
        if inc[0].query():
            del self.incoming[sim]
            self.pool.put(inc[1])
            return True
        return False

    def make_resident(self, sim: int) -> None:
        t = time.perf_counter()
        try:
            return self._make_resident(sim)
        finally:
            self.host_s["make_resident"] += time.perf_counter() - t

    def _make_resident(self, sim: int) -> None:
        from . import ics

        torch = self.torch
        t = torch.empty(self.shape_of(sim), dtype=torch.float64, device=self.device)
        if sim in self.host:
            h, evicted, buf = self.host.pop(sim)
            self.moved["in"] += t.numel() * t.element_size()
            if buf is None:                            # pageable fallback: synchronous copy
                t.copy_(h)
            else:
                cs = self.copy_stream
                cs.wait_stream(torch.cuda.current_stream())  # t's memory may still be in use there
                cs.wait_event(evicted)                 # the eviction copy has filled h
                with torch.cuda.stream(cs):
                    t.copy_(h, non_blocking=True)
                t.record_stream(cs)
                ev = torch.cuda.Event()
                ev.record(cs)
                self.incoming[sim] = (ev, buf)
        else:
            ics.served_state_device(sim, self.sizes[sim], out=t, seed=self.seed, n=self.nxb)
        self.state[sim] = t

    def evict(self, sim: int) -> None:
        t = time.perf_counter()
        try:
            return self._evict(sim)
        finally:
            self.host_s["evict"] += time.perf_counter() - t

    def _evict(self, sim: int) -> None:
        torch = self.torch
        t = self.state.pop(sim)
        inc = self.incoming.pop(sim, None)
        cs = self.evict_stream
        if inc is not None:
            inc[0].synchronize()                       # its admission copy has to land first
            self.pool.put(inc[1])
        buf = self.pool.get(t.numel() * t.element_size())
        self.moved["out"] += t.numel() * t.element_size()
        if buf is None:                                # pool exhausted: pageable, synchronous
            torch.cuda.current_stream().synchronize()
            self.host[sim] = (t.cpu(), None, None)
            return
        h = buf.view(t.dtype).view(t.shape)
        cs.wait_stream(torch.cuda.current_stream())    # the state's last step has finished there
        with torch.cuda.stream(cs):
            h.copy_(t, non_blocking=True)
        t.record_stream(cs)                            # the allocator reuses t after the copy
        ev = torch.cuda.Event()
        ev.record(cs)
        self.host[sim] = (h, ev, buf)

    def current_state(self, sim: int) -> np.ndarray:
        if sim in self.state:
            self.copy_stream.synchronize()
            self.evict_stream.synchronize()
            return self.state[sim].cpu().numpy()
        h, ev, _ = self.host[sim]
        if ev is not None:
            ev.synchronize()
        return h.numpy().copy()

    def launch(self, sims: Sequence[int]):
        t = time.perf_counter()
        try:
            return self._launch(sims)
        finally:
            self.host_s["launch"] += time.perf_counter() - t

    def _launch(self, sims: Sequence[int]):
        torch = self.torch
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        grids, outs, spent = [], [], []
        for x in sims:
            inc = self.incoming.pop(x, None)
            if inc is not None:
                s.wait_event(inc[0])
                spent.append(inc[1])  # back to the pool once this launch is done
            st = self.state[x]
            out = torch.empty_like(st)
            G = self.grid.get(x)
            if G is None:
                L = self.sizes[x]
                nb = L // self.nxb
                G = self.hydro.Grid(self.nxb, (nb, nb, nb), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (0, 0, 0), 1.4,
                                    1e-10, device=self.device, buffers=(st, out))
                self.grid[x] = G
            else:
                G.set_buffers(st, out)
            grids.append(G)
            outs.append(out)
        s.wait_stream(torch.cuda.current_stream())
        B = self.hydro.Batch(grids, stream=s)
        B.step(self.cfl, 1)
        ev = torch.cuda.Event()
        ev.record(s)
        B.close()  # host metadata; the device work list stays alive in the handle
        for x in sims:
            self.steps_done[x] += 1
        return (ev, B.work, list(sims), outs, spent)

    def done(self, handle) -> bool:
        return handle[0].query()

    def settle(self) -> None:
        self.copy_stream.synchronize()
        self.evict_stream.synchronize()
        for ev, buf in self.incoming.values():
            self.pool.put(buf)
        self.incoming.clear()

    def close(self) -> None:
        """Release every device state, grid handle and pinned buffer."""
        self.torch.cuda.synchronize()
        for G in self.grid.values():
            G.close()
        self.grid.clear()
        self.state.clear()
        self.host.clear()
        self.incoming.clear()
        self.pool = PinnedPool(self.torch)

    def finish(self, handle) -> None:
        t = time.perf_counter()
        try:
            return self._finish(handle)
        finally:
            self.host_s["finish"] += time.perf_counter() - t

    def _finish(self, handle) -> None:
        ev, _, sims, outs, spent = handle
        self.torch.cuda.current_stream().wait_event(ev)
        for buf in spent:
            self.pool.put(buf)
        for x, out in zip(sims, outs):
            self.state[x] = out  # the old state buffer returns to the allocator ...
            self.grid[x].release_buffers()  # ... once the handle's wrapper lets go of it too
