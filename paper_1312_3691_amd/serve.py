"""Continuous-batching request loop for drag queries (serving row of the path).

Requests (mesh, query) arrive at any time.  A request is admitted into a free
slot when its per-triangle tally fits the device memory budget (first-fit over
a pool of int64 words; requests that keep only totals need none); each step is
one persistent launch (``tpmc_server_step``) over every active slot, each
getting a share of the step's tile budget, so requests of different meshes and
sizes run together on the device; a request finishes when all its tiles have
been traced, its result is read and its slot and pool words are freed for the
next arrivals.  Integer tallies make each result independent of how its tiles
were spread over steps and of the requests it shared them with.

The loop is pipelined so that the device does not wait for the host: after
step k is enqueued, the results of the requests it completes are enqueued for
collection, and only then are the results of step k - 1 read (they were ready
when step k started), their slots freed and new requests admitted (all
admissions of a step in one call) -- all while step k runs.

The policy lives here; the device work is behind an executor so the policy can
be tested on the CPU (``tests/test_serve_cpu.py``) with a fake executor.
"""
from __future__ import annotations

import asyncio
import time
from dataclasses import dataclass, field


class PoolAllocator:
    """First-fit allocator over [0, capacity) int64 words."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free_list = [(0, self.capacity)] if capacity > 0 else []

    def alloc(self, n: int):
        if n == 0:
            return 0
        for i, (off, size) in enumerate(self.free_list):
            if size >= n:
                if size == n:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + n, size - n)
                return off
        return None

    def free(self, off: int, n: int):
        if n == 0:
            return
        self.free_list.append((off, n))
        self.free_list.sort()
        merged = []
        for o, s in self.free_list:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free_list = merged

    @property
    def free_words(self) -> int:
        return sum(s for _, s in self.free_list)


@dataclass
class Request:
    rid: int
    mesh: str
    query: dict
    t_arrival: float
    future: asyncio.Future
    words: int = 0
    tiles: int = 0
    slot: int = -1
    offset: int = 0
    next_tile: int = 0
    t_admit: float = 0.0


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    latency_ids: list = field(default_factory=list)  # request id of each latency
    admitted: int = 0
    rejected: int = 0
    failed: int = 0
    cancelled: int = 0
    steps: int = 0
    tiles: int = 0
    hits: int = 0
    max_active: int = 0


class Executor:
    """Device side of the loop (see GpuExecutor).  admit_many, collect and
    collected default to admit and results, one call each."""

    def tally_words(self, mesh: str, query: dict) -> int:
        raise NotImplementedError

    def validate(self, mesh: str, query: dict) -> None:
        """Raise for a request that admission would refuse (default: none)."""

    def admit(self, slot: int, mesh: str, query: dict, offset: int) -> int:
        raise NotImplementedError

    def admit_many(self, items) -> list:
        """items: (slot, mesh, query, offset) each; returns the tile counts.
        All or nothing: on an error the ones admitted before it are released."""
        tiles = []
        try:
            for it in items:
                tiles.append(self.admit(*it))
        except Exception:
            for it in items[:len(tiles)]:
                self.release(it[0])
            raise
        return tiles

    def step(self, entries) -> None:
        raise NotImplementedError

    def results(self, slots) -> list:
        raise NotImplementedError

    def collect(self, slots):
        """Enqueue the results of these slots; returns a ticket for collected."""
        return self.results(slots)

    def collected(self, ticket) -> list:
        return ticket

    def release(self, slot: int) -> None:
        raise NotImplementedError


class GpuExecutor(Executor):
    """libtpmc server over resident meshes ({name: tpmc.Mesh})."""

    def __init__(self, ctx, meshes: dict, max_slots: int, pool_words: int, x_ref=(0.0, 0.0, 0.0), A_ref=1.0):
        from . import tpmc
        self.meshes = meshes
        self.server = tpmc.Server(ctx, max_slots, pool_words)
        self.x_ref, self.A_ref = x_ref, A_ref

    def tally_words(self, mesh, query):
        return 0 if int(query.get("flags", 0)) & 1 else 7 * self.meshes[mesh].nt

    def validate(self, mesh, query):
        from . import tpmc
        tpmc.check_query(query, self.meshes[mesh].V)

    def admit(self, slot, mesh, query, offset):
        return self.server.admit(slot, self.meshes[mesh], query, offset)

    def admit_many(self, items):
        return self.server.admit_many([(slot, self.meshes[mesh], q, off) for slot, mesh, q, off in items])

    def step(self, entries):
        self.server.step(entries)

    def results(self, slots):
        return self.server.results(slots, self.x_ref, self.A_ref)

    def collect(self, slots):
        return self.server.collect(slots, self.x_ref, self.A_ref)

    def collected(self, ticket):
        return self.server.collected(ticket)

    def release(self, slot):
        self.server.release(slot)


class Scheduler:
    """Admission by slot and memory budget, tile-budgeted steps, completion."""

    def __init__(self, executor: Executor, max_slots: int, pool_words: int, tiles_per_step: int,
                 clock=time.perf_counter):
        self.ex = executor
        self.max_slots = int(max_slots)
        self.pool = PoolAllocator(pool_words)
        self.tiles_per_step = int(tiles_per_step)
        self.clock = clock
        self.queue: list[Request] = []
        self.active: dict[int, Request] = {}
        self.free_slots = list(range(self.max_slots))
        self.stats = Stats()
        self._next_id = 0
        self._wake = None
        self.pending = None  # (ticket, requests) of the last step's collection, not yet read

    # -- client side -------------------------------------------------------
    def submit(self, mesh: str, query: dict, t_arrival: float | None = None) -> asyncio.Future:
        """Queue a request; its latency counts from t_arrival (default: now),
        so a load generator can pass the scheduled arrival time."""
        loop = asyncio.get_event_loop()
        fut = loop.create_future()
        req = Request(self._next_id, mesh, dict(query), self.clock() if t_arrival is None else t_arrival, fut)
        self._next_id += 1
        try:
            req.words = self.ex.tally_words(mesh, query)
        except Exception as e:  # unknown mesh and the like: fails this request only
            fut.set_exception(e)
            self.stats.failed += 1
            return fut
        if req.words > self.pool.capacity:
            fut.set_exception(MemoryError(f"request needs {req.words} tally words; the pool has "
                                          f"{self.pool.capacity}"))
            self.stats.rejected += 1
            return fut
        self.queue.append(req)
        if self._wake is not None:
            self._wake.set()
        return fut

    # -- device side -------------------------------------------------------
    def _admit(self):
        """Admit queued requests into free slots (FIFO; the head waits for memory),
        all of this round's admissions in one executor call."""
        picked = []
        while self.queue and len(picked) < len(self.free_slots):
            req = self.queue[0]
            if req.future.cancelled():
                self.queue.pop(0)
                self.stats.cancelled += 1
                continue
            try:
                self.ex.validate(req.mesh, req.query)
            except Exception as e:  # invalid query: fails this request only
                self.queue.pop(0)
                req.future.set_exception(e)
                self.stats.failed += 1
                continue
            off = self.pool.alloc(req.words)
            if off is None:  # head of line waits for memory (FIFO, no starvation of big requests)
                break
            self.queue.pop(0)
            req.slot, req.offset = self.free_slots[len(picked)], off
            picked.append(req)
        if not picked:
            return
        del self.free_slots[:len(picked)]
        items = [(r.slot, r.mesh, r.query, r.offset) for r in picked]
        try:
            tiles = self.ex.admit_many(items)
            outcome = [(r, t, None) for r, t in zip(picked, tiles)]
        except Exception:  # one of them was refused: admit one by one, failing only that one
            outcome = []
            for r, it in zip(picked, items):
                try:
                    outcome.append((r, self.ex.admit(*it), None))
                except Exception as e:
                    outcome.append((r, 0, e))
        now = self.clock()
        for r, t, err in outcome:
            if err is not None:
                self.pool.free(r.offset, r.words)
                self.free_slots.insert(0, r.slot)
                r.future.set_exception(err)
                self.stats.failed += 1
                continue
            r.tiles, r.t_admit = int(t), now
            self.active[r.slot] = r
            self.stats.admitted += 1
        self.stats.max_active = max(self.stats.max_active, len(self.active))

    def _retire(self, req: Request):
        self.ex.release(req.slot)
        self.pool.free(req.offset, req.words)
        self.free_slots.append(req.slot)
        del self.active[req.slot]

    def _finish(self, pending):
        """Read a collection enqueued after an earlier step and complete its requests."""
        ticket, done = pending
        try:
            res = self.ex.collected(ticket)
        except Exception as e:  # a device failure fails the requests it held
            res = [e] * len(done)
        now = self.clock()
        for r, out in zip(done, res):
            if isinstance(out, Exception):
                if not r.future.done():
                    r.future.set_exception(out)
                self.stats.failed += 1
            else:
                if not r.future.done():
                    r.future.set_result(out)
                self.stats.latencies_ms.append((now - r.t_arrival) * 1e3)
                self.stats.latency_ids.append(r.rid)
                self.stats.hits += int(out.get("hits", 0)) if isinstance(out, dict) else 0
            self._retire(r)

    def _entries(self, reqs):
        """Share the tile budget: equal shares, remainder to the oldest requests."""
        budget = self.tiles_per_step
        share = max(1, budget // len(reqs))
        entries = []
        for r in reqs:
            left = r.tiles - r.next_tile
            take = min(left, share, budget)
            if take > 0:
                entries.append((r.slot, r.next_tile, take))
                budget -= take
        for r in reqs:  # leftover budget
            if budget <= 0:
                break
            e = next((k for k, en in enumerate(entries) if en[0] == r.slot), None)
            used = entries[e][2] if e is not None else 0
            more = min(r.tiles - r.next_tile - used, budget)
            if more > 0:
                if e is None:
                    entries.append((r.slot, r.next_tile, more))
                else:
                    entries[e] = (r.slot, entries[e][1], used + more)
                budget -= more
        return entries

    def step_once(self) -> bool:
        """Admit, enqueue one step and the collection of the requests it
        completes, then complete the requests of the previous step's
        collection.  False when idle."""
        self._admit()
        in_flight = set(id(r) for r in self.pending[1]) if self.pending else set()
        for slot, req in list(self.active.items()):
            if req.future.cancelled() and id(req) not in in_flight:
                self.stats.cancelled += 1
                self._retire(req)
        reqs = sorted((r for r in self.active.values() if r.next_tile < r.tiles), key=lambda r: r.rid)
        new_pending = None
        if reqs:
            entries = self._entries(reqs)
            try:
                self.ex.step(entries)
            except Exception as e:  # a device failure fails every request of the step
                for r in reqs:
                    if not r.future.done():
                        r.future.set_exception(e)
                    self.stats.failed += 1
                    self._retire(r)
                entries = []
            if entries:
                self.stats.steps += 1
                for slot, t0, n in entries:
                    self.active[slot].next_tile += n
                    self.stats.tiles += n
                done = [r for r in reqs if r.next_tile >= r.tiles]
                if done:
                    try:
                        new_pending = (self.ex.collect([r.slot for r in done]), done)
                    except Exception as e:
                        for r in done:
                            if not r.future.done():
                                r.future.set_exception(e)
                            self.stats.failed += 1
                            self._retire(r)
        if self.pending is not None:
            self._finish(self.pending)
        self.pending = new_pending
        return bool(reqs) or self.pending is not None or bool(self.queue)

    async def run(self, stop: asyncio.Event | None = None):
        """Step while there is work; sleep until a submit when idle."""
        self._wake = asyncio.Event()
        while True:
            busy = self.step_once()
            if busy:
                await asyncio.sleep(0)
                continue
            if stop is not None and stop.is_set():
                return
            self._wake.clear()
            waiter = asyncio.ensure_future(self._wake.wait())
            stopper = asyncio.ensure_future(stop.wait()) if stop is not None else None
            await asyncio.wait([w for w in (waiter, stopper) if w is not None], return_when=asyncio.FIRST_COMPLETED)
            for w in (waiter, stopper):
                if w is not None and not w.done():
                    w.cancel()

    def percentiles(self, skip: int = 0):
        """p50 / p99 latency (ms) of the completed requests, leaving out the
        first `skip` submitted (warm-up)."""
        import numpy as np
        lat = [ms for ms, rid in zip(self.stats.latencies_ms, self.stats.latency_ids) if rid >= skip]
        if not lat:
            return None, None
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
