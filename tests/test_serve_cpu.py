"""Serving policy on the CPU: a fake executor stands in for the device.

The fake result of a request is a function of exactly which tiles were traced
for it, so a request whose tiles were dropped, duplicated or mixed with another
request's gives a different value."""
import asyncio
import random

import pytest

from paper_1312_3691_amd.serve import PoolAllocator, Scheduler, Executor

TILE = 4096


class FakeExecutor(Executor):
    def __init__(self, mesh_tris, fail_admit_seed=None, fail_step_at=None, step_delay=0.0):
        self.mesh_tris = mesh_tris
        self.step_delay = step_delay
        self.slots = {}
        self.fail_admit_seed = fail_admit_seed
        self.fail_step_at = fail_step_at
        self.steps = 0
        self.max_entries = 0
        self.mixed_steps = 0

    def tally_words(self, mesh, query):
        return 0 if query.get("flags", 0) & 1 else 7 * self.mesh_tris[mesh]

    def admit(self, slot, mesh, query, offset):
        if query["seed"] == self.fail_admit_seed:
            raise ValueError("invalid query")
        assert slot not in self.slots
        self.slots[slot] = dict(seed=query["seed"], n=query["n"], seen=[], offset=offset, mesh=mesh)
        return (query["n"] + TILE - 1) // TILE

    def step(self, entries):
        if self.step_delay:
            import time
            time.sleep(self.step_delay)
        self.steps += 1
        if self.fail_step_at == self.steps:
            raise RuntimeError("device fault")
        self.max_entries = max(self.max_entries, len(entries))
        if len({self.slots[s]["mesh"] for s, _, _ in entries}) > 1:
            self.mixed_steps += 1
        for slot, t0, n in entries:
            self.slots[slot]["seen"] += list(range(t0, t0 + n))

    def results(self, slots):
        out = []
        for s in slots:
            d = self.slots[s]
            out.append(dict(value=solo_value(d["seed"], d["n"]) if sorted(d["seen"]) == list(
                range((d["n"] + TILE - 1) // TILE)) else -1, hits=len(d["seen"])))
        return out

    def release(self, slot):
        del self.slots[slot]


def solo_value(seed, n):
    return sum((seed * 1000003 + t) % 997 for t in range((n + TILE - 1) // TILE))


def _req(seed, n, flags=0):
    return dict(seed=seed, n=n, flags=flags, q=(1, 0, 0, 0), S=5.0, T_inf=1000.0, T_w=300.0, alpha=1.0)


def _run(sched, reqs):
    async def main():
        stop = asyncio.Event()
        runner = asyncio.ensure_future(sched.run(stop))
        futs = []
        for mesh, q, delay in reqs:
            if delay:
                await asyncio.sleep(delay)
            futs.append(sched.submit(mesh, q))
        res = await asyncio.gather(*futs, return_exceptions=True)
        stop.set()
        sched._wake.set()
        await runner
        return res
    return asyncio.run(main())


def test_allocator_first_fit_and_merge():
    p = PoolAllocator(100)
    a = p.alloc(30)
    b = p.alloc(30)
    c = p.alloc(30)
    assert (a, b, c) == (0, 30, 60) and p.alloc(20) is None
    p.free(b, 30)
    assert p.alloc(40) is None and p.alloc(25) == 30
    p.free(a, 30)
    p.free(30, 25)
    assert p.alloc(55) == 0
    assert p.free_words == 100 - 55 - 30


def test_every_tile_exactly_once_and_results_equal_solo():
    ex = FakeExecutor({"small": 1000, "big": 50000})
    sched = Scheduler(ex, max_slots=4, pool_words=7 * 60000, tiles_per_step=64)
    rng = random.Random(1)
    reqs = []
    for i in range(40):
        mesh = rng.choice(["small", "big"])
        n = int(10 ** rng.uniform(3, 6.3))
        reqs.append((mesh, _req(i, n, flags=rng.choice([0, 1])), rng.choice([0, 0, 0.0005])))
    res = _run(sched, reqs)
    for (mesh, q, _), r in zip(reqs, res):
        assert r["value"] == solo_value(q["seed"], q["n"])
    assert sched.stats.admitted == 40 and not sched.active and ex.max_entries > 1
    assert ex.mixed_steps > 0  # requests on different meshes shared launches
    p50, p99 = sched.percentiles()
    assert p50 is not None and p99 >= p50


def test_memory_budget_admission_and_rejection():
    ex = FakeExecutor({"m": 1000})
    sched = Scheduler(ex, max_slots=8, pool_words=7 * 1000 * 2, tiles_per_step=8)
    reqs = [("m", _req(i, 50_000), 0) for i in range(6)]
    res = _run(sched, reqs)
    assert all(r["value"] == solo_value(i, 50_000) for i, r in enumerate(res))
    assert sched.stats.max_active == 2  # only two per-triangle tallies fit at once
    ex2 = FakeExecutor({"huge": 10_000})
    sched2 = Scheduler(ex2, max_slots=2, pool_words=100, tiles_per_step=8)
    res2 = _run(sched2, [("huge", _req(1, 1000), 0), ("huge", _req(2, 1000, flags=1), 0)])
    assert isinstance(res2[0], MemoryError) and res2[1]["value"] == solo_value(2, 1000)
    assert sched2.stats.rejected == 1


def test_failed_admission_fails_only_that_request():
    ex = FakeExecutor({"m": 10}, fail_admit_seed=3)
    sched = Scheduler(ex, max_slots=2, pool_words=1000, tiles_per_step=4)
    res = _run(sched, [("m", _req(i, 20_000), 0) for i in range(6)])
    for i, r in enumerate(res):
        if i == 3:
            assert isinstance(r, ValueError)
        else:
            assert r["value"] == solo_value(i, 20_000)
    assert sched.stats.failed == 1


def test_unknown_mesh_fails_only_that_request():
    ex = FakeExecutor({"m": 10})
    sched = Scheduler(ex, max_slots=2, pool_words=1000, tiles_per_step=4)
    res = _run(sched, [("m", _req(0, 9000), 0), ("nope", _req(1, 9000), 0), ("m", _req(2, 9000), 0)])
    assert isinstance(res[1], KeyError) and res[0]["value"] == solo_value(0, 9000)


def test_device_failure_fails_active_requests_then_recovers():
    ex = FakeExecutor({"m": 10}, fail_step_at=2)
    sched = Scheduler(ex, max_slots=2, pool_words=1000, tiles_per_step=2)
    res = _run(sched, [("m", _req(i, 40_000), 0) for i in range(4)])
    assert sum(isinstance(r, RuntimeError) for r in res) == 2
    assert sum(isinstance(r, dict) and r["value"] == solo_value(i, 40_000) for i, r in enumerate(res)) == 2
    assert not sched.active and sched.pool.free_words == 1000


def test_cancellation_frees_the_slot():
    ex = FakeExecutor({"m": 10}, step_delay=0.002)
    sched = Scheduler(ex, max_slots=1, pool_words=1000, tiles_per_step=1)

    async def main():
        stop = asyncio.Event()
        runner = asyncio.ensure_future(sched.run(stop))
        f1 = sched.submit("m", _req(1, 4096 * 50))
        f2 = sched.submit("m", _req(2, 4096 * 3))
        await asyncio.sleep(0.01)
        f1.cancel()
        r2 = await f2
        stop.set()
        sched._wake.set()
        await runner
        return r2
    r2 = asyncio.run(main())
    assert r2["value"] == solo_value(2, 4096 * 3)
    assert sched.stats.cancelled == 1 and not sched.active


class PipelineLog(FakeExecutor):
    """Records the order of device calls: collection tickets are read only
    after the following step has been enqueued, admissions come in groups."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.calls = []
        self.tickets = 0
        self.held = {}

    def admit_many(self, items):
        self.calls.append(("admit_many", len(items)))
        return super().admit_many(items)

    def step(self, entries):
        self.calls.append(("step", len(entries)))
        super().step(entries)

    def collect(self, slots):
        self.tickets += 1
        self.held[self.tickets] = self.results(slots)
        self.calls.append(("collect", self.tickets))
        return self.tickets

    def collected(self, ticket):
        self.calls.append(("collected", ticket))
        return self.held.pop(ticket)


def test_pipelined_steps_and_grouped_admission():
    ex = PipelineLog({"m": 100})
    sched = Scheduler(ex, max_slots=8, pool_words=7 * 100 * 8, tiles_per_step=6)
    reqs = [("m", _req(i, 4096 * (1 + i % 5)), 0) for i in range(30)]
    res = _run(sched, reqs)
    assert all(r["value"] == solo_value(i, 4096 * (1 + i % 5)) for i, r in enumerate(res))
    seq = ex.calls
    # every collection is read after the next step (or, at the end, after the last one) was enqueued
    for k, c in enumerate(seq):
        if c[0] == "collected":
            j = seq.index(("collect", c[1]))
            later_steps = [x for x in seq[j + 1:k] if x[0] == "step"]
            assert later_steps or not any(x[0] == "step" for x in seq[k:]), (c, seq[j:k + 1])
    assert max(n for name, n in seq if name == "admit_many") > 1
    assert not ex.held and sched.pending is None
