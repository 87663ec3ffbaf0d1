"""Launch autotuner for the persistent batched kernel.

The three launch parameters of the persistent launches (tpmc_set_tuning) -- refill_lanes
(how few lanes of a wave may still be traversing before the lanes whose ray
segment ended are served together), tile_particles (particles per work tile
a workgroup claims) and groups_per_cu (persistent workgroups per compute unit)
-- change only speed: particles are independent (Sec. II.A), each draws from
its own counter-based stream, and all sums are exact integers, so every
setting returns bit-identical results.  The best setting depends on the mesh
(tree depth, hit rate) and on the query mix, so it is measured: a coordinate
search over the candidate values on the caller's own workload, each candidate
timed with device events around replays of its launch.  By default the whole
workload is timed: in a shorter launch the tail (the last tiles finishing
while most workgroups idle) weighs more and favours smaller tiles than a full
launch does.

The search logic (`coordinate_search`) is plain Python over a cost function,
so it is tested without a GPU; `tune` supplies the cost from the device.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, Iterable, List, Sequence, Tuple

# candidate values, searched in this order (one coordinate at a time)
REFILL = (16, 24, 32, 40, 48)
TILE = (4096, 16384, 65536)
GROUPS = (4, 8, 16)
DEFAULT = {"refill_lanes": 32, "tile_particles": 16384, "groups_per_cu": 8}
AXES: Tuple[Tuple[str, Sequence[int]], ...] = (("refill_lanes", REFILL), ("tile_particles", TILE),
                                              ("groups_per_cu", GROUPS))


@dataclasses.dataclass
class Trial:
    tuning: Dict[str, int]
    ms: float


def coordinate_search(cost: Callable[[Dict[str, int]], float], start: Dict[str, int] = None,
                      axes: Iterable[Tuple[str, Sequence[int]]] = AXES, rounds: int = 1) -> Tuple[Dict[str, int], List[Trial]]:
    """Minimise cost(tuning) one axis at a time, starting from `start`.
    Each distinct setting is measured once; ties keep the earlier setting."""
    best = dict(DEFAULT if start is None else start)
    seen: Dict[Tuple[Tuple[str, int], ...], float] = {}
    trials: List[Trial] = []

    def measure(t: Dict[str, int]) -> float:
        key = tuple(sorted(t.items()))
        if key not in seen:
            seen[key] = float(cost(dict(t)))
            trials.append(Trial(dict(t), seen[key]))
        return seen[key]

    best_ms = measure(best)
    axes = list(axes)
    for _ in range(max(1, rounds)):
        changed = False
        for name, values in axes:
            for v in values:
                if v == best[name]:
                    continue
                cand = dict(best)
                cand[name] = v
                ms = measure(cand)
                if ms < best_ms:
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    return best, trials


def sample_queries(queries: Sequence[dict], particles: int) -> List[dict]:
    """The caller's queries with the total particle count cut to about
    `particles` (kept in proportion, at least 4096 each unless smaller)."""
    total = sum(int(q["n"]) for q in queries)
    if total <= particles:
        return [dict(q) for q in queries]
    f = particles / total
    return [dict(q, n=min(int(q["n"]), max(4096, int(q["n"] * f)))) for q in queries]


def free_axes(fixed: Dict[str, int] = None) -> List[Tuple[str, Sequence[int]]]:
    """The search axes without the settings held in `fixed`."""
    fixed = fixed or {}
    unknown = set(fixed) - {name for name, _ in AXES} - {"plain_groups_per_cu"}
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    return [(name, values) for name, values in AXES if name not in fixed]


def tune(mesh, queries: Sequence[dict], particles: int = None, reps: int = 1,
         check_results: bool = True, fixed: Dict[str, int] = None) -> Tuple[Dict[str, int], List[Trial]]:
    """Measure the batched launch of `queries` (reduced to about `particles`
    when given) on `mesh` under candidate tunings, set the fastest on the
    mesh's context and return it with every trial.  With check_results, every
    candidate's results must equal the first one's bit for bit (TpmcError
    otherwise).  Settings in `fixed` are held and not searched."""
    import torch

    from . import tpmc

    ctx = mesh.ctx
    sample = [dict(q) for q in queries] if particles is None else sample_queries(queries, particles)
    ref: List = []

    def cost(t: Dict[str, int]) -> float:
        ctx.set_tuning(**t)
        b = tpmc.Batch(mesh, sample)
        try:
            b.launch(use_graph=True)  # capture + first run
            torch.cuda.synchronize()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(reps):
                b.launch(use_graph=True)
            stop.record()
            stop.synchronize()
            ms = start.elapsed_time(stop) / reps
            if check_results:
                key = [(r["CD"], r["hits"], r["segments"]) for r in b.results()]
                if not ref:
                    ref.append(key)
                elif key != ref[0]:
                    raise tpmc.TpmcError(5, f"tuning {t} changed the results")
        finally:
            b.close()
        return ms

    fixed = dict(fixed or {})
    best, trials = coordinate_search(cost, start=dict(ctx.tuning, **fixed), axes=free_axes(fixed))
    ctx.set_tuning(**best)
    return best, trials
