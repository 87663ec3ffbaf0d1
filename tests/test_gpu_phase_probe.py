"""The phase-probe library (libtpmc_probe.so: the batched kernel with shader
clock reads and pass counters compiled in, read through tpmc_phase_probe).

* Instrumenting changes nothing computed: batched results from the probe
  library equal the ordinary library's bit for bit (every field but the work
  count that depends on launch timing), on a plate
  (per-lane LDS tallies), the capped cylinder (workgroup LDS tallies) and a
  satellite with per-query totals.
* Its counts obey the kernel's own bookkeeping: every particle passes the
  estimate once, every survivor is seeded exactly, the particles the estimate
  removes are the result's pre-culled count, every particle queued after its
  root test is handed to a lane, no pass runs with more than 64 or fewer than
  one lane, and the phases' cycles add up to no more than the waves' lives.

The probe library is selected at import (TPMC_PHASE_PROBE=1), so it runs in a
child process; this process runs the ordinary library.
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = r"""
from paper_1312_3691_amd import inputs as I


def cases():
    quats = I.random_quats(4, 5)
    plate = [I.query(q=tuple(quats[k]), S=s, alpha=a, n=300_000, seed=k) for k, (s, a) in
             enumerate(((5.0, 1.0), (2.0, 0.0), (10.0, 0.5)))]
    cyl = [I.query(q=tuple(quats[k]), S=s, alpha=0.9, n=300_000, seed=10 + k, max_reflections=16)
           for k, s in enumerate((1.0, 3.0, 7.0, 0.0))]
    sat = [I.query(q=tuple(quats[k]), S=s, alpha=0.9, n=400_000, seed=20 + k, flags=1, max_reflections=16)
           for k, s in enumerate((4.0, 9.0))]
    return [("plate", I.plate(), plate), ("cylinder", I.capped_cylinder(), cyl),
            ("satellite", I.satellite(4000), sat)]


def run(tpmc, with_probe):
    ctx = tpmc.Context(0)
    out = {}
    for name, (V, T), qs in cases():
        mesh = ctx.build_mesh(V, T)
        b = tpmc.Batch(mesh, qs)
        if with_probe:
            ctx.phase_probe(reset=True)
        b.launch()
        res = [{k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in r.items()} for r in b.results()]
        out[name] = {"results": res, "probe": ctx.phase_probe(reset=True) if with_probe else None,
                     "stack_slots": mesh.info["stack_slots"]}
        b.close()
        mesh.close()
    return out
"""

CHILD = CASES + r"""
import json
import torch  # noqa: F401
from paper_1312_3691_amd import tpmc
assert tpmc.PHASE_PROBE and tpmc.LIB_PATH.endswith("libtpmc_probe.so")
print("PROBE_JSON " + json.dumps(run(tpmc, True)), flush=True)
"""


@pytest.fixture(scope="module")
def runs():
    env = dict(os.environ, TPMC_PHASE_PROBE="1", PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    print("phase probe: child process with libtpmc_probe.so", flush=True)
    cp = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True, text=True,
                        timeout=110)
    assert cp.returncode == 0, cp.stdout[-2000:] + cp.stderr[-4000:]
    line = [ln for ln in cp.stdout.splitlines() if ln.startswith("PROBE_JSON ")][-1]
    probed = json.loads(line[len("PROBE_JSON "):])
    from paper_1312_3691_amd import tpmc
    assert not tpmc.PHASE_PROBE
    ns = {}
    exec(compile(CASES, "cases", "exec"), ns)
    plain = ns["run"](tpmc, False)
    return probed, plain


def _same(a, b):
    if isinstance(a, list) and isinstance(b, list):
        return len(a) == len(b) and all(_same(x, y) for x, y in zip(a, b))
    return a == b or (isinstance(a, float) and isinstance(b, float) and a != a and b != b)  # NaN (S = 0) fields


@pytest.mark.parametrize("name", ["plate", "cylinder", "satellite"])
def test_probe_library_gives_identical_results(runs, name):
    from paper_1312_3691_amd import tpmc
    probed, plain = runs
    assert len(probed[name]["results"]) == len(plain[name]["results"])
    for a, b in zip(probed[name]["results"], plain[name]["results"]):
        for k in b:
            if k in tpmc.WORK_COUNTS:  # how much work the estimate saved depends on launch timing
                continue
            assert _same(a[k], b[k]), (name, k, a[k], b[k])


@pytest.mark.parametrize("name", ["plate", "cylinder", "satellite"])
def test_probe_counts_match_the_kernels_bookkeeping(runs, name):
    probed, _ = runs
    p, res = probed[name]["probe"], probed[name]["results"]
    n = sum(r["rays"] for r in res)
    two_stage = probed[name]["stack_slots"] <= 32
    print(name, json.dumps(p), flush=True)
    assert p["waves"] > 0 and p["waves"] % 4 == 0
    for passes, lanes in (("trav_steps", "trav_lanes"), ("leaf_passes", "leaf_lanes"), ("serves", "serve_lanes"),
                          ("est_batches", "est_particles"), ("seed_batches", "seed_particles"),
                          ("assigns", "assign_lanes")):
        assert p[passes] <= p[lanes] <= 64 * p[passes], (passes, p[passes], p[lanes])
    if two_stage:
        assert p["est_particles"] == n
        assert p["est_kept"] == p["seed_particles"]
        assert sum(r["preculled"] for r in res) == p["est_particles"] - p["est_kept"]
    else:
        assert p["est_batches"] == 0 and p["seed_particles"] == n
    assert p["seed_kept"] == p["assign_lanes"] <= p["seed_particles"]
    hits, segments = sum(r["hits"] for r in res), sum(r["segments"] for r in res)
    assert hits <= p["serve_lanes"] <= segments
    phases = sum(p[k] for k in ("claim_cycles", "trav_cycles", "leaf_cycles", "serve_cycles", "est_cycles",
                                "seed_cycles", "assign_cycles"))
    assert 0 < phases <= p["cycles"], (phases, p["cycles"])
