"""Benchmark: particle-surface hits per second on one MI355X.

Workload (one step): the flat-plate and capped-cylinder verification sweep --
a 1 x 1 m double-sided plate (2 triangles) and a 64-segment capped cylinder
(256 triangles), each at 10 incidence angles 0..90 deg, S in {1, 3, 8},
specular and diffuse (alpha = 1), T_inf = 1000 K, T_w = 300 K: 120 drag
queries.  Each case runs max(1e7, N_3sigma) particles, N_3sigma being the
count at which its 3-sigma relative C_D error falls to 1e-3 (estimated from a
seeded 1e6-particle pilot), so that every case meets the metric's accuracy.
Each mesh's 60 queries run as one persistent, graph-replayed batched launch;
inputs (meshes, BVHs, query tables) are resident on the GPU before the timed
region.

Also reported: each launch's duration (HIP events on its stream), work and
fraction of the ALU peak; the same 120 queries through the plain
one-query-per-launch path (seed -> trace -> forces, host sync per query) with
p50 / p99 query latency; C_D error of every case against the per-facet closed
form; the concave satellite (~50k triangles, 1e8 particles, one query) and the
1024-attitude sweep on it (one graph-replayed launch against the plain path);
the served stream (continuous batching over four resident satellite meshes:
saturation throughput, p50 / p99 latency at 0.8 of it -- the line's
query_ms_p50 / p99 -- and the FIFO plain path); and the CPU oracle on bounded
samples (all usable host threads and one).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain] [--no-satellite]
                    [--no-served]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-surface hits/sec on 1 MI355X at C_D error ≤1e-3; p50/p99 query ms"
T_INF, T_W = 1000.0, 300.0
N_PER_CASE = 10_000_000
ALU_PEAK = 256 * 64 * 2.4e9  # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz (one VALU op per lane per clock)
# Algorithmic lane-operations per unit of work (one VALU operation per lane = 1).
OPS_SEED = 950.0   # per particle: 2 Philox blocks + FP64 inverse-CDF seeding + frame
OPS_NODE = 40.0    # per BVH node visit: two slab tests + stack
OPS_TRI = 45.0     # per watertight triangle test
OPS_HIT = 225.0    # per hit: Philox block + re-emission + tally
OPS_PRECULL = 485.0  # per particle the batched path's seeding estimate removes: 2 Philox blocks (250) + the
                     # FP32 normal-speed estimate, start and two Halley steps (105) + the latitude from the fine
                     # table (25) + frame, Box-Muller and angles (50) + grown two-box test (55), in place of
                     # OPS_SEED and the one root-node visit such a particle costs on the plain path
KERNEL_SOURCES = ["tpmc_device.hpp", "tpmc_math.hpp", "tpmc_kernels.hip", "tpmc_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cases(n=N_PER_CASE, n_case=None):
    """The 120 sweep cases (plate first); n_case gives each case's particle count."""
    from paper_1312_3691_amd import inputs as I
    out = []
    for kind, gen in (("plate", I.plate_cases), ("cylinder", I.cylinder_cases)):
        for i, c in enumerate(gen(n=n)):
            ni = int(n_case[len(out)]) if n_case is not None else n
            q = I.query(q=c["q"], S=c["S"], T_inf=T_INF, T_w=T_W, alpha=c["alpha"], n=ni,
                        seed=len(out), max_reflections=16)
            out.append(dict(kind=kind, angle=c["angle"], query=q))
    return out


CD_REL_MIN = 0.05      # below this |C_D| the accuracy criterion is absolute
N_CASE_MAX = 400_000_000


def case_particles(ctx, dev_mesh, n_floor, n_pilot):
    """Particles per case so that 3 sigma(C_D) <= 1e-3 |C_D|: a seeded pilot of
    n_pilot particles per case (plain path, untimed; its own seeds) gives each
    case's relative scatter per particle, sigma_rel sqrt(N); the case then runs
    max(n_floor, 1.25 N_needed) particles rounded up to a million (capped at
    N_CASE_MAX).  Cases with |C_D| <= CD_REL_MIN keep n_floor (absolute
    criterion: their sigma is far below 1e-3 there)."""
    from paper_1312_3691_amd import tpmc
    pilot = cases(int(n_pilot))
    for c in pilot:
        c["query"] = dict(c["query"], seed=c["query"]["seed"] + 1_000_000)
    res = []
    for kind in ("plate", "cylinder"):  # plain path: the batched kernel's dispatches stay the timed ones
        r, pr = tpmc.run(dev_mesh[kind], [c["query"] for c in pilot if c["kind"] == kind], A_ref=1.0)
        pr.close()
        res += r
    out = []
    for r in res:
        n = n_floor
        if abs(r["CD"]) > CD_REL_MIN and r["CD_sigma"] > 0:
            k = r["CD_sigma"] / abs(r["CD"]) * math.sqrt(n_pilot)
            need = 1.25 * (3.0 * k / 1e-3) ** 2
            n = int(min(N_CASE_MAX, max(n_floor, math.ceil(need / 1e6) * 1e6)))
        out.append(n)
    return out


def launch_ms(ctx, batch, tuning, reps):
    """Mean duration of one graph-replayed launch of `batch` (zeroing, persistent
    kernel, reduction), from HIP events recorded on the context's stream."""
    import torch
    if ctx.tuning != tuning:
        ctx.set_tuning(**tuning)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        batch.launch(use_graph=True)
        e1.record(ctx.stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.mean(ts))


def traversal_work(mesh, queries, n_sub=1_000_000):
    """BVH node visits and triangle tests per ray segment from the counting
    variant of the trace kernel on the first n_sub particles of each query."""
    import torch

    from paper_1312_3691_amd import tpmc
    nodes = tests = segs = 0
    for q in queries:
        qs = dict(q, n=min(n_sub, int(q["n"])))
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        pr = tpmc.PlainRun(mesh, [qs]).seed().trace(counters=cnt)
        r = pr.forces()[0]
        nodes += int(cnt[0])
        tests += int(cnt[1])
        segs += r["segments"]
        pr.close()
    return nodes / segs, tests / segs


TALLY_MODE = {"global": 0, "lds": 1, "lane": 2, "totals": 3}


def batch_instance(mesh, totals_only=False):
    """Template instance batch_kernel<stack slots, tally mode> a batch on `mesh` launches."""
    nt = mesh.nt
    mode = "totals" if totals_only else ("lane" if nt <= 2 else ("lds" if nt <= 512 else "global"))
    return f"batch_kernel<{mesh.info['stack_slots']}, {TALLY_MODE[mode]}>"


def launch_record(kernel, ms, results, V_seg, T_seg):
    """Work of one launch in algorithmic lane-operations (per-unit figures
    OPS_*) and its fraction of the one-op-per-lane-per-clock ALU peak."""
    particles = sum(r["rays"] for r in results)
    segments = sum(r["segments"] for r in results)
    hits = sum(r["hits"] for r in results)
    pre = sum(r.get("preculled", 0) for r in results)
    ops = ((particles - pre) * OPS_SEED + pre * OPS_PRECULL + segments * (V_seg * OPS_NODE + T_seg * OPS_TRI)
           - pre * OPS_NODE + hits * OPS_HIT)
    import re
    m = re.match(r"batch_kernel<[^>]*>", kernel)
    traffic = stored_traffic(m.group(0)) if m else None
    return {"kernel": kernel, "ms": ms, "achieved_tlane_ops": ops / (ms / 1e3) / 1e12, "hbm_bytes": traffic,
            "frac": ops / (ms / 1e3) / ALU_PEAK,
            "work": {"particles": particles, "preculled": pre, "segments": segments, "hits": hits,
                     "node_visits_per_segment": V_seg, "triangle_tests_per_segment": T_seg, "alg_lane_ops": ops}}


def plain_path(ctx, dev_mesh, cl, tunings):
    """The same queries through the plain path (seed -> trace -> forces, host
    sync per query) with latency percentiles, and as one-query batches."""
    from paper_1312_3691_amd import tpmc
    import torch
    lat = []
    p_hits = 0
    for c in cl[:2]:
        tpmc.run(dev_mesh[c["kind"]], [c["query"]])[1].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in cl:
        if ctx.tuning != tunings[c["kind"]]:
            ctx.set_tuning(**tunings[c["kind"]])
        t1 = time.perf_counter()
        r, pr = tpmc.run(dev_mesh[c["kind"]], [c["query"]])
        lat.append((time.perf_counter() - t1) * 1e3)
        p_hits += r[0]["hits"]
        pr.close()
    pdt = time.perf_counter() - t0
    plain = {"hits_per_s": p_hits / pdt, "s_per_step": pdt,
             "query_ms_p50": float(np.percentile(lat, 50)), "query_ms_p99": float(np.percentile(lat, 99))}
    lat_b = []
    for c in cl:
        if ctx.tuning != tunings[c["kind"]]:
            ctx.set_tuning(**tunings[c["kind"]])
        t1 = time.perf_counter()
        b1 = tpmc.Batch(dev_mesh[c["kind"]], [c["query"]])
        b1.launch(use_graph=False).results(A_ref=1.0)
        lat_b.append((time.perf_counter() - t1) * 1e3)
        b1.close()
    plain["single_query_batch_ms_p50"] = float(np.percentile(lat_b, 50))
    plain["single_query_batch_ms_p99"] = float(np.percentile(lat_b, 99))
    return plain


SAT_FLOW = (-0.5, 0.0, -math.sqrt(3.0) / 2.0)


def satellite_query(n, seed=0):
    from paper_1312_3691_amd import inputs as I
    return I.query(q=I.quat_for_flow(SAT_FLOW), S=7.0, T_inf=T_INF, T_w=T_W, alpha=0.9, n=int(n), seed=seed,
                   max_reflections=16)


def sweep_queries(n, nq=1024):
    from paper_1312_3691_amd import inputs as I
    quats = I.random_quats(nq, 1)
    S = 2.0 + 8.0 * np.random.default_rng(1).random(nq)
    return [I.query(q=tuple(quats[i]), S=float(S[i]), T_inf=T_INF, T_w=T_W, alpha=0.9, n=int(n), seed=i, flags=1)
            for i in range(nq)]


def config_satellite(ctx, args, measured):
    """Concave satellite (~50k triangles, S = 7, alpha = 0.9, 16 reflections,
    --particles-sat particles, one query) as one graph-replayed batched launch."""
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    V, T = I.satellite(50_000)
    t0 = time.perf_counter()
    mesh = ctx.build_mesh(V, T, builder=args.bvh)
    build_ms = (time.perf_counter() - t0) * 1e3
    q = satellite_query(args.particles_sat)
    tuning = tune_for(args, mesh, [q], key="satellite")
    b = tpmc.Batch(mesh, [q])
    b.launch().results()
    for _ in range(args.warmup):
        b.launch(use_graph=True).results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = b.launch(use_graph=True).results()[0]
    dt = (time.perf_counter() - t0) / args.steps
    assert r["tr_capped"] == 0 and r["guard_trips"] == 0
    ms = launch_ms(ctx, b, tuning, max(3, args.steps))
    b.close()
    V_seg, T_seg = traversal_work(mesh, [q])
    rec = launch_record(f"{batch_instance(mesh)} (satellite, {len(T)} tris, 1 query)", ms, [r], V_seg, T_seg)
    rec["frac_of_measured_fp32_fma"] = rec["achieved_tlane_ops"] / measured["fp32_fma"]
    return {"workload": f"concave satellite {len(T)} tris, S=7, alpha=0.9, {int(args.particles_sat):.3g} particles, "
                        "16 reflections", "hits_per_s": r["hits"] / dt, "ms_per_step": dt * 1e3,
            "segments_per_s": r["segments"] / dt, "CD": r["CD"], "CD_sigma": r["CD_sigma"],
            "three_sigma_rel": 3.0 * r["CD_sigma"] / abs(r["CD"]), "hits_per_particle": r["hits"] / r["rays"],
            "capped": r["capped"], "bvh_depth": mesh.info["depth"], "stack_slots": mesh.info["stack_slots"],
            "bvh_build_ms": build_ms, "tuning": tuning, "launch": rec, "mesh": mesh}


def config_sweep(ctx, args, measured, mesh):
    """1024 uniform-random attitudes x S ~ U[2, 10], --particles-sweep particles
    each, per-query totals, on the satellite: one graph-replayed persistent
    launch, against the plain path (one call per query, host sync) on the
    first 128 queries."""
    import torch

    from paper_1312_3691_amd import tpmc
    qs = sweep_queries(args.particles_sweep)
    tuning = tune_for(args, mesh, qs, key="sweep")
    b = tpmc.Batch(mesh, qs)
    b.launch().results()
    for _ in range(args.warmup):
        b.launch(use_graph=True).results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = b.launch(use_graph=True).results()
    dt = (time.perf_counter() - t0) / args.steps
    assert all(r["tr_capped"] == 0 and r["guard_trips"] == 0 for r in res)
    ms = launch_ms(ctx, b, tuning, max(3, args.steps))
    b.close()
    V_seg, T_seg = traversal_work(mesh, qs[::64], n_sub=200_000)
    rec = launch_record(f"{batch_instance(mesh, totals_only=True)} (satellite, {mesh.nt} tris, {len(qs)} queries)",
                        ms, res, V_seg, T_seg)
    rec["frac_of_measured_fp32_fma"] = rec["achieved_tlane_ops"] / measured["fp32_fma"]
    hits = sum(r["hits"] for r in res)
    k = 128
    tpmc.run(mesh, [qs[0]])[1].close()
    t1 = time.perf_counter()
    p_hits = 0
    lat = []
    for c in qs[:k]:
        t2 = time.perf_counter()
        r, pr = tpmc.run(mesh, [c])
        lat.append((time.perf_counter() - t2) * 1e3)
        p_hits += r[0]["hits"]
        pr.close()
    pdt = time.perf_counter() - t1
    same = all(a["CD"] == c["CD"] and a["hits"] == c["hits"] for a, c in zip(tpmc.run(mesh, qs[:4])[0], res[:4]))
    rel3 = [3.0 * r["CD_sigma"] / abs(r["CD"]) for r in res if abs(r["CD"]) > 0]
    return {"workload": f"satellite {mesh.nt} tris, {len(qs)} attitudes x S~U[2,10], "
                        f"{int(args.particles_sweep):.3g} particles each, per-query totals",
            "hits_per_s": hits / dt, "ms_per_step": dt * 1e3, "launch": rec,
            "plain_path": {"hits_per_s": p_hits / pdt, "queries_timed": k,
                           "query_ms_p50": float(np.percentile(lat, 50)),
                           "query_ms_p99": float(np.percentile(lat, 99))},
            "batched_over_plain": (hits / dt) / (p_hits / pdt), "first_queries_equal_plain": bool(same),
            "three_sigma_rel_median": float(np.median(rel3)), "tuning": tuning}


def meshes():
    from paper_1312_3691_amd import inputs as I
    return {"plate": I.plate(), "cylinder": I.capped_cylinder()}


EXACT_PATH = os.path.join(ROOT, "tests", "golden", "bench_cases_exact.json")


def exact_cd(kind, angle, S, alpha):
    """Per-facet exact C_D of a benchmark case (drag area, A_ref = 1 m^2), from the
    stored table tests/golden/bench_cases_exact.json (written from the closed
    forms by tests/golden/make_bench_exact.py)."""
    global _EXACT
    if "_EXACT" not in globals():
        _EXACT = {(e["kind"], e["angle"], e["S"], e["alpha"]): e["CD"] for e in json.load(open(EXACT_PATH))["cases"]}
    return _EXACT[(kind, float(angle), float(S), float(alpha))]


def kernel_hash():
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1312_3691_amd", "csrc", s), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(instance: str):
    """HBM bytes (fetched + written) of one launch of a batch_kernel template
    instance, measured with rocprofv3 counters (profiles/traffic.json); used
    only while the kernel sources are unchanged since the measurement."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get("batch_kernel", {}).get(instance)
        if e and d.get("kernel_hash") == kernel_hash():
            return float(e["fetch_bytes"] + e["write_bytes"])
    except Exception:
        return None
    return None


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(cases_kv, m, threads):
    """Oracle hits/s over the first m particles of each (V, T, query)."""
    from oracle import oracle as O
    hits = 0
    t0 = time.perf_counter()
    for V, T, q, bvh in cases_kv:
        r = O.run(V, T, q, p_range=(0, min(m, int(q["n"]))), threads=threads, bvh=bvh)
        hits += int(r["hits"])
    dt = time.perf_counter() - t0
    return hits / dt, hits, dt


def cpu_baseline(case_list, mesh_map, budget_s=12.0, satellite=True):
    """The FP64 oracle, as it stands, on bounded samples of the benchmark's
    own queries: the first particles of every plate / cylinder case with every
    usable host thread (the machine's share: at most 16) and with one, and the
    first particles of the concave-satellite query through the oracle's
    hierarchy (built once, outside the timed span), likewise."""
    from oracle import oracle as O
    from paper_1312_3691_amd import inputs as I
    n_cpu = os.cpu_count() or 1
    try:
        n_aff = len(os.sched_getaffinity(0))
    except AttributeError:
        n_aff = n_cpu
    threads = max(1, min(n_aff, 16))
    kv = [(*mesh_map[c["kind"]], c["query"], False) for c in case_list]
    # calibrate on one plate and one cylinder case
    t0 = time.perf_counter()
    probe = 20000
    _oracle_rate([kv[0], kv[-1]], probe, threads)
    per_particle = (time.perf_counter() - t0) / (2 * probe)
    m = int(max(1000, min(200_000, budget_s / (per_particle * len(case_list)))))
    rate, hits, dt = _oracle_rate(kv, m, threads)
    m1 = max(500, m // threads)  # one thread: every fourth case, the same particles per thread
    rate1, hits1, dt1 = _oracle_rate(kv[::4], m1, 1)
    out = {"value": rate, "unit": "hits/s", "cores": threads, "kind": "oracle",
           "sample": f"first {m} particles of each of the {len(case_list)} plate / cylinder cases "
                     f"({m * len(case_list)} particles, {hits} hits, {dt:.1f} s wall)",
           "host": {"cpu_model": cpu_model(), "os_cpu_count": n_cpu, "affinity_cpus": n_aff,
                    "threads_used": threads},
           "single_thread": {"value": rate1, "unit": "hits/s",
                             "sample": f"first {m1} particles of every fourth case ({hits1} hits, {dt1:.1f} s)"}}
    if satellite:
        V, T = I.satellite(50_000)
        tb = time.perf_counter()
        tree = O.BVH(V, T)
        build_s = time.perf_counter() - tb
        q = satellite_query(1e8)
        ms_, ms1 = 2_000_000, 100_000
        r_sat, h_sat, d_sat = _oracle_rate([(V, T, q, tree)], ms_, threads)
        r_sat1, h_sat1, d_sat1 = _oracle_rate([(V, T, q, tree)], ms1, 1)
        out["concave_satellite"] = {"value": r_sat, "unit": "hits/s", "threads": threads,
                                    "sample": f"first {ms_} of the 1e8 particles of the satellite query "
                                              f"({h_sat} hits, {d_sat:.1f} s); hierarchy build {build_s:.2f} s "
                                              "excluded",
                                    "single_thread": {"value": r_sat1, "unit": "hits/s",
                                                      "sample": f"first {ms1} particles ({h_sat1} hits, "
                                                                f"{d_sat1:.1f} s)"}}
        # attitude sweep: every 128th of the 1024 queries, first particles of each
        sw = sweep_queries(1e6)[::128]
        r_sw, h_sw, d_sw = _oracle_rate([(V, T, dict(q, flags=0), tree) for q in sw], 200_000, threads)
        out["attitude_sweep"] = {"value": r_sw, "unit": "hits/s", "threads": threads,
                                 "sample": f"first 200000 particles of {len(sw)} of the 1024 queries ({h_sw} hits, "
                                           f"{d_sw:.1f} s)"}
        # served stream: the first 8 requests of the default stream over its four meshes, first
        # particles of each
        names, reqs, _ = served_requests(SERVED_DEFAULT_REQUESTS)
        reqs = reqs[:8]
        meshes = {}
        tb = time.perf_counter()
        for k, (nm, nt) in enumerate(names.items()):
            Vm, Tm = I.satellite(nt, seed=k)
            meshes[nm] = (Vm, Tm, O.BVH(Vm, Tm))
        build_s = time.perf_counter() - tb
        kv = [(meshes[m][0], meshes[m][1], q, meshes[m][2]) for m, q in reqs]
        r_sv, h_sv, d_sv = _oracle_rate(kv, 50_000, threads)
        out["served_stream"] = {"value": r_sv, "unit": "hits/s", "threads": threads,
                                "sample": f"first 50000 particles of the stream's first {len(reqs)} requests "
                                          f"({h_sv} hits, {d_sv:.1f} s); meshes and hierarchies built outside the "
                                          f"timed span ({build_s:.1f} s)"}
    return out


COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written per launch
COPY_LAUNCHES = 4


def copy_calibration():
    """Plain device-to-device copies of known size, for scaling the HBM counters."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(COPY_LAUNCHES):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": COPY_LAUNCHES}))


def _counter_rows(path, counter):
    """(kernel name, dispatch id, value in KiB) from a rocprofv3 counter_collection.csv."""
    import csv
    rows = []
    for fn in [os.path.join(dp, f) for dp, _, fs in os.walk(path) for f in fs if f.endswith("counter_collection.csv")]:
        for r in csv.DictReader(open(fn)):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return rows


def summarize_traffic(pmc_dir, path=None):
    """Writes profiles/traffic.json from four rocprofv3 --pmc runs under pmc_dir:
    bench_fetch, bench_write (this benchmark with --steps 1 --warmup 0 --no-cpu
    --no-plain) and copy_fetch, copy_write (--copy-calibration)."""
    out = {}
    scale = {}
    for c, sub in (("FETCH_SIZE", "copy_fetch"), ("WRITE_SIZE", "copy_write")):
        vals = [v for n, _, v in _counter_rows(os.path.join(pmc_dir, sub), c) if "copy" in n.lower() or "elementwise" in n.lower()]
        per = sorted(vals)[len(vals) // 2] * 1024.0  # median dispatch, bytes as the counter reads them
        scale[c] = COPY_BYTES / per
    per_mesh = {}
    for c, sub in (("FETCH_SIZE", "bench_fetch"), ("WRITE_SIZE", "bench_write")):
        import re
        for n, d, v in _counter_rows(os.path.join(pmc_dir, sub), c):
            m = re.search(r"(?<![a-z_])batch_kernel<[^>]*>", n)
            if m:
                per_mesh.setdefault(m.group(0), {}).setdefault(c, []).append(v * 1024.0 * scale[c])
    detail = {}
    for k, d in per_mesh.items():
        f = sorted(d["FETCH_SIZE"])[len(d["FETCH_SIZE"]) // 2]
        w = sorted(d["WRITE_SIZE"])[len(d["WRITE_SIZE"]) // 2]
        detail[k] = {"fetch_bytes": f, "write_bytes": w, "dispatches": len(d["FETCH_SIZE"])}
    out["kernel_hash"] = kernel_hash()
    out["counter_scale"] = scale
    out["note"] = ("median dispatch of each batch_kernel instance; bytes = counter KiB x 1024 x (known copy "
                   "bytes / the counter's reading for that copy)")
    out["batch_kernel"] = detail
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
               "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_BUSY_CYCLES"]
L1_COUNTERS = ["TCP_TOTAL_CACHE_ACCESSES_sum", "TCP_TCC_READ_REQ_sum", "TCP_TCC_ATOMIC_WITH_RET_REQ_sum",
               "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"]


def summarize_counters(pmc_dir):
    """Markdown summary of the batched kernels' instruction and cache counters
    from two rocprofv3 --pmc runs under pmc_dir (sq: SQ_COUNTERS, l1:
    L1_COUNTERS; this benchmark with --steps 1 --warmup 0 --no-cpu --no-plain):
    per kernel, the median dispatch of each counter, the mean active lanes per
    VALU instruction (SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU, of 64) and
    the L1 hit fraction for vector memory."""
    import re
    per = {}
    for sub, names in (("sq", SQ_COUNTERS), ("l1", L1_COUNTERS)):
        for c in names:
            for n, d, v in _counter_rows(os.path.join(pmc_dir, sub), c):
                m = re.search(r"(?<![a-z_])batch_kernel<[^>]*>", n)
                if m:
                    per.setdefault(m.group(0), {}).setdefault(c, []).append(v)
    lines = ["| kernel | " + " | ".join(SQ_COUNTERS + L1_COUNTERS) + " | active lanes per VALU instruction | L1 hit fraction |",
             "|---" * (len(SQ_COUNTERS) + len(L1_COUNTERS) + 3) + "|"]
    for k in sorted(per):
        med = {c: sorted(v)[len(v) // 2] for c, v in per[k].items()}
        lanes = med.get("SQ_THREAD_CYCLES_VALU", 0.0) / max(med.get("SQ_ACTIVE_INST_VALU", 1.0), 1.0)
        acc, miss = med.get("TCP_TOTAL_CACHE_ACCESSES_sum", 0.0), med.get("TCP_TCC_READ_REQ_sum", 0.0)
        hit = 1.0 - miss / acc if acc else float("nan")
        lines.append(f"| `{k}` | " + " | ".join(f"{med.get(c, float('nan')):.4g}" for c in SQ_COUNTERS + L1_COUNTERS)
                     + f" | {lanes:.1f} | {hit:.3f} |")
    print("\n".join(lines))


def summarize_served_trace(trace_dir):
    """Markdown summary of a rocprofv3 --kernel-trace of the served workload
    (run with --served-loads "" so that every batched launch before the FIFO
    plain path is a saturation step): step launches, the time between one
    step's end and the next one's start, how much of that time no kernel ran,
    and the kernels run between steps."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()

    def short(n):
        import re
        m = re.search(r"(?<![A-Za-z0-9_])([A-Za-z_][A-Za-z0-9_]*_kernel)(<[^>]*>)?", n)
        return (m.group(1) + (m.group(2) or "")) if m else n.split("(")[0]

    # the saturation run's steps: the batched launches before the FIFO plain path's first trace launch
    first_plain = min((r[0] for r in rows if "trace_kernel<" in r[2]), default=None)
    steps = [r for r in rows if "batch_kernel<" in r[2] and (first_plain is None or r[0] < first_plain)]
    if len(steps) < 2:
        print("fewer than two step launches in the trace")
        return
    t0, t1 = steps[0][0], steps[-1][1]
    inside = [r for r in rows if r[0] >= t0 and r[1] <= t1]

    def busy(lo, hi):  # union of kernel intervals within [lo, hi]
        tot, cur = 0, lo
        for a, b, _ in inside:
            a, b = max(a, cur), min(b, hi)
            if b > a:
                tot += b - a
                cur = b
        return tot

    dur = np.array([(b - a) * 1e-6 for a, b, _ in steps])
    gap = np.array([(steps[k + 1][0] - steps[k][1]) * 1e-6 for k in range(len(steps) - 1)])
    idle = np.array([g - busy(steps[k][1], steps[k + 1][0]) * 1e-6 for k, g in enumerate(gap)])
    span = (t1 - t0) * 1e-6
    others = {}
    for a, b, n in inside:
        if "batch_kernel<" not in n:
            o = others.setdefault(short(n), [0, 0.0])
            o[0] += 1
            o[1] += (b - a) * 1e-6
    inst = {}
    for _, _, n in steps:
        inst[short(n)] = inst.get(short(n), 0) + 1
    q = lambda v, p: float(np.percentile(v, p))
    out = [f"Step launches: {len(steps)} ({', '.join(f'`{k}` x {v}' for k, v in sorted(inst.items()))}), "
           f"from the first step's start to the last step's end {span:.1f} ms.",
           "",
           "| | median | p90 | max | total |",
           "|---|---|---|---|---|",
           f"| step kernel ms | {q(dur, 50):.2f} | {q(dur, 90):.2f} | {dur.max():.2f} | {dur.sum():.1f} |",
           f"| between steps ms | {q(gap, 50):.3f} | {q(gap, 90):.3f} | {gap.max():.3f} | {gap.sum():.1f} |",
           f"| of which no kernel ran ms | {q(idle, 50):.3f} | {q(idle, 90):.3f} | {idle.max():.3f} | {idle.sum():.1f} |",
           "",
           f"Device busy (union of kernel intervals) {100.0 * busy(t0, t1) * 1e-6 / span:.1f} % of the span; "
           f"step kernels alone {100.0 * dur.sum() / span:.1f} %.",
           "",
           "Kernels between the steps:",
           "",
           "| kernel | launches | total ms |",
           "|---|---|---|"]
    for k, (c, t) in sorted(others.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {c} | {t:.2f} |")
    print("\n".join(out))


def fixed_tuning(args, key):
    """The --tuning settings for `key` (a mesh kind, or the workload), if given."""
    if not args.tuning:
        return None
    txt = open(args.tuning).read() if os.path.exists(args.tuning) else args.tuning
    d = json.loads(txt.strip().splitlines()[-1])
    d = d.get("tuning", d)
    return d.get(key, d if "refill_lanes" in d else None)


def tune_for(args, mesh, queries, key="workload", hold=None):
    """Autotuned launch settings for this mesh and query mix (set on the
    mesh's context, untimed), with the settings in `hold` not searched; fixed
    ones with --tuning, the library defaults with --no-tune."""
    fixed = fixed_tuning(args, key)
    if fixed is not None:
        mesh.ctx.set_tuning(**fixed)
        return mesh.ctx.tuning
    if args.no_tune:
        return mesh.ctx.tuning
    from paper_1312_3691_amd import autotune
    t0 = time.perf_counter()
    best, trials = autotune.tune(mesh, queries, particles=int(args.tune_particles) or None, fixed=hold)
    log(f"autotune nt={mesh.info['nt']}: {best} ({len(trials)} trials, {time.perf_counter() - t0:.1f} s)")
    return best


def _line(metric, value, unit, dt, steps, warmup, config, extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": "f32+f64", "data": "synthetic", "config": config}
    d.update(extra)
    print(json.dumps(d), flush=True)


def workload_satellite(args):
    """Concave satellite (~50k triangles), S = 7, alpha = 0.9, 1e8 particles, one query,
    as one graph-replayed batched launch (the configuration the default run also reports)."""
    import torch

    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    sink = torch.zeros(64, dtype=torch.uint8, device="cuda")
    measured = {k: ctx.ceiling_valu(k, sink) / 1e12 for k in ("fp32_fma", "fp64_fma")}
    sat = config_satellite(ctx, args, measured)
    sat.pop("mesh")
    _line("particle-surface hits/sec on 1 MI355X (concave satellite)", sat["hits_per_s"], "hits/s",
          sat["ms_per_step"] / 1e3, args.steps, args.warmup,
          {"workload": sat["workload"], "path": "batched persistent launch, graph replay", "bvh": args.bvh}, sat)


PRATT_S = (0.5, 1.0, 2.0, 3.0, 5.0, 8.0, 12.0, 20.0, 30.0, 50.0)
PRATT_EPS_D = 1.05349  # eps_D(90 deg) as printed with eq. hypersphere (Pratt's re-emission drag integral)


def workload_pratt(args):
    """Concave spherical shell: an open hemispherical cup (radius 1 m, 4512
    triangles), flow into the cup, full diffuse accommodation, S from 0.5 to 50,
    against Pratt's hyperthermal form C_D = 2 + eps_D sqrt(pi) tau / S (eq.
    hypersphere; A_ref = pi r^2, the rim disk).  eps_D itself comes from the
    tau-slope of C_D at S = 100 on equal seeds (C_D is linear in tau there)."""
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    V, T = I.hemisphere_cup(24, 96)
    t0 = time.perf_counter()
    mesh = ctx.build_mesh(V, T, builder=args.bvh)
    build_ms = (time.perf_counter() - t0) * 1e3
    n = int(args.particles_pratt)
    flow = I.quat_for_flow((0.0, 0.0, -1.0))
    cv = dict(cv_radius=1.0 + 1e-3, cv_center=(0.0, 0.0, 0.0))
    qs = [I.query(q=flow, S=S, T_inf=T_INF, T_w=T_W, alpha=1.0, n=n, seed=i, max_reflections=16, **cv)
          for i, S in enumerate(PRATT_S)]
    taus = (0.5, 1.0)
    qs += [I.query(q=flow, S=100.0, T_inf=1000.0, T_w=1000.0 * t * t, alpha=1.0, n=n, seed=100, max_reflections=16,
                   **cv) for t in taus]
    tuning = tune_for(args, mesh, qs)
    b = tpmc.Batch(mesh, qs)
    b.launch().results(A_ref=math.pi)
    for _ in range(args.warmup):
        b.launch(use_graph=True).results(A_ref=math.pi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = b.launch(use_graph=True).results(A_ref=math.pi)
    dt = (time.perf_counter() - t0) / args.steps
    b.close()
    tau = math.sqrt(T_W / T_INF)
    sweep = [{"S": S, "CD": r["CD"], "CD_sigma": r["CD_sigma"],
              "pratt_CD": 2.0 + PRATT_EPS_D * math.sqrt(math.pi) * tau / S,
              "hits_per_particle": r["hits"] / n, "capped": r["capped"]} for S, r in zip(PRATT_S, res)]
    r0, r1 = res[len(PRATT_S):]
    slope = (r1["CD"] - r0["CD"]) / (taus[1] - taus[0])
    eps = slope * 100.0 / math.sqrt(math.pi)
    # conservative: the two runs share seeds, so their errors are positively correlated
    eps_sig = (r0["CD_sigma"] + r1["CD_sigma"]) / (taus[1] - taus[0]) * 100.0 / math.sqrt(math.pi)
    hits = sum(r["hits"] for r in res)
    _line("particle-surface hits/sec on 1 MI355X (concave shell vs Pratt)", hits / dt, "hits/s", dt, args.steps,
          args.warmup, {"workload": f"hemispherical cup {len(T)} tris, flow into the cup, alpha=1, S in "
                                    f"{list(PRATT_S)} + S=100 at tau in {list(taus)}, {n} particles each",
                        "path": "one batched persistent launch, graph replay", "bvh": args.bvh},
          {"sweep": sweep, "eps_D": {"value": eps, "sigma_bound": eps_sig, "paper": PRATT_EPS_D},
           "segments_per_s": sum(r["segments"] for r in res) / dt, "bvh_build_ms": build_ms, "tuning": tuning})


def workload_boxcv(args):
    """Control-volume shape invariance (Sec. III.A): the 1280-triangle
    icosphere at S = 5, diffuse, seeded on the sphere CV, on the vertex box
    widened by 1e-3 and on an offset cube, 1e8 particles each in one batched
    launch; each C_D against the per-facet exact value (stored from the closed
    forms in tests/golden/closed_forms.json)."""
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    V, T = I.icosphere(3)
    mesh = ctx.build_mesh(V, T, builder=args.bvh)
    n = int(args.particles_boxcv)
    cvs = (("sphere r=1.001", dict(cv_radius=1.001)), ("fitted box", dict(cv_box=True)),
           ("cube half-side 1.6, offset (0.2,-0.3,0.1)", dict(cv_box=True, cv_radius=1.6, cv_center=(0.2, -0.3, 0.1))))
    qs = [I.query(S=5.0, T_inf=T_INF, T_w=T_W, alpha=1.0, n=n, seed=i, **kw) for i, (_, kw) in enumerate(cvs)]
    tuning = tune_for(args, mesh, qs)
    b = tpmc.Batch(mesh, qs)
    b.launch().results(A_ref=math.pi)
    for _ in range(args.warmup):
        b.launch(use_graph=True).results(A_ref=math.pi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = b.launch(use_graph=True).results(A_ref=math.pi)
    dt = (time.perf_counter() - t0) / args.steps
    b.close()
    exact = json.load(open(os.path.join(ROOT, "tests", "golden", "closed_forms.json")))["icosphere3_S5"]["cd_facet"]
    rows = [{"cv": name, "CD": r["CD"], "CD_sigma": r["CD_sigma"], "err_over_sigma": (r["CD"] - exact) / r["CD_sigma"],
             "Gamma_hat": r["Gamma_hat"], "hits_per_particle": r["hits"] / n} for (name, _), r in zip(cvs, res)]
    hits = sum(r["hits"] for r in res)
    _line("particle-surface hits/sec on 1 MI355X (control-volume shape invariance)", hits / dt, "hits/s", dt,
          args.steps, args.warmup,
          {"workload": f"icosphere {len(T)} tris, S=5, alpha=1, sphere / fitted box / offset cube CV, {n} particles each",
           "path": "one batched persistent launch, graph replay", "bvh": args.bvh},
          {"cases": rows, "CD_exact_per_facet": exact, "segments_per_s": sum(r["segments"] for r in res) / dt,
           "tuning": tuning})


ENERGY_ACC = (0.0, 0.25, 0.5, 0.75, 1.0)


def plate_ch(S, angle_deg, tau, alpha_E):
    """Heat-transfer coefficient of the flat plate (one face wetted, A_ref = 1
    m^2) under full diffuse re-emission with energy accommodation alpha_E:
    per molecule E[|w|^2 - |w'|^2] = alpha_E (|w|^2 - 2 tau^2), summed over the
    one-sided flux: alpha_E [M3 + (S_t^2 + 1 - 2 tau^2) M1] / S^3 with the flux
    moments M1 = chi(s) / (2 sqrt(pi)) and M3 = [(s^2 + 1) e^{-s^2} +
    sqrt(pi) s (s^2 + 3/2)(1 + erf s)] / (2 sqrt(pi)) of the normal speed,
    s = S cos(a), S_t = S sin(a)."""
    a = math.radians(angle_deg)
    s, st = S * math.cos(a), S * math.sin(a)
    ec = math.erfc(-s)
    m1 = (math.exp(-s * s) + math.sqrt(math.pi) * s * ec) / (2 * math.sqrt(math.pi))
    m3 = ((s * s + 1) * math.exp(-s * s) + math.sqrt(math.pi) * s * (s * s + 1.5) * ec) / (2 * math.sqrt(math.pi))
    return alpha_E * (m3 + (st * st + 1.0 - 2.0 * tau * tau) * m1) / S ** 3


def workload_ceilings(args):
    """Measured ceilings of the roofline on this GPU (tpmc_ceiling_*): VALU
    issue for FP32 FMA, FP64 FMA and 32-bit integer multiply-add; streaming
    reads from a 2 MiB buffer (held in every XCD's L2), a 64 MiB one (Infinity
    Cache) and a 4 GiB one (HBM); int64 atomic adds in global memory onto 1, 16,
    4096 and 2^20 addresses and in LDS onto 1, 16 and 512 addresses.  Each is
    one event-timed launch after an untimed one."""
    import torch

    from paper_1312_3691_amd import tpmc

    ctx = tpmc.Context(0)
    sink = torch.zeros(64, dtype=torch.uint8, device="cuda")
    out = {"metric": "measured ceilings on 1 MI355X", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "ceiling microkernels (VALU, cache and HBM reads, atomics)"}}
    valu = {k: ctx.ceiling_valu(k, sink) for k in ("fp32_fma", "fp64_fma", "int32_mul_add")}
    log(f"valu {valu}")
    reads = {}
    for name, nbytes, passes in (("l2_2MiB", 2 << 20, 400), ("mall_64MiB", 64 << 20, 20), ("hbm_4GiB", 4 << 30, 2)):
        buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        reads[name] = ctx.ceiling_read(buf, passes)
        del buf
        log(f"read {name} {reads[name] / 1e12:.2f} TB/s")
    abuf = torch.zeros(1 << 20, dtype=torch.int64, device="cuda")
    atom = {str(sl): ctx.ceiling_atomic(abuf, sl, 16) for sl in (1, 16, 4096, 1 << 20)}
    lds = {str(sl): ctx.ceiling_lds_atomic(sink, sl, 256) for sl in (1, 16, 512)}
    torch.cuda.synchronize()
    out.update({"valu_lane_ops_per_s": valu, "valu_published_lane_ops_per_s": ALU_PEAK,
                "read_bytes_per_s": reads, "hbm_published_bytes_per_s": 8e12,
                "global_atomic_i64_per_s_by_slots": atom, "lds_atomic_i64_per_s_by_slots": lds})
    print(json.dumps(out), flush=True)


def workload_energy(args):
    """Energy exchange and incomplete energy accommodation: diffuse
    re-emission at tau_r^2 = alpha_E tau^2 + (1 - alpha_E)|w|^2 / 2, alpha_E
    from 0 to 1, on the plate (S = 3, 30 deg; C_H against its flux-moment
    closed form), the capped cylinder (S = 3, 45 deg) and the concave
    satellite (S = 7, the C3 attitude), 1e7 particles each, one batched launch
    per mesh; reports C_D and the heat-transfer coefficient C_H."""
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    n = int(args.particles_energy)
    tau = math.sqrt(T_W / T_INF)
    setups = (("plate", I.plate(), (math.sin(math.radians(30)), 0.0, -math.cos(math.radians(30))), 3.0, 1.0),
              ("cylinder", I.capped_cylinder(), (math.sqrt(0.5), 0.0, math.sqrt(0.5)), 3.0, 1.0),
              ("satellite", I.satellite(50_000), (-0.5, 0.0, -math.sqrt(3.0) / 2.0), 7.0, 1.0))
    rows, hits, dt_total, tunings = [], 0, 0.0, {}
    for name, (V, T), U, S, alpha in setups:
        mesh = ctx.build_mesh(V, T, builder=args.bvh)
        qs = [I.query(q=I.quat_for_flow(U), S=S, T_inf=T_INF, T_w=T_W, alpha=alpha, n=n, seed=i, alpha_E=aE)
              for i, aE in enumerate(ENERGY_ACC)]
        tunings[name] = tune_for(args, mesh, qs, key=name)
        b = tpmc.Batch(mesh, qs)
        b.launch().results()
        for _ in range(args.warmup):
            b.launch(use_graph=True).results()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = b.launch(use_graph=True).results()
        dt = (time.perf_counter() - t0) / args.steps
        b.close()
        dt_total += dt
        hits += sum(r["hits"] for r in res)
        for aE, r in zip(ENERGY_ACC, res):
            row = {"mesh": name, "S": S, "alpha_E": aE, "CD": r["CD"], "CD_sigma": r["CD_sigma"], "CH": r["CH"],
                   "CH_sigma": r["CH_sigma"], "hits_per_particle": r["hits"] / n}
            if name == "plate":
                row["CH_exact"] = plate_ch(S, 30.0, tau, aE)
            rows.append(row)
    _line("particle-surface hits/sec on 1 MI355X (energy accommodation and heat transfer)", hits / dt_total, "hits/s",
          dt_total, args.steps, args.warmup,
          {"workload": f"plate / capped cylinder / concave satellite, alpha_E in {list(ENERGY_ACC)}, {n} particles "
                       "each, one batched launch per mesh", "path": "batched persistent launch, graph replay",
           "bvh": args.bvh},
          {"cases": rows, "tuning": tunings})


MOMENT_PITCH = tuple(range(-40, 41, 10))
MOMENT_YAW = (-20, 0, 20)


def workload_moments(args):
    """Aerodynamic moment and static stability over an attitude grid: the
    concave satellite (~50k triangles), S = 7, alpha = 0.9, pitch -40..40 deg x
    yaw -20/0/20 deg about the nominal flow -z, all 27 attitudes in one batched
    launch.  C_m = M / (q A_ref c) about the bus centre (origin) with A_ref = 1
    m^2 and c = 1 m; the pitch stiffness dC_m,y / d(pitch) at zero yaw by
    central differences."""
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    V, T = I.satellite(50_000)
    t0 = time.perf_counter()
    mesh = ctx.build_mesh(V, T, builder=args.bvh)
    build_ms = (time.perf_counter() - t0) * 1e3
    n = int(args.particles_moments)
    grid = [(p, y) for y in MOMENT_YAW for p in MOMENT_PITCH]
    qs = [I.query(q=I.quat_for_flow(I.flow_pitch_yaw(p, y)), S=7.0, T_inf=T_INF, T_w=T_W, alpha=0.9, n=n, seed=i,
                  max_reflections=16) for i, (p, y) in enumerate(grid)]
    tuning = tune_for(args, mesh, qs)
    b = tpmc.Batch(mesh, qs)
    b.launch().results()
    for _ in range(args.warmup):
        b.launch(use_graph=True).results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = b.launch(use_graph=True).results(x_ref=(0.0, 0.0, 0.0), A_ref=1.0)
    dt = (time.perf_counter() - t0) / args.steps
    b.close()
    rows = [{"pitch_deg": p, "yaw_deg": y, "CD": r["CD"], "CD_sigma": r["CD_sigma"], "Cm": list(r["M_over_q"]),
             "CF": list(r["F_over_q"])} for (p, y), r in zip(grid, res)]
    cm_y = {p: r["Cm"][1] for p, r in zip([g[0] for g in grid], rows) if r["yaw_deg"] == 0}
    stiff = (cm_y[10] - cm_y[-10]) / math.radians(20.0)
    hits = sum(r["hits"] for r in res)
    _line("particle-surface hits/sec on 1 MI355X (moment and stability sweep)", hits / dt, "hits/s", dt,
          args.steps, args.warmup,
          {"workload": f"concave satellite {len(T)} tris, S=7, alpha=0.9, pitch {list(MOMENT_PITCH)} x yaw "
                       f"{list(MOMENT_YAW)} deg, {n} particles each, moments about the origin",
           "path": "one batched persistent launch, graph replay", "bvh": args.bvh},
          {"grid": rows, "dCmy_dpitch_per_rad": stiff, "segments_per_s": sum(r["segments"] for r in res) / dt,
           "bvh_build_ms": build_ms, "tuning": tuning})


def workload_sweep(args):
    """1024 uniform-random attitudes x S ~ U[2, 10], 1e6 particles each, on the ~50k-triangle
    satellite: one persistent graph-replayed launch against 1024 plain calls (host sync each)."""
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    sink = torch.zeros(64, dtype=torch.uint8, device="cuda")
    measured = {k: ctx.ceiling_valu(k, sink) / 1e12 for k in ("fp32_fma", "fp64_fma")}
    mesh = ctx.build_mesh(*I.satellite(50_000), builder=args.bvh)
    sw = config_sweep(ctx, args, measured, mesh)
    _line("particle-surface hits/sec on 1 MI355X (batched attitude sweep)", sw["hits_per_s"], "hits/s",
          sw["ms_per_step"] / 1e3, args.steps, args.warmup,
          {"workload": sw["workload"], "path": "one persistent graph-replayed launch", "bvh": args.bvh}, sw)


PROBE_PHASES = (("claim", "claim_cycles"), ("traversal", "trav_cycles"), ("leaf", "leaf_cycles"),
                ("service", "serve_cycles"), ("estimate", "est_cycles"), ("seeding", "seed_cycles"),
                ("hand-out", "assign_cycles"))


def probe_record(p, particles, ms):
    """Per-64-particle passes, mean active lanes and share of wave time of each
    phase, from the phase probe's sums over one launch."""
    per64 = 64.0 / particles

    def mean(a, b):
        return p[a] / p[b] if p[b] else None
    share = {name: p[slot] / p["cycles"] for name, slot in PROBE_PHASES}
    share["other"] = 1.0 - sum(share.values())
    return {"ms": ms, "particles": particles, "waves": p["waves"],
            "wave_clock_ghz": p["cycles"] / p["waves"] / (ms * 1e-3) / 1e9,
            "per_64_particles": {"traversal_steps": p["trav_steps"] * per64, "leaf_passes": p["leaf_passes"] * per64,
                                 "service_passes": p["serves"] * per64, "estimate_batches": p["est_batches"] * per64,
                                 "seeding_batches": p["seed_batches"] * per64, "hand_outs": p["assigns"] * per64},
            "mean_lanes": {"traversal": mean("trav_lanes", "trav_steps"), "leaf": mean("leaf_lanes", "leaf_passes"),
                           "service": mean("serve_lanes", "serves"), "estimate": mean("est_particles", "est_batches"),
                           "seeding": mean("seed_particles", "seed_batches"),
                           "hand_out": mean("assign_lanes", "assigns")},
            "estimate_kept": mean("est_kept", "est_particles"), "seeding_kept": mean("seed_kept", "seed_particles"),
            "share": share, "sums": p}


def workload_phase_probe(args):
    """Where the persistent kernel's time goes, from libtpmc_probe.so (the
    library with the batched kernel's phase probe compiled in): one launch each
    of the plate and cylinder batches (per-case N as in the benchmark line, or
    --particles each with --fixed-n), the concave satellite and the attitude
    sweep, with the autotuned settings (or --tuning).  Prints one JSON line with
    each launch's passes and mean active lanes per phase and the share of wave
    time each phase takes, and the same as a markdown table on stderr; then
    the plate and cylinder batches at 2e6 particles per case with 1, 2 and 4
    resident workgroups per CU, whose cycles per pass show which phases are
    bound by latency rather than by issue.  The probe's clock reads lengthen a
    launch by some per cent; the ordinary library has none of this code."""
    os.environ["TPMC_PHASE_PROBE"] = "1"
    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    if not tpmc.PHASE_PROBE:
        raise RuntimeError("the binding was imported before the probe library was selected")
    ctx = tpmc.Context(0)
    mm = meshes()
    dev_mesh = {k: ctx.build_mesh(*v, builder=args.bvh) for k, v in mm.items()}
    if args.fixed_n:
        n_case = [args.particles] * len(cases(1))
    else:
        n_case = case_particles(ctx, dev_mesh, args.particles, args.pilot_particles)
    cl = cases(args.particles, n_case)
    sat = ctx.build_mesh(*I.satellite(50_000), builder=args.bvh)
    runs = [("plate", dev_mesh["plate"], [c["query"] for c in cl if c["kind"] == "plate"], "plate"),
            ("cylinder", dev_mesh["cylinder"], [c["query"] for c in cl if c["kind"] == "cylinder"], "cylinder"),
            ("satellite", sat, [satellite_query(args.particles_sat)], "satellite"),
            ("sweep", sat, sweep_queries(args.particles_sweep), "sweep")]
    out = {}
    for name, mesh, qs, key in runs:
        tuning = tune_for(args, mesh, qs, key=key)
        b = tpmc.Batch(mesh, qs)
        b.launch().results()
        torch.cuda.synchronize()
        ctx.phase_probe(reset=True)
        ms = launch_ms(ctx, b, tuning, 1)
        p = ctx.phase_probe(reset=True)
        res = b.results()
        b.close()
        rec = probe_record(p, sum(r["rays"] for r in res), ms)
        rec.update(kernel=f"{batch_instance(mesh, totals_only=name == 'sweep')} ({name}, {mesh.nt} tris, "
                          f"{len(qs)} queries)", tuning=tuning,
                   preculled_frac=sum(r["preculled"] for r in res) / rec["particles"])
        out[name] = rec
        log(f"{name}: {ms:.2f} ms, shares " + " ".join(f"{k} {v:.3f}" for k, v in rec["share"].items()))
    rows = ["| launch | traversal steps (lanes) | leaf phases (lanes) | service passes (lanes) | "
            "estimate batches (kept) | seeding batches (lanes) | share of wave time: claim / traversal / leaf / "
            "service / estimate / seeding / hand-out / other |", "|---|---|---|---|---|---|---|"]
    for name, r in out.items():
        n, ln, sh = r["per_64_particles"], r["mean_lanes"], r["share"]

        def f(k, lk):
            return f"{n[k]:.2f} ({ln[lk]:.1f})" if ln[lk] is not None else "—"
        est = f"{n['estimate_batches']:.2f} ({r['estimate_kept']:.2f})" if r["estimate_kept"] is not None else "—"
        rows.append(f"| {r['kernel']} | {f('traversal_steps', 'traversal')} | {f('leaf_passes', 'leaf')} | "
                    f"{f('service_passes', 'service')} | {est} | {f('seeding_batches', 'seeding')} | "
                    + " / ".join(f"{100 * sh[k]:.0f}" for k in ("claim", "traversal", "leaf", "service", "estimate",
                                                                 "seeding", "hand-out", "other")) + " % |")
    log("\n".join(rows))
    # occupancy: the same plate and cylinder batches (2e6 particles per case) at 1, 2 and 4 resident
    # workgroups per CU (1-4 waves per SIMD); a phase whose cycles per pass stay flat as waves are
    # added is latency-bound, one whose cycles grow in proportion is issue-bound
    occ, orows = {}, ["| launch | workgroups per CU | ms | cycles per pass: estimate / seeding / traversal step / "
                      "leaf phase / service pass |", "|---|---|---|---|"]
    small = cases(2_000_000)
    for kind in ("plate", "cylinder"):
        qs = [c["query"] for c in small if c["kind"] == kind]
        base = dict(out[kind]["tuning"])
        for g in (1, 2, 4):
            ctx.set_tuning(**dict(base, groups_per_cu=g))
            b = tpmc.Batch(dev_mesh[kind], qs)
            b.launch().results()
            torch.cuda.synchronize()
            ctx.phase_probe(reset=True)
            ms = launch_ms(ctx, b, ctx.tuning, 1)
            p = ctx.phase_probe(reset=True)
            b.close()

            def per(c, n):
                return p[c] / p[n] if p[n] else None
            rec = {"ms": ms, "waves": p["waves"], "estimate": per("est_cycles", "est_batches"),
                   "seeding": per("seed_cycles", "seed_batches"), "traversal": per("trav_cycles", "trav_steps"),
                   "leaf": per("leaf_cycles", "leaf_passes"), "service": per("serve_cycles", "serves")}
            occ[f"{kind}@{g}"] = rec
            orows.append(f"| {kind} | {g} | {ms:.2f} | " + " / ".join(
                "—" if rec[k] is None else f"{rec[k]:.0f}" for k in ("estimate", "seeding", "traversal", "leaf",
                                                                     "service")) + " |")
    log("\n".join(orows))
    print(json.dumps({"probe": "batched kernel phases per 64 particles (libtpmc_probe.so)", "launches": out,
                      "table_md": rows, "occupancy": occ, "occupancy_md": orows}), flush=True)


SERVED_MESHES = {"sat1k": 1_000, "sat20k": 20_000, "sat100k": 100_000, "sat500k": 500_000}
SERVED_WARM, SERVED_MEASURED = 200, 2000  # default served run: warm-up and measured requests
SERVED_DEFAULT_REQUESTS = SERVED_WARM + SERVED_MEASURED


def served_requests(n_req):
    """The served stream's requests: mesh uniform over the four satellites, uniform random
    attitude, S ~ U[2, 10], N log-uniform in [1e5, 1e7], alpha = 0.9, seed = request id.
    Returns the mesh sizes, the requests and the generator, which goes on to draw the
    arrival gaps."""
    from paper_1312_3691_amd import inputs as I
    rng = np.random.default_rng(7)
    names = list(SERVED_MESHES)
    quats = I.random_quats(n_req, 3)
    reqs = []
    for i in range(n_req):
        n = int(10 ** rng.uniform(5, 7))
        reqs.append((names[rng.integers(0, 4)], I.query(q=tuple(quats[i]), S=float(rng.uniform(2, 10)), T_inf=T_INF,
                                                         T_w=T_W, alpha=0.9, n=n, seed=10_000 + i)))
    return dict(SERVED_MESHES), reqs, rng


def workload_served(args):
    """The served stream as its own benchmark line (section text in served_measure)."""
    d = served_measure(args, int(args.warm), int(args.requests),
                       [float(f) for f in args.served_loads.split(",") if f.strip()], int(args.fifo_requests))
    sat = d["saturation"]
    _line("particle-surface hits/sec on 1 MI355X (served stream); p50/p99 query ms", sat["hits_per_s"], "hits/s",
          d["n_meas"] / sat["req_per_s"], 1, d["n_warm"], d.pop("config"),
          {k: v for k, v in d.items() if k not in ("n_warm", "n_meas")})


def served_measure(args, n_warm, n_meas, load_fracs, fifo_requests):
    """Served stream: Poisson arrivals over four resident satellite meshes (~1k, 20k, 100k,
    500k triangles), random attitudes, S ~ U[2, 10], N log-uniform in [1e5, 1e7], alpha = 0.9,
    per-request per-triangle tallies admitted against an HBM budget.  Saturation throughput
    first (everything submitted at once), then offered loads of 0.5 / 0.8 / 0.95 of it, each
    with `--warm` warm-up requests left out of the latency figures; the same stream through a
    FIFO plain path (one query at a time, host sync) for comparison."""
    import asyncio

    import torch

    from paper_1312_3691_amd import inputs as I
    from paper_1312_3691_amd import tpmc
    from paper_1312_3691_amd.serve import GpuExecutor, Scheduler
    ctx = tpmc.Context(0)
    n_req = n_warm + n_meas
    sizes, reqs, rng = served_requests(n_req)
    meshes = {k: ctx.build_mesh(*I.satellite(v, seed=i), builder=args.bvh) for i, (k, v) in enumerate(sizes.items())}
    max_slots = int(args.slots)
    pool_words = int(args.hbm_budget_gb * 2 ** 30) // 8
    # tiles of 16384 particles and a refill threshold of 32 lanes: the tuner, timing one batch,
    # cannot see the per-step costs of claiming tiles (smaller tiles) and of the last tiles of a
    # step (larger ones), nor how a step's mix of meshes shares the waves.  Measured on the
    # pipelined stream at saturation (2000 requests, work claimed per wave in quarter tiles):
    # tiles 16384 / 32768 / 65536 gave 4505 / 4439 / 3996 req/s; refill 16 / 24 / 32 / 40 / 48
    # lanes gave 4091 / 4135 / 4171 / 4069 / 3815 req/s and workgroups per CU 4 / 8 / 16 at
    # refill 32 gave 4171 / 4176 / 4163 (workgroup tiles, 1000 requests).
    tuning = tune_for(args, meshes["sat100k"], [q for m, q in reqs if m == "sat100k"][:64],
                      hold={"tile_particles": 16384, "refill_lanes": 32})
    # the step budget is a particle count, so that the tuned tile size does not change it
    tiles_per_step = max(1, int(args.particles_per_step) // int(tuning["tile_particles"]))
    ex = GpuExecutor(ctx, meshes, max_slots=max_slots, pool_words=pool_words)

    def run(rate):
        sched = Scheduler(ex, max_slots=max_slots, pool_words=pool_words, tiles_per_step=tiles_per_step)
        gaps = rng.exponential(1.0 / rate, n_req) if rate else np.zeros(n_req)

        async def main():
            stop = asyncio.Event()
            runner = asyncio.ensure_future(sched.run(stop))
            futs = []
            # absolute (Poisson) arrival times: every request whose time has come is
            # submitted with that time, however long the scheduler held the loop
            t0 = time.perf_counter()
            arrive = t0 + np.cumsum(gaps)
            t_meas = float(arrive[n_warm]) if rate else t0
            k = 0
            while k < n_req:
                now = time.perf_counter()
                while k < n_req and arrive[k] <= now:
                    futs.append(sched.submit(reqs[k][0], reqs[k][1], t_arrival=float(arrive[k])))
                    k += 1
                if k < n_req:
                    await asyncio.sleep(max(0.0, float(arrive[k]) - time.perf_counter()))
            res = await asyncio.gather(*futs, return_exceptions=True)
            t_end = time.perf_counter()
            stop.set()
            sched._wake.set()
            await runner
            return res, t_end - t_meas

        res, dt = asyncio.run(main())
        ok = [r for r in res[n_warm:] if isinstance(r, dict)]
        p50, p99 = sched.percentiles(skip=n_warm)
        return res, {"req_per_s": len(ok) / dt, "hits_per_s": sum(r["hits"] for r in ok) / dt,
                     "p50_ms": p50, "p99_ms": p99, "steps": sched.stats.steps,
                     "max_active": sched.stats.max_active, "rejected": sched.stats.rejected,
                     "failed": sched.stats.failed, "completed": len(ok)}

    log("served: saturation")
    res, sat = run(0)
    sat_rate = sat["req_per_s"]
    loads = {}
    for frac in load_fracs:
        log(f"served: load {frac}")
        _, st = run(frac * sat_rate)
        loads[str(frac)] = dict(st, offered_req_per_s=frac * sat_rate)
    # FIFO plain path: one request at a time (seed -> trace -> forces, host sync), service
    # times measured; latencies for the 0.8 load's arrival process by a single-server queue
    log("served: FIFO plain path")
    service = []
    for mesh, q in reqs[:n_warm + min(n_meas, fifo_requests)]:
        t0 = time.perf_counter()
        r, pr = tpmc.run(meshes[mesh], [q])
        service.append(time.perf_counter() - t0)
        pr.close()
    service = np.array(service[n_warm:]) if len(service) > n_warm else np.array(service)
    arrivals = np.cumsum(rng.exponential(1.0 / (0.8 * sat_rate), len(service)))
    finish, lat = 0.0, []
    for a, sv in zip(arrivals, service):
        finish = max(finish, a) + sv
        lat.append((finish - a) * 1e3)
    fifo = {"service_ms_mean": float(service.mean() * 1e3), "capacity_req_per_s": float(1.0 / service.mean()),
            "requests": int(len(service)),
            "p50_ms_at_0.8_of_served_saturation": float(np.percentile(lat, 50)),
            "p99_ms_at_0.8_of_served_saturation": float(np.percentile(lat, 99))}
    # where a step's time goes, by mesh: the stream's first 16 requests on each mesh, 2e6
    # particles each, as one batched launch with the served launch settings
    per_mesh = {}
    for name, m in meshes.items():
        qs = [dict(q, n=2_000_000) for mm, q in reqs if mm == name][:16]
        b = tpmc.Batch(m, qs)
        b.launch(use_graph=True)
        res_m = b.results()
        ms = launch_ms(ctx, b, ctx.tuning, 3)
        b.close()
        n_p = sum(r["rays"] for r in res_m)
        per_mesh[name] = {"nt": m.nt, "requests": len(qs), "ms": ms, "particles_per_s": n_p / (ms * 1e-3),
                          "hits_per_s": sum(r["hits"] for r in res_m) / (ms * 1e-3),
                          "preculled_fraction": sum(r["preculled"] for r in res_m) / n_p}
    # every served result equals its solo run (first 8 requests)
    same = True
    for (mesh, q), r in list(zip(reqs, res))[:8]:
        solo, pr = tpmc.run(meshes[mesh], [q])
        same = same and isinstance(r, dict) and all(np.array_equal(np.asarray(solo[0][k]), np.asarray(r[k]))
                                                    for k in tpmc.same_on_every_path(solo[0]))
        pr.close()
    torch.cuda.synchronize()
    out = {"config": {"workload": f"{n_warm} + {n_meas} requests over satellites {list(sizes.values())} tris, "
                                  f"N log-uniform 1e5-1e7, S~U[2,10], alpha=0.9, per-triangle tallies",
                      "slots": max_slots, "hbm_budget_gb": args.hbm_budget_gb,
                      "path": "continuous batching, one persistent launch per step",
                      "particles_per_step": int(args.particles_per_step), "tiles_per_step": tiles_per_step,
                      "bvh": args.bvh},
           "n_warm": n_warm, "n_meas": n_meas,
           "saturation": sat, "loads": loads, "query_ms_p50": loads.get("0.8", {}).get("p50_ms"),
           "query_ms_p99": loads.get("0.8", {}).get("p99_ms"), "fifo_plain_path": fifo,
           "served_over_fifo": sat_rate / fifo["capacity_req_per_s"], "served_equals_solo": bool(same),
           "per_mesh_batched": per_mesh,
           "meshes": {k: {"nt": m.nt, "depth": m.info["depth"], "stack_slots": m.info["stack_slots"]}
                      for k, m in meshes.items()},
           "tuning": tuning}
    for m in meshes.values():
        m.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--particles", type=int, default=N_PER_CASE,
                    help="particles per case, the floor of the per-case count (default 1e7)")
    ap.add_argument("--fixed-n", action="store_true",
                    help="every case runs --particles particles (no accuracy-driven per-case count)")
    ap.add_argument("--pilot-particles", type=float, default=1e6, help="particles per case of the N pilot")
    ap.add_argument("--no-satellite", action="store_true",
                    help="leave out the concave-satellite and attitude-sweep configurations")
    ap.add_argument("--no-served", action="store_true",
                    help="leave out the served stream (run by default with 100 + 1000 requests, the 0.8 load, "
                         "300 FIFO requests)")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the HBM-counter calibration copies")
    ap.add_argument("--summarize-traffic", metavar="PMC_DIR", help="write profiles/traffic.json from counter runs")
    ap.add_argument("--summarize-counters", metavar="PMC_DIR",
                    help="print the batched kernels' instruction and L1 counters from runs under PMC_DIR/sq, PMC_DIR/l1")
    ap.add_argument("--traffic-out", default=None, help="output path for --summarize-traffic")
    ap.add_argument("--summarize-served-trace", metavar="TRACE_DIR",
                    help="step launches and the gaps between them, from a kernel trace of the served workload")
    ap.add_argument("--workload", default="plate-cylinder",
                    choices=["plate-cylinder", "satellite", "sweep", "served", "pratt", "moments", "boxcv",
                             "energy", "ceilings", "phase-probe"],
                    help="plate-cylinder (default, the benchmark line) or an additional configuration")
    ap.add_argument("--particles-sat", type=float, default=1e8)
    ap.add_argument("--particles-sweep", type=float, default=1e6)
    ap.add_argument("--particles-pratt", type=float, default=1e7)
    ap.add_argument("--particles-moments", type=float, default=4e6)
    ap.add_argument("--particles-boxcv", type=float, default=1e8)
    ap.add_argument("--particles-energy", type=float, default=1e7)
    ap.add_argument("--requests", type=int, default=SERVED_MEASURED, help="served: measured requests per load")
    ap.add_argument("--warm", type=int, default=SERVED_WARM, help="served: warm-up requests per load")
    ap.add_argument("--slots", type=int, default=128, help="served: request slots")
    ap.add_argument("--hbm-budget-gb", type=float, default=16.0, help="served: per-request tally budget")
    ap.add_argument("--fifo-requests", type=int, default=600, help="served: requests timed on the plain path")
    ap.add_argument("--served-loads", default="0.5,0.8,0.95",
                    help="served: offered loads as fractions of the saturation throughput (comma-separated)")
    ap.add_argument("--particles-per-step", type=float, default=2048 * 65536,
                    help="served: particles per continuous-batching step (split into tiles of the tuned size)")
    ap.add_argument("--bvh", default="sah", choices=["sah", "lbvh"], help="BVH builder (results do not depend on it)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch autotuner (library defaults)")
    ap.add_argument("--tune-particles", type=float, default=0,
                    help="particles per autotuner trial (default 0: the whole workload)")
    ap.add_argument("--tuning", default=None, metavar="JSON",
                    help="fixed settings instead of the autotuner: a bench line's \"tuning\" object, "
                         "or a file holding a bench line")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic, args.traffic_out)
        return
    if args.summarize_served_trace:
        summarize_served_trace(args.summarize_served_trace)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a query shards by particle range: every GPU traces its own id range on a BVH replica and "
              "the int64 tallies are summed with one all-reduce)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "plate-cylinder":
        {"satellite": workload_satellite, "sweep": workload_sweep, "served": workload_served,
         "pratt": workload_pratt, "moments": workload_moments, "boxcv": workload_boxcv,
         "energy": workload_energy, "ceilings": workload_ceilings,
         "phase-probe": workload_phase_probe}[args.workload](args)
        return

    import torch

    from paper_1312_3691_amd import tpmc

    ctx = tpmc.Context(0)
    mm = meshes()
    dev_mesh, build_ms = {}, {}
    for k, v in mm.items():
        t0 = time.perf_counter()
        dev_mesh[k] = ctx.build_mesh(*v, builder=args.bvh)
        build_ms[k] = (time.perf_counter() - t0) * 1e3
    # per-case particle counts: the case's 1e7, raised where 3 sigma_rel would exceed 1e-3
    if args.fixed_n:
        n_case = [args.particles] * len(cases(1))
    else:
        log("pilot for per-case N")
        n_case = case_particles(ctx, dev_mesh, args.particles, args.pilot_particles)
    cl = cases(args.particles, n_case)
    batches, tunings = {}, {}
    for kind in ("plate", "cylinder"):
        qs = [c["query"] for c in cl if c["kind"] == kind]
        tunings[kind] = tune_for(args, dev_mesh[kind], qs, key=kind)  # sets the context's tuning
        batches[kind] = tpmc.Batch(dev_mesh[kind], qs)
    torch.cuda.synchronize()

    def step(use_graph=True):
        out = []
        for kind in ("plate", "cylinder"):
            if ctx.tuning != tunings[kind]:
                ctx.set_tuning(**tunings[kind])
            b = batches[kind]
            b.launch(use_graph=use_graph)
            out += b.results(A_ref=1.0)
        return out

    log("warmup")
    res = step(use_graph=False)
    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    log("timed steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    hits = sum(r["hits"] for r in res)
    particles = sum(r["rays"] for r in res)
    segments = sum(r["segments"] for r in res)
    assert all(r["tr_capped"] == 0 and r["guard_trips"] == 0 for r in res)

    # each mesh's persistent launch: duration with events on its stream, work from its results
    # and from the counting kernel on 1e6-particle subsets of its queries
    log("launch timing and work counters")
    launches = {}
    ordered = [c for k in ("plate", "cylinder") for c in cl if c["kind"] == k]
    for kind in ("plate", "cylinder"):
        rk = [r for c, r in zip(ordered, res) if c["kind"] == kind]
        qk = [c["query"] for c in cl if c["kind"] == kind]
        ms = launch_ms(ctx, batches[kind], tunings[kind], max(3, args.steps))
        V_seg, T_seg = traversal_work(dev_mesh[kind], qk[::3])
        launches[kind] = launch_record(f"{batch_instance(dev_mesh[kind])} ({kind}, {dev_mesh[kind].nt} tris, "
                                       f"{len(qk)} queries)", ms, rk, V_seg, T_seg)
    sink = torch.zeros(64, dtype=torch.uint8, device="cuda")
    measured = {k: ctx.ceiling_valu(k, sink) / 1e12 for k in ("fp32_fma", "fp64_fma")}
    workload = "plate+cylinder sweep, 120 cases"
    step_ops = sum(l["work"]["alg_lane_ops"] for l in launches.values())
    step_ms = sum(l["ms"] for l in launches.values())
    dom = max(launches.values(), key=lambda l: l["ms"])
    # the dominant kernel is the longer of the two launches; its roofline fraction is the line's
    roofline = {"bound": "alu", "achieved": dom["achieved_tlane_ops"], "peak": ALU_PEAK / 1e12, "unit": "Tlane-op/s",
                "frac": dom["frac"], "traffic": dom["hbm_bytes"], "kernel": dom["kernel"],
                "measured_ceilings": measured,
                "frac_of_measured_fp32_fma": dom["achieved_tlane_ops"] / measured["fp32_fma"],
                "step": {"kernel_ms": step_ms, "alg_lane_ops": step_ops,
                         "frac": step_ops / (step_ms / 1e3) / ALU_PEAK},
                "launches": launches,
                "work_units": {"per_particle_seeding": OPS_SEED, "per_preculled_particle": OPS_PRECULL,
                               "per_node_visit": OPS_NODE,
                               "per_triangle_test": OPS_TRI, "per_hit": OPS_HIT}}

    # accuracy of every case against the per-facet closed form
    # (relative error where the exact value is not ~0; error in units of the run's own sigma)
    errs, rels, zs, need = [], [], [], []
    for c, r in zip(ordered, res):
        ex = exact_cd(c["kind"], c["angle"], c["query"]["S"], c["query"]["alpha"])
        e = abs(r["CD"] - ex)
        errs.append(e)
        if abs(ex) > CD_REL_MIN:
            rels.append(e / abs(ex))
            need.append(3.0 * r["CD_sigma"] / abs(ex))
        zs.append(e / r["CD_sigma"] if r["CD_sigma"] > 0 else (0.0 if e < 1e-12 else math.inf))
    rels, zs, need = np.array(rels), np.array(zs), np.array(need)
    accuracy = {"max_abs_cd_err": float(max(errs)), "median_abs_cd_err": float(np.median(errs)),
                "max_rel_cd_err": float(rels.max()), "median_rel_cd_err": float(np.median(rels)),
                "cases_rel_err_le_1e-3": int((rels <= 1e-3).sum()), "cases_rel": int(len(rels)),
                "cases_3sigma_rel_le_1e-3": int((need <= 1e-3).sum()),
                "max_3sigma_rel": float(need.max()),
                "max_err_over_sigma": float(zs.max()), "cases_within_3_sigma": int((zs <= 3.0).sum()),
                "cases": len(errs),
                "max_cd_sigma": float(max(r["CD_sigma"] for r in res if not math.isnan(r["CD_sigma"]))),
                "note": f"relative error where |exact C_D| > {CD_REL_MIN}; absolute elsewhere"}

    # plain path: one query per launch, host sync per query
    plain = None
    if not args.no_plain:
        log("plain path")
        plain = plain_path(ctx, dev_mesh, cl, tunings)

    sat = sweep = None
    if not args.no_satellite:
        log("concave satellite")
        sat = config_satellite(ctx, args, measured)
        log("attitude sweep")
        sweep = config_sweep(ctx, args, measured, sat["mesh"])
        sat.pop("mesh")

    served = None
    if not args.no_served:
        log("served stream")
        served = served_measure(args, 100, 1000, [0.8], 300)
        served.update(served.pop("config"))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(cl, mm, satellite=not args.no_satellite)

    n_total = sum(n_case)
    line = {"metric": METRIC, "value": hits / dt, "unit": "hits/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"{workload}, {n_total:.4g} particles per step",
                       "meshes": "plate 2 tris, capped cylinder 256 tris", "S": [1, 3, 8],
                       "accommodation": [0.0, 1.0], "angles_deg": list(range(0, 91, 10)),
                       "T_inf_K": T_INF, "T_w_K": T_W,
                       "particles_per_case": ("fixed" if args.fixed_n else
                                              f"max({args.particles:g}, N with 3 sigma_rel <= 1e-3 from a "
                                              f"{args.pilot_particles:g}-particle pilot)"),
                       "particles_per_case_min_max": [min(n_case), max(n_case)],
                       "path": "batched persistent launch per mesh, HIP graph replay", "bvh": args.bvh},
            # query latency: the served stream's at 0.8 of its saturation throughput (the plate +
            # cylinder queries' own, one per launch on the plain path, are in plain_path)
            "query_ms_p50": served["query_ms_p50"] if served else None,
            "query_ms_p99": served["query_ms_p99"] if served else None,
            "segments_per_s": segments / dt, "particles_per_s": particles / dt,
            "accuracy": accuracy, "plain_path": plain,
            "batched_over_plain": (hits / dt) / plain["hits_per_s"] if plain else None,
            "tuning": tunings, "bvh_build_ms": build_ms,
            "roofline": roofline,
            "configs": {"concave_satellite": sat, "attitude_sweep": sweep, "served_stream": served},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
