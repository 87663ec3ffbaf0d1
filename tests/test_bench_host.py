"""Host checks of the benchmark's accounting (no GPU): the work model behind
the roofline fraction, the phase-probe summary, the guard on stored HBM
traffic, and the single-GPU contract of the command line."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench as B  # noqa: E402


def test_peak_is_one_lane_op_per_clock_on_every_lane():
    assert B.ALU_PEAK == pytest.approx(256 * 64 * 2.4e9)
    assert B.ALU_PEAK / 1e12 == pytest.approx(39.3216)


def test_launch_record_work_model():
    """A particle the estimate removes costs OPS_PRECULL in place of an exact
    seeding and of the one root-node visit it would have made; everything
    else is counted per particle, node visit, triangle test and hit."""
    res = [{"rays": 1000, "segments": 1500, "hits": 600, "preculled": 300},
           {"rays": 500, "segments": 800, "hits": 350, "preculled": 0}]
    V, T = 9.5, 3.25
    rec = B.launch_record("batch_kernel<16, 1> (test)", 2.0, res, V, T)
    particles, pre, segments, hits = 1500, 300, 2300, 950
    ops = ((particles - pre) * 950.0 + pre * 485.0 + segments * (V * 40.0 + T * 45.0) - pre * 40.0
           + hits * 225.0)
    assert rec["work"]["alg_lane_ops"] == pytest.approx(ops)
    assert rec["frac"] == pytest.approx(ops / 2e-3 / (256 * 64 * 2.4e9))
    assert rec["achieved_tlane_ops"] == pytest.approx(ops / 2e-3 / 1e12)
    assert rec["work"]["particles"] == particles and rec["work"]["preculled"] == pre
    # with no removed particle the model is the plain path's
    plain = B.launch_record("trace", 1.0, [{"rays": 10, "segments": 12, "hits": 5}], 2.0, 1.0)
    assert plain["work"]["alg_lane_ops"] == pytest.approx(10 * 950 + 12 * (80 + 45) + 5 * 225)
    assert plain["hbm_bytes"] is None  # not a batch_kernel instance


def test_stored_traffic_only_for_unchanged_kernels(monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(path))
    inst, e = next(iter(d["batch_kernel"].items()))
    monkeypatch.setattr(B, "kernel_hash", lambda: d["kernel_hash"])
    assert B.stored_traffic(inst) == pytest.approx(e["fetch_bytes"] + e["write_bytes"])
    assert B.stored_traffic("batch_kernel<99, 9>") is None
    monkeypatch.setattr(B, "kernel_hash", lambda: "0" * 16)  # sources changed since the counter runs
    assert B.stored_traffic(inst) is None


def test_stored_traffic_matches_the_committed_sources():
    """profiles/traffic.json was measured on the kernels as committed."""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert d["kernel_hash"] == B.kernel_hash()


def test_probe_record_shares_and_means():
    p = {k: 0 for k in ("waves", "cycles", "claim_cycles", "claims", "trav_cycles", "trav_steps", "trav_lanes",
                        "leaf_cycles", "leaf_passes", "leaf_lanes", "serve_cycles", "serves", "serve_lanes",
                        "est_cycles", "est_batches", "est_particles", "est_kept", "seed_cycles", "seed_batches",
                        "seed_particles", "seed_kept", "assign_cycles", "assigns", "assign_lanes")}
    p.update(waves=4, cycles=1000, claim_cycles=10, claims=2, trav_cycles=300, trav_steps=20, trav_lanes=800,
             serve_cycles=100, serves=5, serve_lanes=100, est_cycles=200, est_batches=4, est_particles=256,
             est_kept=64, seed_cycles=250, seed_batches=1, seed_particles=64, seed_kept=60, assign_cycles=40,
             assigns=2, assign_lanes=60)
    r = B.probe_record(p, 256, 1.0)
    assert r["per_64_particles"]["traversal_steps"] == pytest.approx(5.0)
    assert r["mean_lanes"]["traversal"] == pytest.approx(40.0)
    assert r["mean_lanes"]["leaf"] is None  # no leaf phase ran
    assert r["estimate_kept"] == pytest.approx(0.25) and r["seeding_kept"] == pytest.approx(60 / 64)
    assert sum(r["share"].values()) == pytest.approx(1.0)
    assert r["share"]["other"] == pytest.approx(0.1)
    assert r["wave_clock_ghz"] == pytest.approx(1000 / 4 / 1e-3 / 1e9)


def test_more_than_one_gpu_is_refused():
    cp = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                        text=True, timeout=120, cwd=ROOT)
    assert cp.returncode == 2
    assert "one GPU only" in cp.stderr and cp.stdout == ""
