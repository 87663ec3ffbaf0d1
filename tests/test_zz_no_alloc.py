"""The batched entry point without allocation (tpmc_batch_run_noalloc, whose
workspace is the library's static device array) against the batched path with
a caller workspace (tpmc_batch_create / launch / results): same kernels, so
every result must be bit-identical.  Two calls in a row on one GPU, the second
with a smaller input, so the second call runs over what the first left in the
array; per-triangle and totals-only tallies; a request larger than the array
is rejected before any work is enqueued."""
import math

import numpy as np
import pytest

from paper_1312_3691_amd import inputs as I

pytestmark = pytest.mark.gpu
KEYS = ("F_over_q", "M_over_q", "Fhat", "Mhat", "CD", "CD_sigma", "Gamma_hat", "rays", "hits", "segments", "missed",
        "escaped", "capped", "Qhat", "CH", "CH_sigma", "tr_capped", "guard_trips")


@pytest.fixture(scope="module")
def T():
    from paper_1312_3691_amd import tpmc
    return tpmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def _queries(n_list, flags=0, seed0=300):
    quats = I.random_quats(len(n_list), 41)
    S = 2.0 + 8.0 * np.random.default_rng(42).random(len(n_list))
    return [I.query(q=tuple(quats[i]), S=float(S[i]), alpha=0.9, n=int(n), seed=seed0 + i, flags=flags)
            for i, n in enumerate(n_list)]


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k]), equal_nan=True), (k, a[k], b[k])


@pytest.mark.parametrize("flags", [0, 1], ids=["per_triangle", "totals_only"])
def test_noalloc_equals_batched_path(ctx, T, flags):
    V, Tr = I.satellite(3000)
    mesh = ctx.build_mesh(V, Tr)
    x_ref, A_ref = (0.2, -0.1, 0.3), 1.5
    for label, ns in (("large", [70_001, 16_384, 16_385, 5_000, 1, 40_000]), ("small", [9_000, 123])):
        qs = _queries(ns, flags=flags)
        print(f"no-alloc vs batched: {label} input, {len(qs)} queries, flags {flags}", flush=True)
        b = T.Batch(mesh, qs)
        ref = b.launch().results(x_ref=x_ref, A_ref=A_ref)
        b.close()
        got = T.batch_run_noalloc(mesh, qs, x_ref=x_ref, A_ref=A_ref)
        assert len(got) == len(qs)
        for a, c in zip(ref, got):
            _same(a, c)
            assert c["rays"] > 0 and c["tr_capped"] == 0 and c["guard_trips"] == 0


def test_noalloc_tiny_mesh_then_rejects_oversize(ctx, T):
    # two-triangle plate (per-lane tallies), twice in a row with a smaller second input
    V, Tr = I.plate()
    mesh = ctx.build_mesh(V, Tr)
    a = math.radians(30.0)
    for n in (200_003, 1_001):
        q = [I.query(q=I.quat_for_flow((math.sin(a), 0, -math.cos(a))), S=3.0, alpha=1.0, n=n, seed=n)]
        print(f"no-alloc vs batched: plate, N = {n}", flush=True)
        b = T.Batch(mesh, q)
        ref = b.launch().results()
        b.close()
        _same(ref[0], T.batch_run_noalloc(mesh, q)[0])
    # 50k-triangle mesh: 12 per-triangle queries need more than the static array
    Vs, Ts = I.satellite(50_000)
    big = ctx.build_mesh(Vs, Ts)
    qs = _queries([1000] * 12)
    assert 12 * 7 * 8 * len(Ts) > T.NOALLOC_MAX_BYTES
    with pytest.raises(T.TpmcError) as e:
        T.batch_run_noalloc(big, qs)
    assert e.value.status == 4
    # and the array is still usable afterwards
    q = _queries([2000])
    b = T.Batch(big, q)
    ref = b.launch().results()
    b.close()
    _same(ref[0], T.batch_run_noalloc(big, q)[0])
