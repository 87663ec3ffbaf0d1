"""The batched path's two-stage seeding (an FP32 estimate of each particle's
first ray tested against the BVH root's boxes grown by 2 % of the CV radius;
only the particles it does not rule out are seeded exactly and traced).

* The margin rests on the estimate's error: measured over 1e5 particles per
  case (tpmc_precull_check), the estimated ray stays within a hundredth of
  the margin of the exact one (Sec. III.A.1-3 in FP64) for every mesh, S
  from 0 to 30 and attitude, and the estimate covers nearly every particle
  at S = 0 and for S inside its tables (it leaves the others, and
  0 < S < 0.25, to the exact seeding).  Its latitude comes from a fine
  table without iteration, so S midway between the table's rows is where it
  errs most: swept across the table, it stays within a twentieth of the
  margin.
* The particles it removes are misses either way: batched results equal the
  plain path's bit for bit (every field but the work count), on flat, convex
  and concave bodies at grazing and head-on incidence; the plain path
  reports no removed particles, the batched path some (never more than its
  misses), and the cylinder, where most particles reach the box, switches
  the estimate off after a few batches.
"""
import math

import numpy as np
import pytest

from paper_1312_3691_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_1312_3691_amd import tpmc
    return tpmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


MESHES = {"plate": I.plate, "cylinder": I.capped_cylinder, "satellite": lambda: I.satellite(4000),
          "icosphere": lambda: I.icosphere(3)}


@pytest.mark.parametrize("kind", sorted(MESHES))
def test_estimate_error_far_below_margin(ctx, T, kind):
    mesh = ctx.build_mesh(*MESHES[kind]())
    quats = I.random_quats(2, 77)
    n = 100_000
    for S in (0.0, 0.2, 1.0, 3.0, 8.0, 10.0, 12.0, 30.0):
        for k, qq in enumerate(quats):
            q = I.query(q=tuple(qq), S=S, alpha=0.9, n=n, seed=31 + k)
            worst, covered = mesh.precull_check(q)
            print(f"{kind} S={S} attitude {k}: max error / margin {worst:.3e}, covered {covered}", flush=True)
            assert worst < 1e-2, (kind, S, k, worst)
            if S == 0.0 or 1.0 <= S <= 10.0:  # the estimate's range: S = 0 and S inside the start tables
                assert covered >= 0.9 * n, (kind, S, k, covered)
    mesh.close()


def test_estimate_error_across_the_latitude_table(ctx, T):
    """The estimate takes the latitude from a fine table as it is (cubic in
    ln S between its rows, linear in the logit), so its error peaks where the
    interpolation is poorest: midway between rows.  Over S at every fourth
    row of the table and midway between rows (0.25 <= S <= 10), two attitudes
    each, the estimated rays stay within a twentieth of the margin; the worst
    over the same S at every row and half row, 2e4 particles each, measured
    1.3e-2 of the margin."""
    mesh = ctx.build_mesh(*MESHES["cylinder"]())
    quats = I.random_quats(2, 5)
    worst = (0.0, None)
    k0 = math.ceil((math.log(0.25) + 1.45) / 0.01)
    k1 = math.floor((math.log(10.0) + 1.45) / 0.01)
    n = 10_000
    for k in range(k0, k1 + 1, 4):
        S = math.exp(-1.45 + 0.01 * k)  # odd k: midway between rows (kLatFDL = 0.02)
        for a, qq in enumerate(quats):
            w, covered = mesh.precull_check(I.query(q=tuple(qq), S=S, alpha=0.9, n=n, seed=7 + a))
            assert covered >= 0.9 * n, (S, a, covered)
            worst = max(worst, (w, (round(S, 4), a)))
    print(f"largest error / margin {worst[0]:.3e} at S, attitude {worst[1]}", flush=True)
    assert worst[0] < 5e-2, worst
    mesh.close()


def _grazing(angle_deg):
    a = math.radians(angle_deg)
    return I.quat_for_flow((math.sin(a), 0.0, -math.cos(a)))


def test_batched_equals_plain_with_precull(ctx, T):
    cases = [("plate", [I.query(q=_grazing(ang), S=S, alpha=acc, n=300_007, seed=11 + i)
                        for i, (ang, S, acc) in enumerate([(80, 3.0, 1.0), (60, 8.0, 0.0), (0, 1.0, 1.0),
                                                           (89, 8.0, 1.0)])]),
             ("satellite", [I.query(q=tuple(qq), S=S, alpha=0.9, n=200_003, seed=50 + i)
                            for i, (qq, S) in enumerate(zip(I.random_quats(3, 8), (2.0, 7.0, 10.0)))]),
             ("cylinder", [I.query(q=_grazing(ang), S=S, alpha=1.0, n=400_009, seed=70 + i)
                           for i, (ang, S) in enumerate([(30, 3.0), (90, 8.0)])])]
    for kind, qs in cases:
        mesh = ctx.build_mesh(*MESHES[kind]())
        plain, pr = T.run(mesh, qs, A_ref=1.0)
        pr.close()
        b = T.Batch(mesh, qs)
        batched = b.launch(use_graph=True).results(A_ref=1.0)
        b.close()
        for q, p, g in zip(qs, plain, batched):
            for k in T.same_on_every_path(p):
                assert np.array_equal(np.asarray(p[k]), np.asarray(g[k])), (kind, q["seed"], k)
            assert p["preculled"] == 0
            assert g["preculled"] <= g["missed"]
            print(f"{kind} seed {q['seed']}: missed {g['missed']}, preculled {g['preculled']} of {q['n']}", flush=True)
            if kind == "cylinder":
                assert g["preculled"] < 0.1 * q["n"], g["preculled"]  # switched off: most particles reach the box
            else:
                assert g["preculled"] > 0.2 * g["missed"], (g["preculled"], g["missed"])
        mesh.close()
