"""Writes bench_cases_exact.json: the per-facet exact C_D (drag area F.U/q,
A_ref = 1 m^2) of every case of the plate + capped-cylinder benchmark sweep,
the reference its accuracy report compares against.  Calls only
oracle/closed_forms.py and the input generators (no GPU code).  Run from the
repository root:
    python tests/golden/make_bench_exact.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import closed_forms as CF  # noqa: E402
from paper_1312_3691_amd import inputs as I  # noqa: E402

T_INF, T_W = 1000.0, 300.0


def main():
    tau = math.sqrt(T_W / T_INF)
    out = {"_note": "T_inf = 1000 K, T_w = 300 K.  Plate: double-sided 1 x 1 m, alpha from the normal, free "
                    "stream (sin a, 0, -cos a).  Capped cylinder: r = 0.5, L = 1, 64 segments, angle from the "
                    "axis, free stream (sin a, 0, cos a).  alpha = accommodation (0 specular, 1 diffuse).",
           "cases": []}
    meshes = {"plate": I.plate(), "cylinder": I.capped_cylinder()}
    for kind, gen in (("plate", I.plate_cases), ("cylinder", I.cylinder_cases)):
        V, T = meshes[kind]
        for c in gen(n=1):
            U = I.flow_dir(c["q"])
            F, _, _ = CF.mesh_force(V, T, U, c["S"], tau, c["alpha"], two_sided=(kind == "plate"))
            out["cases"].append({"kind": kind, "angle": float(c["angle"]), "S": float(c["S"]),
                                 "alpha": float(c["alpha"]), "CD": float(F @ U)})
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_cases_exact.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
