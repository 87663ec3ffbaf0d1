"""Writes closed_forms.json: free-molecular closed-form drag values used as
expected values by the oracle tests.  Calls only oracle/closed_forms.py and the
input generators (no GPU code).  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import closed_forms as CF  # noqa: E402
from paper_1312_3691_amd import inputs as I  # noqa: E402

TAU = math.sqrt(300.0 / 1000.0)


def main():
    out = {"_note": "T_inf = 1000 K, T_w = 300 K (tau^2 = 0.3).  Plate: double-sided 1 x 1 m, A_ref = 1 m^2, "
                    "alpha from the normal (eq. plate with the re-emission term halved). Sphere: A_ref = pi r^2 "
                    "(eq. sphere). Cylinder: r = 0.5, L = 1, 64 segments, per-facet exact drag area F.U/q, "
                    "angle from the axis.  Icosphere: subdivision 3, r = 1, free stream +x."}
    plate = []
    for S in (1.0, 3.0, 8.0):
        for a in range(0, 91, 10):
            r = math.radians(a)
            U = (math.sin(r), 0.0, -math.cos(r))
            V, T = I.plate()
            Fd, _, _ = CF.mesh_force(V, T, U, S, TAU, 1.0, two_sided=True)
            Fs, _, _ = CF.mesh_force(V, T, U, S, TAU, 0.0, two_sided=True)
            import numpy as np
            U = np.array(U)
            plate.append(dict(S=S, alpha=a, cd_diffuse=CF.plate_cd(S, a, TAU), cd_printed=CF.plate_cd_printed(S, a, TAU),
                              cd_specular=CF.plate_cd_specular(S, a),
                              cl_diffuse=float(np.linalg.norm(Fd - (Fd @ U) * U)),
                              cl_specular=float(np.linalg.norm(Fs - (Fs @ U) * U))))
    out["plate"] = plate
    out["sphere"] = [dict(S=S, cd=CF.sphere_cd(S, TAU), cd_specular=CF.sphere_cd_specular(S)) for S in (2, 3, 5, 7, 8, 10)]
    V, T = I.capped_cylinder()
    cyl = []
    for S in (1.0, 3.0, 8.0):
        for a in range(0, 91, 10):
            r = math.radians(a)
            U = (math.sin(r), 0.0, math.cos(r))
            Fd, _, _ = CF.mesh_force(V, T, U, S, TAU, 1.0)
            Fs, _, _ = CF.mesh_force(V, T, U, S, TAU, 0.0)
            cyl.append(dict(S=S, angle=a, cd_diffuse=float(Fd @ U), cd_specular=float(Fs @ U)))
    out["cylinder"] = cyl
    V, T = I.icosphere(3)
    F, _, _ = CF.mesh_force(V, T, (1.0, 0.0, 0.0), 5.0, TAU, 1.0)
    out["icosphere3_S5"] = dict(cd_facet=float(F[0] / math.pi), cd_smooth=CF.sphere_cd(5.0, TAU))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
