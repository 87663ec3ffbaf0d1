"""Seeded synthetic inputs: meshes, attitudes and query records.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It holds no part of the drag method's arithmetic: it only
builds triangle meshes (the paper meshed its test shapes with Gmsh, Sec. III.C;
these procedural generators stand in for them), attitude quaternions and query
parameter records.

Conventions
-----------
* A mesh is ``(V, T)``: ``V`` float32 ``[nv, 3]`` metres in the body frame,
  ``T`` uint32 ``[nt, 3]`` vertex indices.  Closed meshes are wound so that
  ``(v1 - v0) x (v2 - v0)`` points out of the body.
* An attitude is a unit quaternion ``(w, x, y, z)`` of the rotation R from body
  to wind axes.  The free stream runs along +x of the wind axes, so its
  direction in the body frame is the first row of R.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Attitudes
# ---------------------------------------------------------------------------


def quat_from_matrix(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z) of a proper rotation matrix (Shepperd)."""
    R = np.asarray(R, dtype=np.float64)
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    cands = [tr, R[0, 0], R[1, 1], R[2, 2]]
    i = int(np.argmax(cands))
    if i == 0:
        s = math.sqrt(1.0 + tr) * 2.0
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif i == 1:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2.0
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif i == 2:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2.0
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2.0
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


def matrix_from_quat(q) -> np.ndarray:
    w, x, y, z = (float(v) for v in np.asarray(q, dtype=np.float64) / np.linalg.norm(q))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def quat_for_flow(u_body, up_hint=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Attitude whose free-stream direction in the body frame is ``u_body``."""
    u = np.asarray(u_body, dtype=np.float64)
    u = u / np.linalg.norm(u)
    h = np.asarray(up_hint, dtype=np.float64)
    if abs(np.dot(h, u)) > 0.9:
        h = np.array([0.0, 1.0, 0.0]) if abs(u[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e2 = np.cross(u, h)
    e2 /= np.linalg.norm(e2)
    e1 = np.cross(e2, u)
    R = np.stack([u, e1, e2])  # rows: wind axes in body coordinates
    return quat_from_matrix(R)


def flow_dir(q) -> np.ndarray:
    return matrix_from_quat(q)[0]


def flow_pitch_yaw(pitch_deg: float, yaw_deg: float) -> tuple:
    """Free-stream direction in the body frame for an attitude grid about the
    nominal flow -z (into the satellite's dish): pitch about y, then yaw about
    x, U = (sin p, cos p sin y, -cos p cos y)."""
    p, y = math.radians(pitch_deg), math.radians(yaw_deg)
    return (math.sin(p), math.cos(p) * math.sin(y), -math.cos(p) * math.cos(y))


def random_quats(n: int, seed: int) -> np.ndarray:
    """Uniform random rotations (Shoemake, Graphics Gems III, 1992)."""
    rng = np.random.default_rng(seed)
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    q[q[:, 0] < 0] *= -1
    return q


# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------


def _orient_outward(V: np.ndarray, T: np.ndarray, centre) -> np.ndarray:
    T = T.copy()
    v0, v1, v2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(v1 - v0, v2 - v0)
    flip = np.einsum("ij,ij->i", n, (v0 + v1 + v2) / 3.0 - np.asarray(centre)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def icosphere(subdivisions: int = 3, radius: float = 1.0):
    """Icosahedron (golden-ratio coordinates) with midpoint subdivision, vertices
    projected to the sphere.  3 subdivisions: 642 vertices, 1280 triangles."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    base = []
    for s1 in (-1, 1):
        for s2 in (-1, 1):
            base += [(0, s1, s2 * p), (s1, s2 * p, 0), (s2 * p, 0, s1)]
    V = np.array(base, dtype=np.float64)
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                if all(abs(np.linalg.norm(V[a] - V[b]) - 2.0) < 1e-9 for a, b in ((i, j), (j, k), (i, k))):
                    faces.append((i, j, k))
    T = np.array(faces, dtype=np.int64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    for _ in range(subdivisions):
        cache = {}
        verts = list(V)

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = (verts[a] + verts[b]) * 0.5
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in T:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        V = np.array(verts)
        T = np.array(nf, dtype=np.int64)
    T = _orient_outward(V, T, (0, 0, 0))
    return (V * radius).astype(np.float32), T.astype(np.uint32)


def plate(size: float = 1.0):
    """Square plate of side ``size`` in the plane z = 0 (two triangles)."""
    h = 0.5 * size
    V = np.array([(-h, -h, 0), (h, -h, 0), (h, h, 0), (-h, h, 0)], dtype=np.float32)
    T = np.array([(0, 1, 2), (0, 2, 3)], dtype=np.uint32)
    return V, T


def capped_cylinder(radius: float = 0.5, length: float = 1.0, segments: int = 64):
    """Closed cylinder, axis z, centred at the origin: 2*segments side triangles
    plus two fans of ``segments`` triangles (256 triangles for 64 segments)."""
    ang = 2.0 * np.pi * np.arange(segments) / segments
    ring = np.stack([radius * np.cos(ang), radius * np.sin(ang)], axis=1)
    z0, z1 = -0.5 * length, 0.5 * length
    V = np.concatenate([
        np.column_stack([ring, np.full(segments, z0)]),
        np.column_stack([ring, np.full(segments, z1)]),
        [[0.0, 0.0, z0], [0.0, 0.0, z1]],
    ])
    tris = []
    for i in range(segments):
        j = (i + 1) % segments
        tris += [(i, j, segments + j), (i, segments + j, segments + i)]
    cb, ct = 2 * segments, 2 * segments + 1
    for i in range(segments):
        j = (i + 1) % segments
        tris += [(cb, j, i), (ct, segments + i, segments + j)]
    T = _orient_outward(V, np.array(tris, dtype=np.int64), (0, 0, 0))
    return V.astype(np.float32), T.astype(np.uint32)


def hemisphere_cup(n_theta: int = 24, n_phi: int = 64, radius: float = 1.0):
    """Open hemispherical shell (a concave cup), z <= 0, rim in the plane z = 0.
    Seen from +z the inside is concave; a flow along -z enters the cup.
    Triangles are double-sided in the method, so winding only fixes n_g."""
    th = np.linspace(0.0, 0.5 * np.pi, n_theta + 1)  # polar angle from -z axis
    verts = [(0.0, 0.0, -radius)]
    for t in th[1:]:
        for k in range(n_phi):
            ph = 2.0 * np.pi * k / n_phi
            verts.append((radius * math.sin(t) * math.cos(ph), radius * math.sin(t) * math.sin(ph), -radius * math.cos(t)))
    V = np.array(verts)
    tris = []
    for k in range(n_phi):
        tris.append((0, 1 + k, 1 + (k + 1) % n_phi))
    for i in range(1, n_theta):
        a0, b0 = 1 + (i - 1) * n_phi, 1 + i * n_phi
        for k in range(n_phi):
            k1 = (k + 1) % n_phi
            tris += [(a0 + k, b0 + k, b0 + k1), (a0 + k, b0 + k1, a0 + k1)]
    T = _orient_outward(V, np.array(tris, dtype=np.int64), (0, 0, 0))
    return V.astype(np.float32), T.astype(np.uint32)


def _grid_rect(p0, du, dv, nu, nv):
    """Regular grid of a parallelogram p0 + s du + t dv, s, t in [0, 1]."""
    s = np.linspace(0.0, 1.0, nu + 1)
    t = np.linspace(0.0, 1.0, nv + 1)
    S, Tt = np.meshgrid(s, t, indexing="ij")
    V = np.asarray(p0) + S[..., None] * np.asarray(du) + Tt[..., None] * np.asarray(dv)
    V = V.reshape(-1, 3)
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
    a, b, c, d = idx[:-1, :-1], idx[1:, :-1], idx[1:, 1:], idx[:-1, 1:]
    T = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3), np.stack([a, c, d], -1).reshape(-1, 3)])
    return V, T


def satellite(target_tris: int = 50_000, jitter_sigma: float = 1e-3, seed: int = 0):
    """Procedural concave satellite: box bus [-0.5,0.5]x[-0.5,0.5]x[-1,1] m, two
    4 x 1 m panels in the plane x = 0 (y in +-[0.5, 4.5], z in [-0.5, 0.5]), and a
    paraboloid dish of diameter 2 m, z = 1 + rho^2 / (4 f), f = 0.6 m, opening
    towards +z.  The triangle budget is split about 14 % bus, 13 % each panel,
    60 % dish.  Vertices get seeded Gaussian jitter of ``jitter_sigma`` metres."""
    budget = max(int(target_tris), 200)
    parts_V, parts_T = [], []
    nv_off = 0

    def add(V, T):
        nonlocal nv_off
        parts_V.append(V)
        parts_T.append(T + nv_off)
        nv_off += len(V)

    # bus: six gridded faces, areas 1,1 (z faces) and 2,2,2,2 (side faces)
    bus_budget = 0.14 * budget
    g = max(1, int(round(math.sqrt(bus_budget / 20.0))))  # triangles = 2 g^2 (2 + 4 * 2) = 20 g^2
    faces = [
        ((-0.5, -0.5, -1.0), (0, 1, 0), (1, 0, 0), g, g),        # z = -1 (outward -z)
        ((-0.5, -0.5, 1.0), (1, 0, 0), (0, 1, 0), g, g),         # z = +1
        ((-0.5, -0.5, -1.0), (1, 0, 0), (0, 0, 2), g, 2 * g),    # y = -0.5
        ((-0.5, 0.5, -1.0), (0, 0, 2), (1, 0, 0), 2 * g, g),     # y = +0.5
        ((-0.5, -0.5, -1.0), (0, 0, 2), (0, 1, 0), 2 * g, g),    # x = -0.5
        ((0.5, -0.5, -1.0), (0, 1, 0), (0, 0, 2), g, 2 * g),     # x = +0.5
    ]
    bus_V, bus_T = [], []
    off = 0
    for p0, du, dv, nu, nvv in faces:
        V, T = _grid_rect(p0, du, dv, nu, nvv)
        bus_V.append(V)
        bus_T.append(T + off)
        off += len(V)
    bV = np.concatenate(bus_V)
    bT = np.concatenate(bus_T)
    # merge duplicate edge vertices so the bus is watertight
    key = np.round(bV * 1e6).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    bV = bV[first]
    bT = inv.reshape(-1)[bT]
    bT = _orient_outward(bV, bT, (0, 0, 0))
    add(bV, bT)

    # panels: 4 x 1 m, grid aspect 4:1
    panel_budget = 0.13 * budget
    pg = max(1, int(round(math.sqrt(panel_budget / 8.0))))  # 2 * (4 pg) * pg triangles
    for sgn in (-1.0, 1.0):
        y0 = 0.5 * sgn
        V, T = _grid_rect((0.0, y0, -0.5), (0.0, 4.0 * sgn, 0.0), (0.0, 0.0, 1.0), 4 * pg, pg)
        add(V, T)

    # dish: polar grid, rim at rho = 1
    dish_budget = 0.60 * budget
    nr = max(2, int(round(math.sqrt(dish_budget / (2.0 * 4.0)))))
    nphi = 4 * nr
    f = 0.6
    verts = [(0.0, 0.0, 1.0)]
    for i in range(1, nr + 1):
        rho = i / nr
        for k in range(nphi):
            ph = 2.0 * np.pi * k / nphi
            verts.append((rho * math.cos(ph), rho * math.sin(ph), 1.0 + rho * rho / (4.0 * f)))
    V = np.array(verts)
    tris = [(0, 1 + k, 1 + (k + 1) % nphi) for k in range(nphi)]
    for i in range(1, nr):
        a0, b0 = 1 + (i - 1) * nphi, 1 + i * nphi
        for k in range(nphi):
            k1 = (k + 1) % nphi
            tris += [(a0 + k, b0 + k, b0 + k1), (a0 + k, b0 + k1, a0 + k1)]
    add(V, np.array(tris, dtype=np.int64))

    V = np.concatenate(parts_V)
    T = np.concatenate(parts_T)
    if jitter_sigma > 0:
        rng = np.random.default_rng(seed)
        V = V + rng.normal(0.0, jitter_sigma, size=V.shape)
    return V.astype(np.float32), T.astype(np.uint32)


# ---------------------------------------------------------------------------
# Query records
# ---------------------------------------------------------------------------


BOX_CV = 2  # query flag: box control volume
ENERGY_ACC = 4  # query flag: diffuse re-emission with energy accommodation alpha_E


def query(q=(1.0, 0.0, 0.0, 0.0), S=5.0, T_inf=1000.0, T_w=300.0, alpha=1.0, n=100_000, seed=0,
          max_reflections=16, cv_center=(0.0, 0.0, 0.0), cv_radius=0.0, flags=0, cv_box=False,
          alpha_E=None) -> dict:
    """A drag query as a plain dict (both the GPU binding and the oracle wrapper
    accept it).  ``cv_radius <= 0`` asks for the automatic bounding sphere;
    ``cv_box`` seeds on an axis-aligned box instead (the cube of half-side
    ``cv_radius`` about ``cv_center``, or the widened vertex box); ``alpha_E``
    (when given) is the energy accommodation of diffuse re-emission (full, 1,
    otherwise)."""
    return dict(q=tuple(float(v) for v in q), S=float(S), T_inf=float(T_inf), T_w=float(T_w),
                alpha=float(alpha), n=int(n), seed=int(seed), max_reflections=int(max_reflections),
                cv_center=tuple(float(v) for v in cv_center), cv_radius=float(cv_radius),
                flags=int(flags) | (BOX_CV if cv_box else 0) | (ENERGY_ACC if alpha_E is not None else 0),
                alpha_E=float(1.0 if alpha_E is None else alpha_E))


def plate_cases(angles_deg=range(0, 91, 10), S_values=(1.0, 3.0, 8.0), n=10_000_000):
    """Flat-plate incidence sweep: free stream (sin a, 0, -cos a), a from the normal."""
    out = []
    for S in S_values:
        for acc in (0.0, 1.0):
            for a in angles_deg:
                r = math.radians(a)
                out.append(dict(mesh="plate", angle=float(a), S=S, alpha=acc,
                                q=quat_for_flow((math.sin(r), 0.0, -math.cos(r))), n=n))
    return out


def cylinder_cases(angles_deg=range(0, 91, 10), S_values=(1.0, 3.0, 8.0), n=10_000_000):
    """Capped-cylinder sweep: free stream (sin a, 0, cos a), a from the axis."""
    out = []
    for S in S_values:
        for acc in (0.0, 1.0):
            for a in angles_deg:
                r = math.radians(a)
                out.append(dict(mesh="cylinder", angle=float(a), S=S, alpha=acc,
                                q=quat_for_flow((math.sin(r), 0.0, math.cos(r))), n=n))
    return out
