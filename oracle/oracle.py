"""ctypes wrapper of the FP64 CPU oracle (``tpmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  It shares no code with the HIP path;
the only thing both sides take from a common place is the synthetic input
(``paper_1312_3691_amd.inputs``).

Parallelism: the particle range is split into a fixed number of chunks (not
into one chunk per thread), each chunk is traced independently and the chunk
sums are merged in chunk order, so results do not depend on the thread count.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

N_CHUNKS = 64
BOX_CV_FLAG = 2  # query flag: box control volume
ENERGY_ACC_FLAG = 4  # query flag: diffuse re-emission with energy accommodation alpha_E


class OrcQuery(ctypes.Structure):
    _fields_ = [("q_wxyz", ctypes.c_double * 4), ("S", ctypes.c_double), ("T_inf", ctypes.c_double),
                ("T_w", ctypes.c_double), ("alpha", ctypes.c_double), ("n_particles", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("max_reflections", ctypes.c_uint32), ("round_fp32", ctypes.c_int32),
                ("cv_center", ctypes.c_double * 3), ("cv_radius", ctypes.c_double), ("cv_box", ctypes.c_int32),
                ("energy_acc", ctypes.c_int32), ("alpha_E", ctypes.c_double)]


class OrcConsts(ctypes.Structure):
    _fields_ = [("U", ctypes.c_double * 3), ("e1", ctypes.c_double * 3), ("e2", ctypes.c_double * 3),
                ("S", ctypes.c_double), ("tau", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Z", ctypes.c_double), ("Gamma_hat", ctypes.c_double), ("c0", ctypes.c_double * 3),
                ("r", ctypes.c_double), ("N", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("rmax", ctypes.c_uint32), ("round_fp32", ctypes.c_int32), ("s_zero", ctypes.c_int32),
                ("box", ctypes.c_int32), ("h", ctypes.c_double * 3), ("face_s", ctypes.c_double * 6),
                ("face_cum", ctypes.c_double * 6), ("eacc", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("alpha_E", ctypes.c_double)]


class OrcScalars(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("D_c", ctypes.c_double), ("D2", ctypes.c_double),
                ("D2_c", ctypes.c_double), ("rays", ctypes.c_uint64), ("hits", ctypes.c_uint64),
                ("segments", ctypes.c_uint64), ("missed", ctypes.c_uint64), ("escaped", ctypes.c_uint64),
                ("capped", ctypes.c_uint64), ("E", ctypes.c_double), ("E_c", ctypes.c_double),
                ("E2", ctypes.c_double), ("E2_c", ctypes.c_double)]


class OrcResult(ctypes.Structure):
    _fields_ = [("F_over_q", ctypes.c_double * 3), ("M_over_q", ctypes.c_double * 3),
                ("Fhat", ctypes.c_double * 3), ("CD", ctypes.c_double), ("CD_sigma", ctypes.c_double),
                ("Gamma_hat", ctypes.c_double), ("rays", ctypes.c_uint64), ("hits", ctypes.c_uint64),
                ("segments", ctypes.c_uint64), ("missed", ctypes.c_uint64), ("escaped", ctypes.c_uint64),
                ("capped", ctypes.c_uint64), ("Qhat", ctypes.c_double), ("CH", ctypes.c_double),
                ("CH_sigma", ctypes.c_double), ("Mhat", ctypes.c_double * 3)]


_ip = ctypes.POINTER(ctypes.c_int32)
_dpt = ctypes.POINTER(ctypes.c_double)


class OrcParticleOut(ctypes.Structure):
    _fields_ = [("first_tri", _ip), ("nhits", _ip), ("D", _dpt), ("E", _dpt), ("w_entry", _dpt),
                ("w_exit", _dpt), ("dw", _dpt), ("L", _dpt)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
            for name in ("orc_chi", "orc_Z"):
                getattr(L, name).argtypes = [ctypes.c_double]
                getattr(L, name).restype = ctypes.c_double
            for name in ("orc_gamma_hat", "orc_F_mu", "orc_inv_F_mu", "orc_F_n", "orc_inv_F_n"):
                getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_double]
                getattr(L, name).restype = ctypes.c_double
            L.orc_setup.argtypes = [ctypes.POINTER(OrcQuery), dp, ctypes.c_uint64, ctypes.POINTER(OrcConsts)]
            L.orc_setup.restype = ctypes.c_int
            L.orc_seed_range.argtypes = [ctypes.POINTER(OrcConsts), ctypes.c_uint64, ctypes.c_uint64, dp, dp, dp]
            L.orc_reflect.argtypes = [ctypes.POINTER(OrcConsts), ctypes.c_uint64, ctypes.c_uint32, dp, dp, dp]
            L.orc_intersect.argtypes = [dp, dp, dp, dp, dp, dp, dp]
            L.orc_intersect.restype = ctypes.c_int
            up = ctypes.POINTER(ctypes.c_uint32)
            L.orc_bvh_build.argtypes = [dp, ctypes.c_uint64, up, ctypes.c_uint64]
            L.orc_bvh_build.restype = ctypes.c_void_p
            L.orc_bvh_free.argtypes = [ctypes.c_void_p]
            L.orc_bvh_nodes.argtypes = [ctypes.c_void_p]
            L.orc_bvh_nodes.restype = ctypes.c_uint64
            L.orc_closest.argtypes = [dp, up, ctypes.c_uint64, ctypes.c_void_p, dp, dp, ctypes.c_int64, dp, dp]
            L.orc_closest.restype = ctypes.c_int64
            L.orc_trace_range.argtypes = [dp, ctypes.c_uint64, up, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.POINTER(OrcConsts), ctypes.c_uint64, ctypes.c_uint64, dp, dp,
                                          ctypes.POINTER(OrcScalars), ctypes.POINTER(OrcParticleOut)]
            L.orc_trace_range.restype = ctypes.c_int
            L.orc_finalize.argtypes = [ctypes.POINTER(OrcConsts), dp, ctypes.c_uint64, ctypes.POINTER(OrcScalars),
                                       dp, ctypes.c_double, ctypes.POINTER(OrcResult)]
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def make_query(qd: dict, round_fp32: bool = True) -> OrcQuery:
    q = OrcQuery()
    q.q_wxyz[:] = [float(v) for v in qd["q"]]
    q.S, q.T_inf, q.T_w, q.alpha = qd["S"], qd["T_inf"], qd["T_w"], qd["alpha"]
    q.n_particles, q.seed = int(qd["n"]), int(qd["seed"])
    q.max_reflections = int(qd.get("max_reflections", 16))
    q.round_fp32 = 1 if round_fp32 else 0
    q.cv_center[:] = [float(v) for v in qd.get("cv_center", (0.0, 0.0, 0.0))]
    q.cv_radius = float(qd.get("cv_radius", 0.0))
    q.cv_box = 1 if int(qd.get("flags", 0)) & BOX_CV_FLAG else 0
    q.energy_acc = 1 if int(qd.get("flags", 0)) & ENERGY_ACC_FLAG else 0
    q.alpha_E = float(qd.get("alpha_E", 1.0))
    return q


def setup(V, qd: dict, round_fp32: bool = True) -> OrcConsts:
    Vd = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1, 3))
    c = OrcConsts()
    q = make_query(qd, round_fp32)
    if lib().orc_setup(ctypes.byref(q), _dp(Vd), Vd.shape[0], ctypes.byref(c)) != 0:
        raise ValueError("oracle: invalid query")
    return c


def consts_dict(c: OrcConsts) -> dict:
    return {f: (list(getattr(c, f)) if isinstance(getattr(c, f), ctypes.Array) else getattr(c, f))
            for f, _ in c._fields_}


def seed(V, qd: dict, p0: int = 0, p1: int | None = None, round_fp32: bool = True):
    """Seeded particle states (x, w) in FP64 (FP32-rounded values when round_fp32)."""
    c = setup(V, qd, round_fp32)
    p1 = int(qd["n"]) if p1 is None else int(p1)
    n = p1 - p0
    x = np.zeros((n, 3))
    w = np.zeros((n, 3))
    mu = np.zeros(n)
    lib().orc_seed_range(ctypes.byref(c), p0, p1, _dp(x), _dp(w), _dp(mu))
    return x, w, mu


def reflect(V, qd: dict, pid: int, bounce: int, w_in, n_g):
    c = setup(V, qd)
    wi = np.ascontiguousarray(w_in, dtype=np.float64)
    ng = np.ascontiguousarray(n_g, dtype=np.float64)
    wo = np.zeros(3)
    lib().orc_reflect(ctypes.byref(c), pid, bounce, _dp(wi), _dp(ng), _dp(wo))
    return wo


def intersect(o, d, v0, v1, v2):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (o, d, v0, v1, v2)]
    t = np.zeros(1)
    b = np.zeros(3)
    hit = lib().orc_intersect(*[_dp(a) for a in arrs], _dp(t), _dp(b))
    return (float(t[0]), b) if hit else None


# Meshes above this many triangles are traced through the oracle's own
# median-split hierarchy unless a call says otherwise (same closest hits).
BVH_MIN_TRIS = 2000


class BVH:
    """The oracle's median-split hierarchy of one mesh (FP64, built on the host).
    Keeps its own copies of the vertex and index arrays."""

    def __init__(self, V, T):
        self.V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1, 3))
        self.T = np.ascontiguousarray(np.asarray(T, dtype=np.uint32).reshape(-1, 3))
        self._h = lib().orc_bvh_build(_dp(self.V), self.V.shape[0],
                                      self.T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), self.T.shape[0])
        self.nodes = int(lib().orc_bvh_nodes(self._h))

    @property
    def handle(self):
        return self._h

    def matches(self, V, T) -> bool:
        V = np.asarray(V, dtype=np.float64).reshape(-1, 3)
        T = np.asarray(T).reshape(-1, 3)
        return V.shape == self.V.shape and T.shape == self.T.shape and np.array_equal(V, self.V) and \
            np.array_equal(T, self.T)

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.orc_bvh_free(h)


def closest(V, T, o, d, prev=-1, bvh=None):
    """Closest hit of one ray (triangle index or -1, t, barycentrics), by brute
    force or through ``bvh`` (a ``BVH`` of the same mesh)."""
    Vd = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1, 3))
    Ti = np.ascontiguousarray(np.asarray(T, dtype=np.uint32).reshape(-1, 3))
    oo = np.ascontiguousarray(o, dtype=np.float64)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    t = np.zeros(1)
    b = np.zeros(3)
    k = lib().orc_closest(_dp(Vd), Ti.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), Ti.shape[0],
                          bvh.handle if bvh is not None else None, _dp(oo), _dp(dd), int(prev), _dp(t), _dp(b))
    return int(k), float(t[0]), b


def _neumaier_merge(parts):
    s = np.zeros_like(parts[0])
    c = np.zeros_like(parts[0])
    for x in parts:
        t = s + x
        big = np.abs(s) >= np.abs(x)
        c += np.where(big, (s - t) + x, (x - t) + s)
        s = t
    return s + c


def run(V, T, qd: dict, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0, threads: int | None = None,
        p_range=None, per_particle: bool = False, round_fp32: bool = True, n_chunks: int = N_CHUNKS,
        bvh="auto", exits: bool = False) -> dict:
    """Run the oracle on particles ``p_range`` (default all N) of query ``qd``.

    Returns a dict with the finalised result (computed with the query's N, so
    it is only a drag estimate when ``p_range`` covers all particles), the raw
    per-triangle sums ``tri`` ([nt, 7]: dw xyz, p x dw xyz, count), the scalar
    sums and, if asked, per-particle ``first_tri``, ``nhits``, ``D`` and ``E``;
    with ``exits`` also ``w_entry``, ``w_exit``, ``dw`` and ``L`` ([n, 3]).

    ``bvh``: "auto" traces meshes above BVH_MIN_TRIS triangles through the
    oracle's hierarchy, True / False force it on / off, or a prebuilt ``BVH``
    of the same mesh.  The closest hits, hence the results, do not depend on it.
    """
    L = lib()
    Vd = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1, 3))
    Ti = np.ascontiguousarray(np.asarray(T, dtype=np.uint32).reshape(-1, 3))
    nt = Ti.shape[0]
    if isinstance(bvh, BVH):
        if not bvh.matches(Vd, Ti):
            raise ValueError("oracle: the hierarchy was built for another mesh")
        tree = bvh
    elif bvh is True or (bvh == "auto" and nt > BVH_MIN_TRIS):
        tree = BVH(Vd, Ti)
    else:
        tree = None
    c = setup(Vd, qd, round_fp32)
    p0, p1 = (0, int(qd["n"])) if p_range is None else (int(p_range[0]), int(p_range[1]))
    n = p1 - p0
    k = max(1, min(n_chunks, n))
    bounds = [p0 + (n * i) // k for i in range(k + 1)]
    first = np.full(n, -1, np.int32) if per_particle else None
    nh = np.zeros(n, np.int32) if per_particle else None
    Dp = np.zeros(n) if per_particle else None
    Ep = np.zeros(n) if per_particle else None
    vec = {name: np.zeros((n, 3)) for name in ("w_entry", "w_exit", "dw", "L")} if exits else {}

    def work(i):
        a, b = bounds[i], bounds[i + 1]
        ts = np.zeros(nt * 7)
        tc = np.zeros(nt * 7)
        sc = OrcScalars()
        po = OrcParticleOut()
        if per_particle:
            po.first_tri = first[a - p0:].ctypes.data_as(_ip)
            po.nhits = nh[a - p0:].ctypes.data_as(_ip)
            po.D = _dp(Dp[a - p0:])
            po.E = _dp(Ep[a - p0:])
        for name, arr in vec.items():
            setattr(po, name, _dp(arr[a - p0:]))
        L.orc_trace_range(_dp(Vd), Vd.shape[0], Ti.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), nt,
                          tree.handle if tree is not None else None, ctypes.byref(c), a, b, _dp(ts), _dp(tc),
                          ctypes.byref(sc), ctypes.byref(po))
        return ts + tc, sc

    nthreads = threads or min(os.cpu_count() or 1, 16)
    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        parts = list(ex.map(work, range(k)))
    tri = _neumaier_merge([p[0] for p in parts])
    tot = OrcScalars()
    Ds = _neumaier_merge([np.array([p[1].D + p[1].D_c, p[1].D2 + p[1].D2_c, p[1].E + p[1].E_c, p[1].E2 + p[1].E2_c])
                          for p in parts])
    tot.D, tot.D2, tot.E, tot.E2 = float(Ds[0]), float(Ds[1]), float(Ds[2]), float(Ds[3])
    for f in ("rays", "hits", "segments", "missed", "escaped", "capped"):
        setattr(tot, f, sum(getattr(p[1], f) for p in parts))
    res = OrcResult()
    xr = np.ascontiguousarray(x_ref, dtype=np.float64)
    L.orc_finalize(ctypes.byref(c), _dp(tri), nt, ctypes.byref(tot), _dp(xr), float(A_ref), ctypes.byref(res))
    out = {f: (np.array(getattr(res, f)) if isinstance(getattr(res, f), ctypes.Array) else getattr(res, f))
           for f, _ in res._fields_}
    out.update(tri=tri.reshape(nt, 7), D_sum=tot.D, D2_sum=tot.D2, consts=consts_dict(c),
               threads=nthreads)
    if per_particle:
        out.update(first_tri=first, nhits=nh, D=Dp, E=Ep)
    out.update(vec)
    out["bvh_nodes"] = tree.nodes if tree is not None else 0
    return out
