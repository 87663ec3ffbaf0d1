"""Python binding of libtpmc.so (C ABI in include/tpmc.h).

Argument marshalling only: every step of the drag computation runs in the
library's HIP kernels.  PyTorch supplies device memory (the workspaces) and the
HIP stream.  Importing this module fails loudly when libtpmc.so is missing;
there is no CPU fallback.  With TPMC_PHASE_PROBE=1 in the environment it loads
libtpmc_probe.so instead, the same library with the batched kernel's phase
probe compiled in (Context.phase_probe).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  -- loads PyTorch's HIP runtime, which libtpmc.so is linked against

_HERE = os.path.dirname(os.path.abspath(__file__))
PHASE_PROBE = os.environ.get("TPMC_PHASE_PROBE", "0") == "1"
LIB_PATH = os.path.join(_HERE, "libtpmc_probe.so" if PHASE_PROBE else "libtpmc.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{os.path.basename(LIB_PATH)} not built ({LIB_PATH}); "
                      "run `python -m paper_1312_3691_amd.build` first")
_lib = ctypes.CDLL(LIB_PATH)

Q_NO_TRIANGLE_TALLY = 1

STATUS = {0: "TPMC_OK", 1: "TPMC_E_INVALID", 2: "TPMC_E_MESH", 3: "TPMC_E_CV", 4: "TPMC_E_WORKSPACE",
          5: "TPMC_E_DEVICE", 6: "TPMC_E_BUSY"}


class TpmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Query(ctypes.Structure):
    _fields_ = [("q_wxyz", ctypes.c_double * 4), ("S", ctypes.c_double), ("T_inf", ctypes.c_double),
                ("T_w", ctypes.c_double), ("alpha", ctypes.c_double), ("n_particles", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("max_reflections", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("cv_center", ctypes.c_double * 3), ("cv_radius", ctypes.c_double),
                ("energy_accommodation", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("F_over_q", ctypes.c_double * 3), ("M_over_q", ctypes.c_double * 3), ("Fhat", ctypes.c_double * 3),
                ("CD", ctypes.c_double), ("CD_sigma", ctypes.c_double), ("Gamma_hat", ctypes.c_double),
                ("rays", ctypes.c_uint64), ("hits", ctypes.c_uint64), ("segments", ctypes.c_uint64),
                ("missed", ctypes.c_uint64), ("escaped", ctypes.c_uint64), ("capped", ctypes.c_uint64),
                ("Qhat", ctypes.c_double), ("CH", ctypes.c_double), ("CH_sigma", ctypes.c_double),
                ("Mhat", ctypes.c_double * 3), ("tr_capped", ctypes.c_uint64), ("guard_trips", ctypes.c_uint64),
                ("preculled", ctypes.c_uint64)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_uint64), ("nt", ctypes.c_uint64), ("depth", ctypes.c_uint32),
                ("stack_slots", ctypes.c_uint32), ("box_lo", ctypes.c_double * 3), ("box_hi", ctypes.c_double * 3),
                ("sphere_center", ctypes.c_double * 3), ("sphere_radius", ctypes.c_double),
                ("device_bytes", ctypes.c_uint64), ("builder", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

# BVH builders (tpmc_bvh_builder); results do not depend on the choice
BUILDERS = {"sah": 0, "lbvh": 1}


_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_QP = ctypes.POINTER(Query)
_RP = ctypes.POINTER(Result)

class Tuning(ctypes.Structure):
    _fields_ = [("refill_lanes", _u32), ("tile_particles", _u32), ("groups_per_cu", _u32),
                ("plain_groups_per_cu", _u32)]


_SIGS = {
    "tpmc_last_error": ([], ctypes.c_char_p),
    "tpmc_abi_version": ([], ctypes.c_int),
    "tpmc_create": ([ctypes.c_int, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_get_tuning": ([_vp, ctypes.POINTER(Tuning)], ctypes.c_int),
    "tpmc_set_tuning": ([_vp, ctypes.POINTER(Tuning)], ctypes.c_int),
    "tpmc_set_stream": ([_vp, _vp], ctypes.c_int),
    "tpmc_destroy_ctx": ([_vp], None),
    "tpmc_build_mesh": ([_vp, _fp, _u64, ctypes.POINTER(_u32), _u64, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_build_mesh_ex": ([_vp, _fp, _u64, ctypes.POINTER(_u32), _u64, _u32, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_get_mesh_info": ([_vp, ctypes.POINTER(MeshInfo)], ctypes.c_int),
    "tpmc_destroy_mesh": ([_vp], None),
    "tpmc_workspace_bytes": ([_vp, _vp, _QP, _u32, ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_seed": ([_vp, _vp, _QP, _u32, _vp, _u64, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_particles_planes": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_trace": ([_vp, _vp, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_trace_ex": ([_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_forces": ([_vp, _vp, _dp, ctypes.c_double, _RP], ctypes.c_int),
    "tpmc_tally_copy": ([_vp, _vp, _u32, _dp], ctypes.c_int),
    "tpmc_destroy_particles": ([_vp], None),
    "tpmc_destroy_tally": ([_vp], None),
    "tpmc_batch_workspace_bytes": ([_vp, _vp, _QP, _u32, ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_batch_create": ([_vp, _vp, _QP, _u32, _vp, _u64, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_batch_launch": ([_vp, _vp, ctypes.c_int], ctypes.c_int),
    "tpmc_batch_results": ([_vp, _vp, _dp, ctypes.c_double, _RP], ctypes.c_int),
    "tpmc_destroy_batch": ([_vp], None),
    "tpmc_batch_run_noalloc": ([_vp, _vp, _QP, _u32, _dp, ctypes.c_double, _RP], ctypes.c_int),
    "tpmc_server_workspace_bytes": ([_u32, _u64, ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_server_create": ([_vp, _u32, _u64, _vp, _u64, ctypes.POINTER(_vp)], ctypes.c_int),
    "tpmc_server_admit": ([_vp, _u32, _vp, _QP, _u64, ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_server_admit_many": ([_vp, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_vp), _QP, ctypes.POINTER(_u64),
                                ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_server_collect": ([_vp, ctypes.POINTER(_u32), _u32, _dp, ctypes.c_double, ctypes.POINTER(_u32)],
                            ctypes.c_int),
    "tpmc_server_collected": ([_vp, _u32, _RP, _u32], ctypes.c_int),
    "tpmc_server_step": ([_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u64), ctypes.POINTER(_u64), _u32], ctypes.c_int),
    "tpmc_server_results": ([_vp, ctypes.POINTER(_u32), _u32, _dp, ctypes.c_double, _RP], ctypes.c_int),
    "tpmc_server_release": ([_vp, _u32], ctypes.c_int),
    "tpmc_destroy_server": ([_vp], None),
    "tpmc_check_mesh": ([_fp, _u64, ctypes.POINTER(_u32), _u64], ctypes.c_int),
    "tpmc_check_query": ([_QP, _fp, _u64], ctypes.c_int),
    "tpmc_ceiling_valu": ([_vp, _u32, _vp, _dp], ctypes.c_int),
    "tpmc_ceiling_read": ([_vp, _vp, _u64, _u32, _dp], ctypes.c_int),
    "tpmc_ceiling_atomic": ([_vp, _vp, _u32, _u32, _dp], ctypes.c_int),
    "tpmc_ceiling_lds_atomic": ([_vp, _vp, _u32, _u32, _dp], ctypes.c_int),
    "tpmc_precull_check": ([_vp, _vp, _QP, _vp, _u64, _dp, ctypes.POINTER(_u64)], ctypes.c_int),
    "tpmc_phase_probe": ([_vp, ctypes.POINTER(_u64), _u32, ctypes.c_int], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

ABI_VERSION = 9  # the structures below are laid out for this version of include/tpmc.h
if _lib.tpmc_abi_version() != ABI_VERSION:
    raise ImportError(f"libtpmc.so has ABI version {_lib.tpmc_abi_version()}, this binding expects "
                      f"{ABI_VERSION}: rebuild the library (python -c 'import __graft_entry__ as g; g.build()')")


# slots of tpmc_phase_probe, in order (include/tpmc.h)
PROBE_SLOTS = ("waves", "cycles", "claim_cycles", "claims",
               "trav_cycles", "trav_steps", "trav_lanes",
               "leaf_cycles", "leaf_passes", "leaf_lanes",
               "serve_cycles", "serves", "serve_lanes",
               "est_cycles", "est_batches", "est_particles", "est_kept",
               "seed_cycles", "seed_batches", "seed_particles", "seed_kept",
               "assign_cycles", "assigns", "assign_lanes")


def _check(status: int):
    if status != 0:
        raise TpmcError(status, _lib.tpmc_last_error().decode())


def make_query(qd: dict) -> Query:
    q = Query()
    q.q_wxyz[:] = [float(v) for v in qd["q"]]
    q.S, q.T_inf, q.T_w, q.alpha = float(qd["S"]), float(qd["T_inf"]), float(qd["T_w"]), float(qd["alpha"])
    q.n_particles, q.seed = int(qd["n"]), int(qd["seed"])
    q.max_reflections = int(qd.get("max_reflections", 16))
    q.flags = int(qd.get("flags", 0))
    q.cv_center[:] = [float(v) for v in qd.get("cv_center", (0.0, 0.0, 0.0))]
    q.cv_radius = float(qd.get("cv_radius", 0.0))
    q.energy_accommodation = float(qd.get("alpha_E", 1.0))
    return q


def _queries(qds) -> ctypes.Array:
    arr = (Query * len(qds))()
    for i, qd in enumerate(qds):
        arr[i] = make_query(qd)
    return arr


WORK_COUNTS = ("preculled",)  # result fields that count work done, which differs between paths


def same_on_every_path(result: dict) -> list:
    """The fields of a result dict that every path (plain, batched, served,
    any tuning) reproduces bit for bit: all but the work counts."""
    return [k for k in result if k not in WORK_COUNTS]


def result_dict(r: Result) -> dict:
    out = {}
    for f, _ in Result._fields_:
        v = getattr(r, f)
        out[f] = np.array(v[:]) if isinstance(v, ctypes.Array) else v
    return out


def _mesh_arrays(V, T):
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float32).reshape(-1, 3))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.uint32).reshape(-1, 3))
    return V, T


def check_mesh(V, T) -> None:
    """Host-only validation (no device needed)."""
    V, T = _mesh_arrays(V, T)
    _check(_lib.tpmc_check_mesh(V.ctypes.data_as(_fp), V.shape[0], T.ctypes.data_as(ctypes.POINTER(_u32)),
                                T.shape[0]))


def check_query(qd: dict, V=None) -> None:
    """Host-only validation of one query (the control-volume test needs V)."""
    q = make_query(qd)
    if V is None:
        _check(_lib.tpmc_check_query(ctypes.byref(q), None, 0))
    else:
        Vc = np.ascontiguousarray(np.asarray(V, dtype=np.float32).reshape(-1, 3))
        _check(_lib.tpmc_check_query(ctypes.byref(q), Vc.ctypes.data_as(_fp), Vc.shape[0]))


def _torch():
    import torch
    return torch


def _workspace(nbytes: int, device: int):
    """Device workspace from PyTorch's allocator, 256-byte aligned."""
    torch = _torch()
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=f"cuda:{device}")
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off, int(nbytes)


class Context:
    """A libtpmc context on one GPU, issuing work on PyTorch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise TpmcError(5, "no GPU visible: libtpmc runs on MI355X (gfx950) only")
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _vp()
        _check(_lib.tpmc_create(self.device, _vp(stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.tpmc_destroy_ctx(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_mesh(self, V, T, builder: str = "sah") -> "Mesh":
        return Mesh(self, V, T, builder)

    @property
    def tuning(self) -> dict:
        t = Tuning()
        _check(_lib.tpmc_get_tuning(self._h, ctypes.byref(t)))
        return {"refill_lanes": t.refill_lanes, "tile_particles": t.tile_particles,
                "groups_per_cu": t.groups_per_cu, "plain_groups_per_cu": t.plain_groups_per_cu}

    def set_tuning(self, **kw) -> None:
        """Replace some fields of the launch tuning (tpmc_set_tuning); results do not change."""
        cur = self.tuning
        unknown = set(kw) - set(cur)
        if unknown:
            raise ValueError(f"unknown tuning fields {sorted(unknown)}")
        cur.update(kw)
        t = Tuning(int(cur["refill_lanes"]), int(cur["tile_particles"]), int(cur["groups_per_cu"]),
                   int(cur["plain_groups_per_cu"]))
        _check(_lib.tpmc_set_tuning(self._h, ctypes.byref(t)))

    # measured ceilings (tpmc_ceiling_*); buffers are device tensors of the caller
    CEILING_VALU_KINDS = {"fp32_fma": 0, "fp64_fma": 1, "int32_mul_add": 2}

    def ceiling_valu(self, kind: str, sink) -> float:
        out = ctypes.c_double()
        _check(_lib.tpmc_ceiling_valu(self._h, self.CEILING_VALU_KINDS[kind], _vp(sink.data_ptr()), ctypes.byref(out)))
        return out.value

    def ceiling_read(self, buf, passes: int) -> float:
        out = ctypes.c_double()
        nbytes = buf.numel() * buf.element_size()
        _check(_lib.tpmc_ceiling_read(self._h, _vp(buf.data_ptr()), nbytes, passes, ctypes.byref(out)))
        return out.value

    def ceiling_atomic(self, buf, slots: int, per_thread: int) -> float:
        if buf.numel() * buf.element_size() < 8 * slots:
            raise ValueError("buffer smaller than slots int64 words")
        out = ctypes.c_double()
        _check(_lib.tpmc_ceiling_atomic(self._h, _vp(buf.data_ptr()), slots, per_thread, ctypes.byref(out)))
        return out.value

    def ceiling_lds_atomic(self, sink, slots: int, per_thread: int) -> float:
        out = ctypes.c_double()
        _check(_lib.tpmc_ceiling_lds_atomic(self._h, _vp(sink.data_ptr()), slots, per_thread, ctypes.byref(out)))
        return out.value

    def phase_probe(self, reset: bool = True) -> dict:
        """Sums of the batched kernel's phase probe since the last reset (after
        the stream's work), by slot name; raises TpmcError from a library built
        without the probe (tpmc_phase_probe)."""
        out = (_u64 * len(PROBE_SLOTS))()
        _check(_lib.tpmc_phase_probe(self._h, out, len(PROBE_SLOTS), 1 if reset else 0))
        return {k: int(v) for k, v in zip(PROBE_SLOTS, out)}


class Mesh:
    """Triangle mesh with its device-resident BVH (builder "sah" or "lbvh")."""

    def __init__(self, ctx: Context, V, T, builder: str = "sah"):
        V, T = _mesh_arrays(V, T)
        if builder not in BUILDERS:
            raise TpmcError(1, f"unknown BVH builder {builder!r} (one of {sorted(BUILDERS)})")
        self.ctx = ctx
        self.V, self.T = V, T
        h = _vp()
        _check(_lib.tpmc_build_mesh_ex(ctx._h, V.ctypes.data_as(_fp), V.shape[0],
                                       T.ctypes.data_as(ctypes.POINTER(_u32)), T.shape[0], BUILDERS[builder],
                                       ctypes.byref(h)))
        self._h = h
        info = MeshInfo()
        _check(_lib.tpmc_get_mesh_info(h, ctypes.byref(info)))
        self.info = {f: (list(getattr(info, f)) if isinstance(getattr(info, f), ctypes.Array) else getattr(info, f))
                     for f, _ in MeshInfo._fields_}
        self.nt = int(info.nt)

    def precull_check(self, query: dict):
        """Largest error of the batched path's seeding estimate over the query's
        particles, as a fraction of its margin, and the number of particles it
        covered (tpmc_precull_check)."""
        PRECULL_CHECK_BYTES = 1024
        buf, ptr, nb = _workspace(PRECULL_CHECK_BYTES, self.ctx.device)
        q = make_query(query)
        worst, n = ctypes.c_double(), _u64()
        _check(_lib.tpmc_precull_check(self.ctx._h, self._h, ctypes.byref(q), _vp(ptr), nb, ctypes.byref(worst),
                                       ctypes.byref(n)))
        del buf
        return worst.value, int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.tpmc_destroy_mesh(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PlainRun:
    """seed -> trace -> forces for a list of queries (one kernel launch per
    query and stage).  Keeps the workspace alive while its handles live."""

    def __init__(self, mesh: Mesh, queries, first_tri: bool = False):
        torch = _torch()
        self.mesh, self.ctx = mesh, mesh.ctx
        self.qds = list(queries)
        self._qarr = _queries(self.qds)
        nbytes = _u64()
        _check(_lib.tpmc_workspace_bytes(self.ctx._h, mesh._h, self._qarr, len(self.qds), ctypes.byref(nbytes)))
        self.ws_tensor, self.ws_ptr, self.ws_bytes = _workspace(nbytes.value, self.ctx.device)
        self.n_total = sum(int(q["n"]) for q in self.qds)
        self.first_tri = (torch.full((self.n_total,), -3, dtype=torch.int32, device=f"cuda:{self.ctx.device}")
                          if first_tri else None)
        self._p = None
        self._t = None

    def seed(self):
        p = _vp()
        _check(_lib.tpmc_seed(self.ctx._h, self.mesh._h, self._qarr, len(self.qds), _vp(self.ws_ptr),
                              self.ws_bytes, ctypes.byref(p)))
        self._p = p
        return self

    def planes(self):
        """Seeded states as six torch FP32 views (x0, x1, x2, w0, w1, w2)."""
        torch = _torch()
        arr = (_vp * 6)()
        n = _u64()
        _check(_lib.tpmc_particles_planes(self._p, arr, ctypes.byref(n)))
        base = self.ws_tensor.data_ptr()
        out = []
        for k in range(6):
            off = arr[k] - base
            out.append(self.ws_tensor[off: off + 4 * n.value].view(torch.float32))
        return out

    def trace(self, counters=None):
        """counters: optional torch int64 device tensor [2] (nodes visited, triangle tests)."""
        t = _vp()
        ft = _vp(self.first_tri.data_ptr()) if self.first_tri is not None else None
        ct = _vp(counters.data_ptr()) if counters is not None else None
        _check(_lib.tpmc_trace_ex(self.ctx._h, self.mesh._h, self._p, ft, ct, ctypes.byref(t)))
        self._t = t
        return self

    def forces(self, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0):
        res = (Result * len(self.qds))()
        xr = (ctypes.c_double * 3)(*[float(v) for v in x_ref])
        _check(_lib.tpmc_forces(self.ctx._h, self._t, xr, float(A_ref), res))
        return [result_dict(r) for r in res]

    def tally(self, query: int = 0) -> np.ndarray:
        out = np.zeros((self.mesh.nt, 7))
        _check(_lib.tpmc_tally_copy(self.ctx._h, self._t, int(query), out.ctypes.data_as(_dp)))
        return out

    def close(self):
        if self._t:
            _lib.tpmc_destroy_tally(self._t)
            self._t = None
        if self._p:
            _lib.tpmc_destroy_particles(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(mesh: Mesh, queries, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0, first_tri: bool = False):
    """Plain path: seed, trace and reduce; returns (results, PlainRun)."""
    pr = PlainRun(mesh, queries, first_tri=first_tri).seed().trace()
    return pr.forces(x_ref, A_ref), pr


class Batch:
    """Batched path: all queries in one persistent launch (optionally replayed
    from a captured HIP graph)."""

    def __init__(self, mesh: Mesh, queries):
        self.mesh, self.ctx = mesh, mesh.ctx
        self.qds = list(queries)
        self._qarr = _queries(self.qds)
        nbytes = _u64()
        _check(_lib.tpmc_batch_workspace_bytes(self.ctx._h, mesh._h, self._qarr, len(self.qds), ctypes.byref(nbytes)))
        self.ws_tensor, self.ws_ptr, self.ws_bytes = _workspace(nbytes.value, self.ctx.device)
        h = _vp()
        _check(_lib.tpmc_batch_create(self.ctx._h, mesh._h, self._qarr, len(self.qds), _vp(self.ws_ptr),
                                      self.ws_bytes, ctypes.byref(h)))
        self._h = h

    def launch(self, use_graph: bool = False):
        _check(_lib.tpmc_batch_launch(self.ctx._h, self._h, 1 if use_graph else 0))
        return self

    def results(self, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0):
        res = (Result * len(self.qds))()
        xr = (ctypes.c_double * 3)(*[float(v) for v in x_ref])
        _check(_lib.tpmc_batch_results(self.ctx._h, self._h, xr, float(A_ref), res))
        return [result_dict(r) for r in res]

    def close(self):
        if getattr(self, "_h", None):
            _lib.tpmc_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_MAX_BYTES = 32 << 20  # TPMC_NOALLOC_MAX_BYTES


def batch_run_noalloc(mesh: Mesh, queries, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0):
    """Batched path with the library's static device workspace (no device
    allocation); see tpmc_batch_run_noalloc in include/tpmc.h."""
    qarr = _queries(list(queries))
    res = (Result * len(qarr))()
    xr = (ctypes.c_double * 3)(*[float(v) for v in x_ref])
    _check(_lib.tpmc_batch_run_noalloc(mesh.ctx._h, mesh._h, qarr, len(qarr), xr, float(A_ref), res))
    return [result_dict(r) for r in res]


class Server:
    """libtpmc serving slots (continuous batching); see paper_1312_3691_amd.serve."""

    def __init__(self, ctx: Context, max_slots: int, pool_words: int):
        self.ctx = ctx
        self.max_slots = int(max_slots)
        nbytes = _u64()
        _check(_lib.tpmc_server_workspace_bytes(self.max_slots, int(pool_words), ctypes.byref(nbytes)))
        self.ws_tensor, self.ws_ptr, self.ws_bytes = _workspace(nbytes.value, ctx.device)
        h = _vp()
        _check(_lib.tpmc_server_create(ctx._h, self.max_slots, int(pool_words), _vp(self.ws_ptr), self.ws_bytes,
                                       ctypes.byref(h)))
        self._h = h
        self._q = {}

    def admit(self, slot: int, mesh: Mesh, qd: dict, tally_offset: int = 0) -> int:
        q = make_query(qd)
        self._q[slot] = (q, mesh)
        nt = _u64()
        _check(_lib.tpmc_server_admit(self._h, int(slot), mesh._h, ctypes.byref(q), int(tally_offset),
                                      ctypes.byref(nt)))
        return int(nt.value)

    def admit_many(self, items) -> list:
        """items: (slot, mesh, query dict, tally offset) each; returns the tile counts."""
        n = len(items)
        if n == 0:
            return []
        sl = (_u32 * n)(*[int(i[0]) for i in items])
        ms = (_vp * n)(*[i[1]._h for i in items])
        qs = _queries([i[2] for i in items])
        off = (_u64 * n)(*[int(i[3]) for i in items])
        nt = (_u64 * n)()
        _check(_lib.tpmc_server_admit_many(self._h, n, sl, ms, qs, off, nt))
        for i in items:
            self._q[i[0]] = (i[2], i[1])
        return [int(v) for v in nt]

    def collect(self, slots, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0) -> tuple:
        """Enqueue the results of these slots; returns a ticket for collected()."""
        n = len(slots)
        sl = (_u32 * n)(*[int(s) for s in slots])
        xr = (ctypes.c_double * 3)(*[float(v) for v in x_ref])
        t = _u32()
        _check(_lib.tpmc_server_collect(self._h, sl, n, xr, float(A_ref), ctypes.byref(t)))
        return (int(t.value), n)

    def collected(self, ticket) -> list:
        t, n = ticket
        res = (Result * n)()
        _check(_lib.tpmc_server_collected(self._h, t, res, n))
        return [result_dict(r) for r in res]

    def step(self, entries):
        n = len(entries)
        if n == 0:
            return
        sl = (_u32 * n)(*[int(e[0]) for e in entries])
        t0 = (_u64 * n)(*[int(e[1]) for e in entries])
        ct = (_u64 * n)(*[int(e[2]) for e in entries])
        _check(_lib.tpmc_server_step(self._h, sl, t0, ct, n))

    def results(self, slots, x_ref=(0.0, 0.0, 0.0), A_ref: float = 1.0):
        n = len(slots)
        sl = (_u32 * n)(*[int(s) for s in slots])
        res = (Result * n)()
        xr = (ctypes.c_double * 3)(*[float(v) for v in x_ref])
        _check(_lib.tpmc_server_results(self._h, sl, n, xr, float(A_ref), res))
        return [result_dict(r) for r in res]

    def release(self, slot: int):
        _check(_lib.tpmc_server_release(self._h, int(slot)))
        self._q.pop(slot, None)

    def close(self):
        if getattr(self, "_h", None):
            _lib.tpmc_destroy_server(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
