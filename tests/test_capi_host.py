"""C-ABI contract tests that need no GPU: the library loads, exports every
function include/tpmc.h declares, and its host-side validation maps each bad
input to its status code.  No compute call is made here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1312_3691_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "tpmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(tpmc_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def T():
    from paper_1312_3691_amd import tpmc
    return tpmc


def test_every_declared_symbol_is_exported(T):
    names = _declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(T.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.tpmc_abi_version() == 5


def test_struct_sizes_match_header(T):
    # tpmc_query: 4+1+2+1 doubles, 2 u64, 2 u32, 4 doubles, 1 double = 120 bytes
    assert ctypes.sizeof(T.Query) == 8 * 8 + 16 + 8 + 32 + 8
    # tpmc_result: 12 doubles, 6 u64, 3 doubles
    assert ctypes.sizeof(T.Result) == 12 * 8 + 6 * 8 + 3 * 8
    # tpmc_mesh_info: 2 u64, 2 u32, 10 doubles, u64, 2 u32 = 120 bytes
    assert ctypes.sizeof(T.MeshInfo) == 16 + 8 + 80 + 8 + 8


def _status(fn):
    from paper_1312_3691_amd import tpmc
    try:
        fn()
    except tpmc.TpmcError as e:
        return e.status
    return 0


def test_mesh_validation(T):
    V, Tr = I.plate()
    assert _status(lambda: T.check_mesh(V, Tr)) == 0
    assert _status(lambda: T.check_mesh(V, Tr[:0])) == 2
    bad = Tr.copy()
    bad[1, 2] = 4
    assert _status(lambda: T.check_mesh(V, bad)) == 2
    Vn = V.copy()
    Vn[2, 1] = np.nan
    assert _status(lambda: T.check_mesh(Vn, Tr)) == 2
    Vi = V.copy()
    Vi[0, 0] = np.inf
    assert _status(lambda: T.check_mesh(Vi, Tr)) == 2
    # zero-area triangles are accepted
    Vz = np.vstack([V, V[:1]])
    Tz = np.vstack([Tr, [[0, 4, 0]]]).astype(np.uint32)
    assert _status(lambda: T.check_mesh(Vz, Tz)) == 0


@pytest.mark.parametrize("field,value", [("S", -1.0), ("S", float("nan")), ("S", 101.0), ("T_inf", 0.0),
                                         ("T_w", -3.0), ("alpha", 1.5), ("alpha", -0.1), ("n", 0),
                                         ("max_reflections", 0), ("max_reflections", 65), ("flags", 8)])
def test_query_validation(T, field, value):
    q = I.query()
    q[field] = value
    assert _status(lambda: T.check_query(q)) == 1


def test_query_attitude_and_cv(T):
    V, _ = I.icosphere(1)
    assert _status(lambda: T.check_query(I.query(q=(1.0, 0, 0, 0)), V)) == 0
    assert _status(lambda: T.check_query(I.query(q=(1.001, 0, 0, 0)), V)) == 1
    assert _status(lambda: T.check_query(I.query(q=(0.5, 0.5, 0.5, 0.5)), V)) == 0
    # user control volume must enclose every vertex
    assert _status(lambda: T.check_query(I.query(cv_radius=0.9), V)) == 3
    assert _status(lambda: T.check_query(I.query(cv_radius=1.01), V)) == 0
    assert _status(lambda: T.check_query(I.query(cv_radius=1.01, cv_center=(0.2, 0, 0)), V)) == 3
    assert _status(lambda: T.check_query(I.query(cv_radius=1.01, cv_center=(0, float("nan"), 0)), V)) == 1
    # box control volume: a cube of half-side cv_radius must contain every vertex
    # (the unit icosphere fits a cube of half-side 1, not one offset by 0.2)
    assert _status(lambda: T.check_query(I.query(cv_box=True), V)) == 0
    assert _status(lambda: T.check_query(I.query(cv_box=True, cv_radius=1.0), V)) == 0
    assert _status(lambda: T.check_query(I.query(cv_box=True, cv_radius=0.99), V)) == 3
    assert _status(lambda: T.check_query(I.query(cv_box=True, cv_radius=1.1, cv_center=(0.2, 0, 0)), V)) == 3
    assert _status(lambda: T.check_query(I.query(cv_box=True, cv_radius=0.9, cv_center=(0.0, 0, 0)), V)) == 3
    assert _status(lambda: T.check_query(I.query(flags=8), V)) == 1  # unknown bit above the known flags
    # energy accommodation in [0, 1] when its flag is set
    assert _status(lambda: T.check_query(I.query(alpha_E=0.0), V)) == 0
    assert _status(lambda: T.check_query(I.query(alpha_E=1.0), V)) == 0
    assert _status(lambda: T.check_query(I.query(alpha_E=1.2), V)) == 1
    assert _status(lambda: T.check_query(I.query(alpha_E=float("nan")), V)) == 1


def test_no_device_is_a_clean_error(T):
    """Without a visible GPU the context call fails with a status, never a crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = T._lib.tpmc_create(0, None, ctypes.byref(h))
    assert st in (1, 5) and not h.value
    assert len(T._lib.tpmc_last_error()) > 0
    with pytest.raises(T.TpmcError):
        T.Context(0)


def test_null_handles_are_rejected(T):
    lib = T._lib
    assert lib.tpmc_forces(None, None, None, 1.0, None) == 1
    assert lib.tpmc_trace(None, None, None, None) == 1
    n = ctypes.c_uint64()
    assert lib.tpmc_workspace_bytes(None, None, None, 0, ctypes.byref(n)) == 1
    lib.tpmc_destroy_ctx(None)
    lib.tpmc_destroy_mesh(None)
    lib.tpmc_destroy_particles(None)
    lib.tpmc_destroy_tally(None)
    lib.tpmc_destroy_batch(None)


def test_input_generators_sizes():
    assert I.icosphere(3)[1].shape == (1280, 3) and I.icosphere(3)[0].shape == (642, 3)
    assert I.capped_cylinder()[1].shape == (256, 3)
    V, Tr = I.satellite(50_000)
    assert 40_000 < len(Tr) < 60_000
    q = I.quat_for_flow((0.3, -0.2, 0.9))
    u = I.flow_dir(q)
    assert np.allclose(u, np.array([0.3, -0.2, 0.9]) / math.sqrt(0.94), atol=1e-12)
