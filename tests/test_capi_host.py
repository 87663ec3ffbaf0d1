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
    assert lib.tpmc_abi_version() == T.ABI_VERSION == 9


def test_probe_library_exports_the_same_abi(T):
    """libtpmc_probe.so (the batched kernel with its phase probe) is the same
    C ABI; only it answers tpmc_phase_probe, the ordinary library refuses."""
    probe = ctypes.CDLL(os.path.join(os.path.dirname(T.LIB_PATH), "libtpmc_probe.so"))
    plain = ctypes.CDLL(os.path.join(os.path.dirname(T.LIB_PATH), "libtpmc.so"))
    for n in _declared_functions():
        assert hasattr(probe, n), n
    assert probe.tpmc_abi_version() == T.ABI_VERSION
    out = (ctypes.c_uint64 * 24)()
    plain.tpmc_last_error.restype = ctypes.c_char_p
    assert plain.tpmc_phase_probe(None, out, 24, 0) == 1  # TPMC_E_INVALID: built without the probe
    assert b"without the phase probe" in plain.tpmc_last_error()
    assert probe.tpmc_phase_probe(None, out, 24, 0) == 1  # a probe library: NULL context
    probe.tpmc_last_error.restype = ctypes.c_char_p
    assert b"must not be NULL" in probe.tpmc_last_error()


def test_probe_slot_names_match_header(T):
    text = open(os.path.join(ROOT, "include", "tpmc.h")).read()
    n = int(re.search(r"#define TPMC_PROBE_SLOTS (\d+)", text).group(1))
    assert len(T.PROBE_SLOTS) == n == len(set(T.PROBE_SLOTS))


def _c_layout(struct: str, fields) -> list:
    """sizeof and offsetof of a tpmc.h struct, as the C compiler lays it out."""
    import subprocess
    import tempfile
    lines = [f'printf("%zu\\n", sizeof({struct}));'] + [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src = "#include <stddef.h>\n#include <stdio.h>\n#include \"tpmc.h\"\nint main(void) {\n" + "\n".join(lines) + "\nreturn 0; }\n"
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(c, "w") as f:
            f.write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        return [int(v) for v in subprocess.check_output([exe]).split()]


@pytest.mark.parametrize("name", ["Query", "Result", "MeshInfo", "Tuning"])
def test_struct_layouts_match_header(T, name):
    cls = getattr(T, name)
    cname = {"Query": "tpmc_query", "Result": "tpmc_result", "MeshInfo": "tpmc_mesh_info", "Tuning": "tpmc_tuning"}[name]
    fields = [f for f, _ in cls._fields_]
    want = _c_layout(cname, fields)
    got = [ctypes.sizeof(cls)] + [getattr(cls, f).offset for f in fields]
    assert got == want, dict(zip(["sizeof"] + fields, zip(got, want)))


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


def test_noalloc_limit_matches_header(T):
    text = open(os.path.join(ROOT, "include", "tpmc.h")).read()
    m = re.search(r"#define TPMC_NOALLOC_MAX_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == T.NOALLOC_MAX_BYTES
