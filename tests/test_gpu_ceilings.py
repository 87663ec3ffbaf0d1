"""The ceiling microkernels (tpmc_ceiling_*): plausible rates against the
published figures, exact counts from the atomic kernels, and argument checks."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1312_3691_amd import tpmc
    ctx = tpmc.Context(0)
    return torch, tpmc, ctx


def test_valu_ceilings_near_published(env):
    torch, tpmc, ctx = env
    sink = torch.zeros(64, dtype=torch.uint8, device="cuda")
    published = 256 * 64 * 2.4e9  # lane operations per second, one per lane per clock
    for kind in ("fp32_fma", "fp64_fma"):
        r = ctx.ceiling_valu(kind, sink)
        # FP32 may issue up to twice per lane per clock (the published FP32 figure is twice the FP64 one)
        assert 0.5 * published < r < 2.2 * published, (kind, r)
    assert ctx.ceiling_valu("int32_mul_add", sink) > 0.05 * published
    assert int(sink.sum()) == 0  # the sink is never written


def test_read_ceiling_and_arguments(env):
    torch, tpmc, ctx = env
    buf = torch.ones(1 << 20, dtype=torch.int32, device="cuda")  # 4 MiB
    r = ctx.ceiling_read(buf, 8)
    assert 1e11 < r < 1e15, r
    assert int(buf.sum()) == 1 << 20  # read only
    out = ctypes.c_double()
    p = ctypes.c_void_p(buf.data_ptr())
    assert tpmc._lib.tpmc_ceiling_read(ctx._h, p, 24, 1, ctypes.byref(out)) == 1  # not a multiple of 16
    assert tpmc._lib.tpmc_ceiling_read(ctx._h, p, 0, 1, ctypes.byref(out)) == 1
    assert tpmc._lib.tpmc_ceiling_read(ctx._h, p, 64, 0, ctypes.byref(out)) == 1
    assert tpmc._lib.tpmc_ceiling_valu(ctx._h, 3, p, ctypes.byref(out)) == 1


def test_atomic_ceilings_count_exactly(env):
    torch, tpmc, ctx = env
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    lanes = n_cu * 8 * 256
    for slots in (1, 16, 4096):
        buf = torch.zeros(4096, dtype=torch.int64, device="cuda")
        r = ctx.ceiling_atomic(buf, slots, 4)
        torch.cuda.synchronize()
        assert r > 0
        # one untimed and one timed launch, 4 adds of 1 per lane each
        assert int(buf.sum()) == 2 * 4 * lanes, slots
        assert int(buf[slots:].abs().sum()) == 0
    sink = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for slots in (1, 16, 512):
        assert ctx.ceiling_lds_atomic(sink, slots, 16) > 0
    assert int(sink.sum()) == 0
    out = ctypes.c_double()
    p = ctypes.c_void_p(sink.data_ptr())
    assert tpmc._lib.tpmc_ceiling_lds_atomic(ctx._h, p, 1025, 1, ctypes.byref(out)) == 1
    assert tpmc._lib.tpmc_ceiling_atomic(ctx._h, p, 0, 1, ctypes.byref(out)) == 1
    assert tpmc._lib.tpmc_ceiling_atomic(ctx._h, p, 1, 4097, ctypes.byref(out)) == 1
