"""Register budget of the persistent batched kernel (host-only: compiles the
kernels to gfx950 assembly and reads the code-object metadata).

The batched kernel is bound by VALU issue with four 64-lane waves per
workgroup; at 128 VGPRs or fewer a SIMD holds four waves (512 per lane), one
more than at 129-170, which hides the latency of the traversal loads and
measured 13-15 % faster on the plate and cylinder launches.  Every instance
of the batched path must therefore fit in 128 VGPRs without spilling."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_3691_amd", "csrc")


def _metadata():
    from paper_1312_3691_amd import build as B
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [B.hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-S",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-disable-machine-licm",
               "-I", os.path.join(ROOT, "include"), "-o", out, os.path.join(CSRC, "tpmc_kernels.hip")]
        subprocess.run(cmd, check=True, capture_output=True)
        text = open(out).read()
    meta = {}
    for m in re.finditer(r"\.name:\s+(\S+)\n(.*?)(?=\n  - \.|\Z)", text, re.S):
        body = m.group(2)
        get = lambda k: int((re.search(r"\." + k + r":\s+(\d+)", body) or [0, 0])[1])
        meta[m.group(1)] = {"vgpr": get("vgpr_count"), "spill": get("vgpr_spill_count"),
                            "lds": get("group_segment_fixed_size")}
    return meta


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_batch_kernel_fits_four_waves_per_simd():
    meta = _metadata()
    # batch_kernel<STACK, MODE>: global atomics, workgroup LDS, per-lane LDS and totals-only
    # tallies at every stack depth (the mixed mode of serving steps is not held to it)
    inst = {k: v for k, v in meta.items() if re.search(r"batch_kernelILi\d+ELi[0-3]E", k)}
    assert len(inst) == 20, sorted(inst)
    for k, v in inst.items():
        assert v["vgpr"] <= 128 and v["spill"] == 0, (k, v)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_batch_kernel_lds_fits_four_workgroups_per_cu():
    """Four workgroups of four waves fill a CU's 160 KB of LDS at 40 KB each: the
    static LDS (stack, seeding queue, survivor rings) plus the tallies sized at
    launch must fit that for the benchmark's instances -- the plate (2 triangles,
    per-lane tallies), the cylinder (256 triangles, workgroup tallies), the
    satellite (global atomics) and the attitude sweep (per-wave totals)."""
    meta = _metadata()
    lds = {}
    for k, v in meta.items():
        m = re.search(r"batch_kernelILi(\d+)ELi(\d+)E", k)
        if m:
            lds[(int(m.group(1)), int(m.group(2)))] = v["lds"]
    dynamic = {(4, 2): 2 * 7 * 256 * 8, (16, 1): 256 * 7 * 8, (32, 0): 0, (32, 3): 7 * 4 * 8}
    for key, dyn in dynamic.items():
        assert lds[key] + dyn <= 160 * 1024 // 4, (key, lds[key], dyn)
