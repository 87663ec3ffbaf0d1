"""Build libtpmc.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1312_3691_amd.build        # or build() from Python

Every HIP source is compiled with packed-FP32 instruction selection disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).  The build also links
libtpmc_probe.so, the same library with the batched kernel's phase probe
compiled in (TPMC_PHASE_PROBE=1, read through tpmc_phase_probe); the binding
loads it instead of libtpmc.so only when TPMC_PHASE_PROBE=1 is set.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtpmc.so")
PROBE_LIB = os.path.join(HERE, "libtpmc_probe.so")
PROBE_SOURCES = ["tpmc_capi.hip", "tpmc_kernels.hip"]  # the sources the probe switch changes
SOURCES = ["tpmc_capi.hip", "tpmc_kernels.hip", "tpmc_bvh.hip", "tpmc_ceilings.hip"]
HEADERS = ["tpmc_device.hpp", "tpmc_math.hpp", "tpmc_internal.h", "tpmc_launch.h"]
ARCH = os.environ.get("TPMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libtpmc.so)")


BUILD_DIR = os.path.join(HERE, "..", "_build")


def torch_lib_dir() -> str:
    """PyTorch's lib directory (found without importing torch).  The library is
    linked against PyTorch's HIP runtime so that one process holds exactly one
    HIP runtime: device pointers and streams from PyTorch are then valid here."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("PyTorch (ROCm build) is required")
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}: a ROCm build of PyTorch is required")
    return d


def compile_command(src: str, obj: str, defines=()) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-mcode-object-version=5", "-O3", "-std=c++17", "-fPIC", "-c",
            *["-D" + d for d in defines],
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # Machine LICM hoists the FP64 polynomial constants of exp/erfc out of the
            # Newton and particle loops into ~300 registers (occupancy 1); without it
            # the seeding fits in ~92 VGPRs.
            "-mllvm", "-disable-machine-licm",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
            "-I", os.path.join(HERE, "..", "include"), "-o", obj, src]


def link_command(objs: list, out: str) -> list:
    tl = torch_lib_dir()
    # the system linker driver, so that no ROCm library path is added implicitly
    return ["g++", "-shared", "-fPIC", "-o", out] + objs + [
        "-L" + tl, "-l:libamdhip64.so", "-Wl,--disable-new-dtags,-rpath," + tl, "-lstdc++", "-lm"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]))
    noise = [ln for ln in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if verbose and noise:
        print("\n".join(noise))


def _link(objs, lib, verbose):
    tmp = lib + ".tmp%d" % os.getpid()
    _run(link_command(objs, tmp), verbose)
    os.replace(tmp, lib)


def build(verbose: bool = False, probe: bool = True) -> str:
    """Compile every HIP source and link paper_1312_3691_amd/libtpmc.so, then
    (probe) libtpmc_probe.so; always rebuilds.  Returns the path of libtpmc.so."""
    probe_dir = os.path.join(BUILD_DIR, "probe")
    os.makedirs(probe_dir, exist_ok=True)
    objs = {s: os.path.join(BUILD_DIR, s.replace(".hip", ".o")) for s in SOURCES}
    jobs = [compile_command(os.path.join(CSRC, s), objs[s]) for s in SOURCES]
    probe_objs = dict(objs)
    if probe:
        for s in PROBE_SOURCES:
            probe_objs[s] = os.path.join(probe_dir, s.replace(".hip", ".o"))
            jobs.append(compile_command(os.path.join(CSRC, s), probe_objs[s], defines=("TPMC_PHASE_PROBE=1",)))
    # the compiles are independent: run them side by side
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        for f in [ex.submit(_run, cmd, verbose) for cmd in jobs]:
            f.result()
    _link([objs[s] for s in SOURCES], LIB, verbose)
    if probe:
        _link([probe_objs[s] for s in SOURCES], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
