"""Compile the HIP library (gfx950) into paper_1712_09430_amd/libcatpc.so.

hipcc flags: -ffp-contract=off and no fast-math keep every float operation a
separately rounded IEEE operation (the filter's operation order is part of its
definition); packed FP32 instructions are disabled.  The machine scheduler
orders instructions for instruction-level parallelism (`max-ilp`): the grid
build, the neighbour search and the tracklet kernel are latency-bound chains,
and this order is about 1 % faster per step than the occupancy-driven default
(results are the same: scheduling does not reorder float operations' rounding).
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcatpc.so")
SOURCES = ["kernels.hip", "api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-sched-strategy=max-ilp",
         "-Wall", "-Wno-unused-result"]


# Profiling build: the same sources with the tracklet kernel's phase clocks
# compiled in (catpc_phase_clocks); used by phase_clocks.py, never by the
# product path.
PHASE_LIB = os.path.join(HERE, "libcatpc_phase.so")


def build(force: bool = True, lib: str = LIB, defines=()) -> str:
    if not force and os.path.exists(lib):
        return lib
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in SOURCES:
            o = os.path.join(tmp, src + ".o")
            subprocess.run([HIPCC, *FLAGS, *defines, "-c", os.path.join(HERE, "csrc", src), "-o", o], check=True)
            objs.append(o)
        out = lib + ".tmp"
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out], check=True)
        os.replace(out, lib)
    return lib


def build_phase_clocks(force: bool = True) -> str:
    return build(force, PHASE_LIB, ("-DCATPC_PHASE_CLOCKS=1",))


if __name__ == "__main__":
    print(build())
    print(build_phase_clocks())
