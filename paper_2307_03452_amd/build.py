"""Build liberi4.so (the gfx950 HIP library) in-tree with hipcc.

Each translation unit is compiled on its own, in parallel (the two plan
kernels and the fused kernels are the long ones), then linked."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liberi4.so")
STAGES_LIB = os.path.join(HERE, "liberi4_stages.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["eri4_plan64.hip", "eri4_plan32.hip", "eri4_plan64p.hip", "eri4_plan32p.hip", "eri4_fused.hip", "eri4_small.hip",
           "eri4_solid.hip", "eri4_coulomb.hip", "eri4_exchange.hip", "eri4.hip", "eri4_tables.cpp"]
HEADERS = ["eri4_device.h", "eri4_internal.h", "eri4_launch.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, stage_timers: bool = False) -> str:
    """Compile and link the library; stage_timers builds the variant with the
    per-stage cycle counters (liberi4_stages.so, -DERI4_STAGE_TIMERS)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = STAGES_LIB if stage_timers else LIB
    objdir = OBJDIR + ("_stages" if stage_timers else "")
    extra = ["-DERI4_STAGE_TIMERS"] if stage_timers else []
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I" + INC, "-I" + CSRC, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, stage_timers="--stage-timers" in sys.argv))
