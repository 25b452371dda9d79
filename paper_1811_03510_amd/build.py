"""Builds the HIP library libccs.so for gfx950 in-tree (hipcc, no JIT).

Each source is compiled to an object with its own flags, then linked.  The
intersection kernel runs with the IEEE mode bit off, fp32 denormals flushed and
no signed zeros, so that (a + b) * 0.5 folds into one add with the /2 output
modifier; every fused multiply-add it relies on is written explicitly, so
contraction is off.  Its inputs are validated with integer bit tests, and no NaN
can arise from validated inputs.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libccs.so")
ARCH = "gfx950"

# Packed fp32 arithmetic stays off: the library's correctness must not depend on it.
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]
TRACE_FLAGS = ["-mno-amdgpu-ieee", "-fno-honor-nans", "-fgpu-flush-denormals-to-zero", "-fno-signed-zeros",
               "-ffp-contract=off"]
# policy.hip forms the learned order's inputs exactly as the intersection kernel does, and
# compact.hip decides which rays are traced exactly as the intersection kernel does
PER_FILE = {"trace.hip": TRACE_FLAGS, "policy.hip": TRACE_FLAGS, "compact.hip": TRACE_FLAGS,
            "refit.hip": ["-ffp-contract=off"]}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        cmd = [hipcc, *COMMON, *PER_FILE.get(os.path.basename(src), []), *extra, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, sources()))
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
