"""Builds libsusp.so (the HIP force engine and its C ABI) for gfx950, in-tree.

Device code is compiled without packed FP32 instructions (the target feature
-packed-fp32-ops; the host pass of hipcc reports that it does not know the
feature, which is harmless).  The build keeps the device assembly of each source
and fails if any v_pk_*_f32 instruction appears in it.
"""
import glob
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsusp.so")
SOURCES = ["susp_kernels.hip", "susp_runtime.hip"]

# -ffp-contract=off: FP64 geometry, predicate and spring update are evaluated
# one correctly rounded operation at a time.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-save-temps=obj"]
PACKED_FP32 = re.compile(r"\bv_pk_(add|mul|fma|mov)_f32\b")


def check_no_packed_fp32(asm_files):
    """Raises if the device assembly holds a packed FP32 instruction."""
    for f in asm_files:
        for k, line in enumerate(open(f)):
            if PACKED_FP32.search(line) and not line.lstrip().startswith(";"):
                raise RuntimeError(f"{os.path.basename(f)}:{k + 1}: packed FP32 instruction in device code: "
                                   f"{line.strip()}")


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    shutil.rmtree(OUT, ignore_errors=True)
    os.makedirs(OUT)
    objs = []
    for src in SOURCES:
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=OUT)
        objs.append(obj)
    asm = glob.glob(os.path.join(OUT, "*-hip-amdgcn-amd-amdhsa-gfx950.s"))
    if len(asm) != len(SOURCES):
        raise RuntimeError(f"expected the device assembly of {len(SOURCES)} sources, found {len(asm)}")
    check_no_packed_fp32(asm)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=OUT)
    os.replace(tmp, LIB)
    if verbose:
        print(f"device assembly checked: no packed FP32 instructions in {', '.join(map(os.path.basename, asm))}",
              flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
