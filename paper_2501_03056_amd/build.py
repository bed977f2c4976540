"""Build libfppg.so (the HIP/C++ relaxation library) in-tree for gfx950.

    python -m paper_2501_03056_amd.build        # or build() from Python

The library is one shared object compiled by hipcc from csrc/*.hip. Flags:
  --offload-arch=gfx950                 CDNA4 only
  -ffp-contract=off                     the binary32 neighbour predicate and the
                                        cell keys must round every operation
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                        no packed FP32 instructions
"""
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfppg.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm not installed?)")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every source into LIB (always recompiles). Returns the library path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-I", INCLUDE, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
