"""Build libfppg.so (the HIP/C++ relaxation library) in-tree for gfx950.

    python -m paper_2501_03056_amd.build        # or build() from Python

The library is one shared object compiled by hipcc from csrc/*.hip, with the
hash of its sources and flags embedded (fppg_source_hash); the loader rebuilds
a library whose hash differs from the sources in the tree. Flags:
  --offload-arch=gfx950                 CDNA4 only
  -ffp-contract=off                     the binary32 neighbour predicate and the
                                        cell keys must round every operation
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                        no packed FP32 instructions
"""
import glob
import hashlib
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


FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
HASH_MARK = b"FPPG_SOURCE_HASH:"


def source_hash() -> str:
    """SHA-256 (first 32 hex digits) of every file the library is compiled
    from (csrc/*.hip, csrc/*.h, include/*.h, by relative path) and the flags."""
    h = hashlib.sha256()
    files = sources() + sorted(glob.glob(os.path.join(CSRC, "*.h"))) + \
        sorted(glob.glob(os.path.join(INCLUDE, "*.h")))
    for f in files:
        h.update(os.path.relpath(f, os.path.dirname(HERE)).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:32]


def built_hash(path: str = None):
    """The source hash embedded in a built library (None if absent or unreadable)."""
    path = path or LIB
    try:
        with open(path, "rb") as fh:
            data = fh.read()
    except OSError:
        return None
    i = data.find(HASH_MARK)
    if i < 0:
        return None
    return data[i + len(HASH_MARK): i + len(HASH_MARK) + 32].decode("ascii", "replace")


def build(verbose: bool = False) -> str:
    """Compile every source into LIB (always recompiles). Returns the library path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, f'-DFPPG_SOURCE_HASH="{source_hash()}"', "-I", INCLUDE, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
