"""Builds librs_poly.so (HIP kernels for gfx950 + the C ABI) in-tree.

    python -m paper_1312_5155_amd.build        # or build() from Python

Each source compiles to its own object (in parallel), then one link makes
the library, which lands next to this file, where the binding loads it.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librs_poly.so")

SOURCES = ["codec.hip", "bitmatrix.hip", "gf.cpp", "api.cpp", "batch.cpp", "serve.cpp",
           "roof.hip", "noalloc.hip",
           "nibble.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Werror", "-Wno-unused-command-line-argument",
    # packed FP32 instructions stay off in every device pass
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]

# hipcc's host pass does not know the packed-fp32 feature and says so
_NOISE = "is not a recognized feature for this target"


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if _NOISE not in l)
    return res.returncode, err


def build(verbose: bool = False) -> str:
    srcs = sources()
    with tempfile.TemporaryDirectory(prefix="rs_poly_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[HIPCC] + FLAGS + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
        jobs = min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        failed = False
        for (rc, err), src in zip(results, srcs):
            if rc != 0:
                failed = True
                sys.stderr.write(f"--- {os.path.basename(src)}\n{err}\n")
            elif verbose and err.strip():
                sys.stderr.write(err + "\n")
        if failed:
            raise RuntimeError("hipcc failed building librs_poly.so")
        tmp = LIB + ".tmp"
        rc, err = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs +
                       ["-o", tmp], verbose)
        if rc != 0:
            sys.stderr.write(err + "\n")
            raise RuntimeError("hipcc failed linking librs_poly.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
