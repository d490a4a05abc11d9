"""Build the relpic HIP library (librelpic.so) in-tree for gfx950.

Each source is compiled to an object in parallel (hipcc, non-relocatable
device code: every translation unit carries its own kernels), then the
objects are linked into the shared library.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librelpic.so")
SOURCES = ["capi.hip", "batch.hip", "adjoint.hip", "kernels_adjoint.hip", "kernels_field.hip", "kernels_leap.hip", "kernels_particle.hip", "kernels_batch.hip", "kernels_aux.hip",
           "sort.hip", "kspace.hip", "init_fields.hip", "solver_setup.cpp"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # no packed FP32 math: keep every float op scalar
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="relpic_build_") as tmpdir:
        def compile_one(src):
            obj = os.path.join(tmpdir, src + ".o")
            cmd = [hipcc] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            # hipcc's host pass warns that it does not know the packed-FP32 feature: harmless
            err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln)
            if err.strip():
                print(err, file=sys.stderr, flush=True)
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, cmd)
            return obj

        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
