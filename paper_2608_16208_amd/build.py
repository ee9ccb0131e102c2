"""Build the HIP library libffbie.so for gfx950 in-tree with hipcc: every
source is compiled to an object in parallel, then the objects are linked."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/ffbie_api.hip", "csrc/ffbie_kernels.hip", "csrc/ffbie_assembly.hip",
           "csrc/ffbie_solve.hip", "csrc/ffbie_gemm.hip", "csrc/ffbie_mlp.hip", "csrc/ffbie_blockjacobi.hip",
           "csrc/ffbie_banded.hip"]
LIB = os.path.join(HERE, "libffbie.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]
# Per-source additions.  The coefficient kernels are built without machine-level
# loop-invariant hoisting: their pair loops then recompute cheap invariants
# instead of holding them in registers, which frees the VGPRs for a fourth
# wavefront per SIMD (and removes the SGPR spills the hoisted sincos
# coefficients caused).
EXTRA = {"csrc/ffbie_kernels.hip": ["-mllvm", "-disable-machine-licm"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
    return res.returncode, "\n".join(errs)


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
    with tempfile.TemporaryDirectory(prefix="ffbie_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[hipcc] + FLAGS + EXTRA.get(s, []) + ["-c", os.path.join(HERE, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        for (rc, err), s in zip(results, SOURCES):
            if rc != 0:
                sys.stderr.write(err + "\n")
                raise RuntimeError("hipcc failed compiling " + s)
        tmp = LIB + ".tmp"
        rc, err = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                       verbose)
        if rc != 0:
            sys.stderr.write(err + "\n")
            raise RuntimeError("hipcc failed linking libffbie.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
