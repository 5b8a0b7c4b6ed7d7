"""Compile the HIP sources of the OMM library for gfx950 into an in-tree shared library.

    python -m paper_2209_05934_amd.build [source ...]

writes paper_2209_05934_amd/lib/libomm_mi355x.so.  Every call recompiles every
source (or only the named ones, reusing the other objects of an earlier build).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIBNAME = "libomm_mi355x.so"
# (source, object, extra flags): the three tile-product steps are compiled once
# per arithmetic precision (OMM_PREC 0: FP64, 1: FP32, 2: BF16) so that their
# many kernel instances build in parallel
PRODUCT_SOURCES = ["dir_products.hip", "proj_products.hip", "grad_products.hip"]
SOURCES = ([("symbolic.hip", "symbolic.o", [])]
           + [(src, src.replace(".hip", f"_p{k}.o"), [f"-DOMM_PREC={k}"])
              for src in PRODUCT_SOURCES for k in range(3)]
           + [(src, src.replace(".hip", ".o"), []) for src in ("numeric.hip", "cholesky.hip", "engine.hip")]
           + [("coeff_io.cpp", "coeff_io.o", []), ("kpoint.cpp", "kpoint.o", [])])
ARCH = os.environ.get("OMM_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-I" + os.path.join(ROOT, "include"),
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def lib_path() -> str:
    return os.path.join(LIBDIR, LIBNAME)


def build(verbose: bool = False, jobs: int = 0, only: tuple = ()) -> str:
    """Compile every source (or, with `only`, just those sources, reusing the other
    objects of an earlier build) and link the library."""
    hipcc = _hipcc()
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(item) -> str:
        src, objname, extra = item
        obj = os.path.join(objdir, objname)
        cmd = [hipcc, *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose:
            print(f"compiled {objname}", flush=True)
        return obj

    if jobs <= 0:
        jobs = min(len(SOURCES), os.cpu_count() or 4)
    # longest first, so the slowest objects start at once
    order = sorted(SOURCES, key=lambda it: 0 if it[0] in PRODUCT_SOURCES else 1)
    todo = [it for it in order if not only or it[0] in only]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, todo))
    objs = [os.path.join(objdir, it[1]) for it in SOURCES]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"objects missing (build everything first): {missing}")
    out = lib_path()
    tmp = out + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs,
           "-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}", flush=True)
    return out


if __name__ == "__main__":
    # python -m paper_2209_05934_amd.build [source ...]: all sources, or only the named ones
    build(verbose=True, only=tuple(sys.argv[1:]))
    sys.exit(0)
