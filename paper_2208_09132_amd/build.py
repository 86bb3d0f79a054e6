"""Build the gfx950 HIP library ``libcdugks.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcdugks.so")
# (source, object name, extra flags): the face-sum unit is compiled once per
# dimension; all units compile in parallel
UNITS = [("cdugks_kernels.hip", "cdugks_kernels", []),
         ("cdugks_face_sums.hip", "cdugks_face_sums_d1", ["-DCDG_FACE_DIM=1"]),
         ("cdugks_face_sums.hip", "cdugks_face_sums_d2", ["-DCDG_FACE_DIM=2"]),
         ("cdugks_face_sums.hip", "cdugks_face_sums_d3", ["-DCDG_FACE_DIM=3"]),
         ("cdugks_batched.hip", "cdugks_batched", []),
         ("cdugks_api.cpp", "cdugks_api", []),
         ("cdugks_serve.cpp", "cdugks_serve", []),
         ("cdugks_vgrid.cpp", "cdugks_vgrid", [])]
JOBS = int(os.environ.get("CDUGKS_BUILD_JOBS", "8"))
ARCH = os.environ.get("CDUGKS_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # contraction only within a source expression: every kernel instantiation
    # (single problem, batched, any dimension mix) rounds identically
    "-ffp-contract=on",
    # packed FP32 instructions stay off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src, name, extra in UNITS:
        obj = os.path.join(objdir, name + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([hipcc, *HIPCC_FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)

    with ThreadPoolExecutor(max_workers=max(1, JOBS)) as ex:
        results = list(ex.map(run, cmds))
    for cmd, res in zip(cmds, results):
        if res.returncode != 0:
            errs = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
            raise RuntimeError("hipcc failed: " + " ".join(cmd) + "\n" + "\n".join(errs[-60:]))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
