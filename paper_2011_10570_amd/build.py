"""Builds the in-tree shared library ``libltsmi.so`` (C ABI of include/lts.h) for gfx950.

    python -m paper_2011_10570_amd.build        # always recompiles

hipcc cross-compiles the device code without a GPU present.  Packed-FP32 VALU
instructions are disabled for all device code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libltsmi.so")
ARCH = os.environ.get("LTS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["mesh.cpp", "coeffs.cpp", "remesh.cpp", "api.cpp", "k_fused.hip", "k_fused_batch.hip", "k_ghost.hip", "k_stream.hip",
           "k_phase.hip"]

# -ffp-contract=on: a multiply-add is fused only inside one expression, so the
# rounding of a stencil or combine does not depend on how the compiler lays out
# the surrounding code (loops unrolled or not, kernel shape); every kernel that
# evaluates the same expression gets bitwise the same result.
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-ffp-contract=on",
          f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="ltsbuild_") as tmp:
        objs, procs = [], []
        # the sources compile independently: all at once, then one link
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        errors = []
        for src, pr in procs:
            out, err = pr.communicate()
            if pr.returncode != 0:
                errors.append(f"compile of {src} failed:\n{out}\n{err}")
        if errors:
            raise RuntimeError("\n".join(errors))
        out_tmp = LIB + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
