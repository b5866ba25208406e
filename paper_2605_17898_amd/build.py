"""Build libmfgp.so (HIP for gfx950) in-tree.

Every source under csrc/ is compiled with hipcc for gfx950; the entry-sweep
source is compiled once per kernel family so the instantiations build in
parallel.  Objects go to _build/, the library to this package directory.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmfgp.so")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    # no packed FP32 (v_pk_*_f32) anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: with AGPR accumulators the compiler
    # copied them between the two register files inside the sweep loops
    # (about 20 of 120 VALU slots per step), and on gfx950 every VALU slot adds
    # to the sweep time because the FP32 MFMA pipe does not overlap the VALU.
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-result",
]

UNITS = [
    ("sweep_fam.hip", "sweep_rbf.o", ["-DMFGP_FAM=0"]),
    ("sweep_fam.hip", "sweep_m12.o", ["-DMFGP_FAM=1"]),
    ("sweep_fam.hip", "sweep_m32.o", ["-DMFGP_FAM=2"]),
    ("sweep_fam.hip", "sweep_m52.o", ["-DMFGP_FAM=3"]),
    ("core.hip", "core.o", []),
    ("vec.hip", "vec.o", []),
    ("cg.hip", "cg.o", []),
    ("adjoint.hip", "adjoint.o", []),
    ("mfma.hip", "mfma.o", []),
    ("abi.hip", "abi.o", []),
    ("timing.hip", "timing.o", []),
    ("batch.hip", "batch.o", []),
    ("hybrid.hip", "hybrid.o", []),
    ("gram.hip", "gram.o", []),
    ("sum.hip", "sum.o", []),
    ("ski.hip", "ski.o", []),
    ("precond.hip", "precond.o", []),
    ("prod.hip", "prod.o", []),
]
HOST_UNITS = [("slq.cpp", "slq.o")]
# Standalone measurement programs (not linked into the library): the issue-rate
# probe whose cycle costs turn a sweep's instruction counts into its bound.
PROGRAMS = [("issue_rates.hip", "issue_rates")]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the mfgp library needs ROCm's hipcc to build")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    cmds = []
    for src, obj, extra in UNITS:
        cmds.append([cc, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)])
    for src, obj in HOST_UNITS:
        cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o",
                     os.path.join(BUILD, obj)])
    for src, exe in PROGRAMS:
        cmds.append([cc, *HIP_FLAGS, os.path.join(CSRC, src), "-o", os.path.join(PKG, exe)])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for r in ex.map(_run, cmds):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    objs = [os.path.join(BUILD, o) for _, o, _ in UNITS] + [os.path.join(BUILD, o) for _, o in HOST_UNITS]
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-L/opt/rocm/lib", "-lrocblas", "-lhipfft",
          "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
