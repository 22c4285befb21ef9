"""Compile the HIP sources under csrc/ into libocttrack.so (gfx950).

Objects are compiled in parallel with hipcc and linked into one shared
library next to this file.  The build always recompiles.  Files named
*_inst.hip hold the instantiations of a kernel template and are compiled
once per (precision, spreading mode), so that the largest kernels build in
parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libocttrack.so")
ARCH = os.environ.get("OT_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # no implicit multiply-add contraction: every instantiation of the per-point code
    # (plain, fused, batched) rounds the same way; the fused ops it wants are written out
    "-ffp-contract=off",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _compile(src: str, obj: str, extra=()) -> None:
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}:\n{r.stderr}")
    # hipcc's host pass warns about the GPU-only target feature: harmless
    errs = [l for l in r.stderr.splitlines() if "warning" in l and "packed-fp32-ops" not in l]
    if errs:
        sys.stderr.write("\n".join(errs) + "\n")


# (suffix, defines) of the instantiations of every *_inst.hip file
INST = [("f32_atomic", ["-DOT_INST_T=float", "-DOT_INST_MODE=0"]),
        ("f32_fixed", ["-DOT_INST_T=float", "-DOT_INST_MODE=1"]),
        ("f64_atomic", ["-DOT_INST_T=double", "-DOT_INST_MODE=0"]),
        ("f64_fixed", ["-DOT_INST_T=double", "-DOT_INST_MODE=1"])]


def _units(bdir: str):
    """(source, object, extra flags) of every object of the library."""
    out = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        base = os.path.basename(src)[:-4]
        if base.endswith("_inst"):
            for suf, defs in INST:
                out.append((src, os.path.join(bdir, f"{base}_{suf}.o"), defs))
        else:
            out.append((src, os.path.join(bdir, base + ".o"), []))
    return out


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    units = _units(bdir)
    objs = [o for _, o, _ in units]
    jobs = min(len(units), int(os.environ.get("MAX_JOBS", "8")))
    # the slowest units first, so that they do not start last
    units.sort(key=lambda u: 0 if u[2] else 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda u: _compile(*u), units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
