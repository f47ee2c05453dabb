"""Build libfock.so (HIP kernels + C ABI host library) for gfx950 in-tree.

    python -m paper_2606_05297_amd.build [--jobs N]

Every source is compiled with hipcc for --offload-arch=gfx950 with packed
FP32 instructions disabled, then linked into paper_2606_05297_amd/libfock.so.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfock.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = [
    "kernels_h.hip",
    "stencil2.hip",
    "noalloc.hip",
    "probe.hip",
    "kernels_pool.hip",
    "kernels_gate.hip",
    "kernels_gate_da.hip",
    "kernels_gate_db.hip",
    "kernels_gate_dc.hip",
    "kernels_gate_dd.hip",
    "kernels_gate_de.hip",
    "kernels_gate_df.hip",
    "gate_half.hip",
    "gate_real.hip", "gate_real_fuse.hip",
    "sector.hip",
    "sweep_kernels.hip",
    "sweep.cpp",
    "host_common.cpp",
    "api.cpp",
    "adapt.cpp",
    "hva.cpp",
    "bfgs.cpp",
    "fuse_kernels.hip",
    "gate1_kernels.hip",
    "f64_kernels.hip",
    "adapt64.cpp",
    "dense_gate.hip",
    "mlp_kernels.hip",
    "mlp.cpp",
]

COMMON = [
    "--offload-arch=gfx950",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


# Sources with matrix-core (MFMA) instructions; their device assembly is checked
# after compilation (see check_mfma_operands).
MFMA_SOURCES = ["dense_gate.hip", "mlp_kernels.hip"]

_MFMA_RE = re.compile(r"v_mfma_\w+\s+([av])\[(\d+):(\d+)\],[^\n]*,\s*([av])\[(\d+):(\d+)\]\s*$", re.M)


def check_mfma_operands(src: str) -> int:
    """Compile `src` to gfx950 device assembly and reject any matrix instruction
    whose destination registers partially overlap its accumulator input (the
    two must be identical or disjoint; a partial overlap gives wrong sums).
    Returns the number of MFMA instructions inspected."""
    asm = os.path.join(BUILD, os.path.splitext(src)[0] + ".s")
    cmd = [HIPCC, *COMMON, "--cuda-device-only", "-S", "-x", "hip", os.path.join(CSRC, src), "-o", asm]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"assembly generation failed: {' '.join(cmd)}\n{r.stderr}")
    with open(asm) as fh:
        n, bad = mfma_overlaps(fh.read())
    if bad:
        raise RuntimeError(f"{src}: matrix instruction with partially overlapping dst/srcC: {bad[0]}")
    return n


def mfma_overlaps(text: str):
    """(number of MFMA instructions, those whose dst and srcC ranges overlap
    without being identical) in device assembly text."""
    n, bad = 0, []
    for m in _MFMA_RE.finditer(text):
        n += 1
        dk, d0, d1, ck, c0, c1 = m.group(1), int(m.group(2)), int(m.group(3)), m.group(4), int(m.group(5)), int(m.group(6))
        if dk == ck and (d0, d1) != (c0, c1) and not (d1 < c0 or c1 < d0):
            bad.append(m.group(0).strip())
    return n, bad


def build(jobs: int = 8, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, SOURCES))
        nm = sum(ex.map(check_mfma_operands, MFMA_SOURCES))
    if verbose:
        print(f"checked {nm} matrix instructions")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    try:
        build(a.jobs)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
