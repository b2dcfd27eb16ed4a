"""Build librmq.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1706_06940_amd.build        # or build() from Python

Every call recompiles.  Objects go to paper_1706_06940_amd/_build/, the
shared library to paper_1706_06940_amd/librmq.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librmq.so")

SOURCES = [
    "blockmin.hip",
    "sparse_table.hip",
    "query.hip",
    "radix_sort.hip",
    "contract.hip",
    "capi.hip",
    "noalloc.hip",
    "server.hip",
    "lca.hip",
]

ARCH = "gfx950"
FLAGS = [
    "-O3",
    "-std=c++17",
    f"--offload-arch={ARCH}",
    "-fPIC",
    "-Wall",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def hipcc() -> str:
    return os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


def scratch_kernels(remarks: str) -> list[tuple[str, int]]:
    """Kernels that the compiler's resource-usage remarks show using scratch
    (per-lane private memory: register spills or private arrays)."""
    found, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and int(m.group(1)) > 0:
            found.append((name, int(m.group(1))))
    return found


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # No kernel may use scratch: every one is sized to keep its state in
    # registers and LDS, and a spill (which can come from a small change, as
    # a run-time shift count once did) costs a pass several times its time.
    spills = scratch_kernels(r.stderr)
    if spills:
        raise RuntimeError(f"kernels of {src} use scratch: " +
                           ", ".join(f"{k} ({b} bytes/lane)" for k, b in spills))
    return obj


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
