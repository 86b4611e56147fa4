"""Build libldpcfd.so (all HIP sources, gfx950) in-tree with hipcc.

The field-size templated kernels are compiled once per field size m = 2..8
(csrc/kernels_q.hip with LDPC_FD_LOGQ = m) next to the host translation unit
(csrc/ldpc_fd.hip), all in parallel, then linked into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libldpcfd.so")
CSRC = os.path.join(PKG, "csrc")
OBJDIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("LDPC_FD_ARCH", "gfx950")
FIELD_SIZES = range(2, 9)

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from forming packed FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]

NOISE = "is not a recognized feature for this target"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _units():
    units = [(os.path.join(CSRC, "ldpc_fd.hip"), os.path.join(OBJDIR, "ldpc_fd.o"), [])]
    for m in FIELD_SIZES:
        units.append((os.path.join(CSRC, "kernels_q.hip"), os.path.join(OBJDIR, f"kernels_q{m}.o"),
                      [f"-DLDPC_FD_LOGQ={m}"]))
    return units


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source and link libldpcfd.so (always recompiles)."""
    os.makedirs(OBJDIR, exist_ok=True)
    cc = hipcc()
    cmds = [[cc, *HIPCC_FLAGS, *extra, "-c", "-o", obj, src] for src, obj, extra in _units()]
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    for cmd, (rc, err) in zip(cmds, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed ({rc}) on {cmd[-1]} {' '.join(cmd[-5:-4])}:\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[obj for _, obj, _ in _units()]]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
