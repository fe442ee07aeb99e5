"""Build libtadj.so in-tree for gfx950 with hipcc.

    python -m paper_2505_23618_amd.build        (or: python paper_2505_23618_amd/build.py)

Regenerates csrc/tables_gen.h, compiles every csrc/*.hip and csrc/*.cpp into
_build/, and links paper_2505_23618_amd/libtadj.so.  Always recompiles.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
BUILD = PKG.parent / "_build"
LIB = PKG / "libtadj.so"
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code: the compiler must
# not form v_pk_{add,mul,fma}_f32 from scalar or float2 code.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]

# Per-file additions.  The pipelined batched kernels take tile indices with
# single-lane atomics whose results are consumed after a wait of their own;
# the atomic optimizer would rewrite them into wave-wide forms that read the
# result at once, waiting on the loads in flight.
FILE_FLAGS = {"batch_kernels.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{err}")
    return err


def build(verbose: bool = False, jobs: int | None = None) -> Path:
    subprocess.run([sys.executable, str(CSRC / "gen_tables.py")], check=True)
    BUILD.mkdir(exist_ok=True)
    srcs = sorted(list(CSRC.glob("*.hip")) + list(CSRC.glob("*.cpp")))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

    def compile_one(src: Path) -> Path:
        obj = BUILD / (src.stem + ".o")
        msg = _run([hipcc, *HIP_FLAGS, *FILE_FLAGS.get(src.name, []), "-c", str(src), "-o", str(obj)])
        if verbose and msg:
            print(msg)
        return obj

    jobs = jobs or min(8, max(1, len(srcs)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB.with_suffix(".so.tmp")
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
