"""Build libflic.so (HIP kernels for gfx950 + the C-ABI host code) in-tree.

    python -m paper_2003_00575_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflic.so")
SOURCES = [os.path.join(CSRC, "flic_kernels.hip"), os.path.join(CSRC, "flic_api.cpp"),
           os.path.join(CSRC, "flic_ground.hip"), os.path.join(CSRC, "flic_noalloc.hip"),
           os.path.join(CSRC, "flic_serve.cpp"), os.path.join(CSRC, "flic_stage.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the edge test must be a chain of separately rounded
# binary32 operations (no fused multiply-add), bit-identical to the CPU.
# -packed-fp32-ops off: no v_pk_*_f32 instructions are generated.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]
TILE_WIDTHS = (64, 128, 256)
OBJ_DIR = os.path.join(HERE, "_build")


def build(verbose: bool = False) -> str:
    """Compile the clustering kernels once per tile width and skip-edge
    mode, the ground kernel and the host API, in parallel, then link
    libflic.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    cmds = []
    for tw in TILE_WIDTHS:
        for maps in (0, 1):
            obj = os.path.join(OBJ_DIR, f"flic_kernels_w{tw}_m{maps}.o")
            cmds.append((obj, [HIPCC, *FLAGS, f"-DFLIC_TILE_W={tw}", f"-DFLIC_MAPS={maps}", "-c", "-o", obj,
                               SOURCES[0]]))
    for src in SOURCES[1:]:
        obj = os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")
        cmds.append((obj, [HIPCC, *FLAGS, "-c", "-o", obj, src]))
    procs = []
    for obj, cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((obj, subprocess.Popen(cmd)))
    failed = [obj for obj, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc ({', '.join(os.path.basename(f) for f in failed)})")
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for o, _ in cmds]]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


def device_asm(out_path: str, source: int = 0) -> str:
    """Write the gfx950 assembly of SOURCES[source] (for instruction checks)."""
    cmd = [HIPCC, *[f for f in FLAGS if f != "-fPIC"], "-S", "--cuda-device-only",
           "-o", out_path, SOURCES[source]]
    subprocess.check_call(cmd)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
