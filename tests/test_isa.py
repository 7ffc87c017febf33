"""The clustering kernels' gfx950 assembly holds no floating-point fused
multiply-add and no packed FP32 instruction, so the edge test of Eq. (4) is a
chain of separately rounded binary32 operations (bit-identical to the CPU
oracle).  Compiles the 64-column kernels in both skip-edge modes (about 100 s
on 2 cores; integer multiply-adds from address arithmetic are allowed)."""
import os
import re
import subprocess

import pytest

from paper_2003_00575_amd import build

FLOAT_FUSED = re.compile(r"\bv_(?:fma|fmac|mad|mac|pk_fma|pk_mul|pk_add|fma_mix|mad_mix)\w*_f(?:16|32|64)\b"
                         r"|\bv_(?:fmac|fma|mad)_(?:f16|f32|f64|legacy)\w*")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    d = tmp_path_factory.mktemp("isa")
    procs = []
    for maps in (0, 1):
        out = str(d / f"w64_m{maps}.s")
        cmd = [build.HIPCC, *[f for f in build.FLAGS if f != "-fPIC"], "-DFLIC_TILE_W=64", f"-DFLIC_MAPS={maps}",
               "-S", "--cuda-device-only", "-o", out, build.SOURCES[0]]
        procs.append((out, subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)))
    outs = []
    for out, p in procs:
        assert p.wait() == 0
        outs.append(out)
    return outs


def test_no_float_fma_or_packed_fp32(asm):
    for path in asm:
        text = open(path).read()
        assert "k_tile_label" in text and "k_border_unite" in text and "k_relabel" in text
        hits = sorted(set(FLOAT_FUSED.findall(text)))
        assert not hits, f"{os.path.basename(path)}: {hits}"


def test_pattern_catches_float_fma():
    # the check itself: float forms match, integer address arithmetic does not
    assert FLOAT_FUSED.findall("v_fma_f32 v1, v2, v3, v4\n v_pk_mul_f32 v[0:1]\n v_fmac_f32_e32 v1")
    assert not FLOAT_FUSED.findall("v_mad_u64_u32 v[0:1]\n v_mad_i32_i24 v2\n v_mad_u32_u24 v3")
