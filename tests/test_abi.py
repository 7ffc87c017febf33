"""C-ABI checks that run without a GPU: the library loads, exports every
function include/flic.h declares, and rejects invalid arguments on the host
before any HIP call (labels_out untouched)."""
import ctypes
import os
import re

import pytest

from paper_2003_00575_amd import flic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flic.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(flic_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(flic.LIB_PATH):
        from paper_2003_00575_amd import build
        build.build()
    return flic.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


# Fake, never-dereferenced addresses: validation must reject before any HIP call.
R, LBL, CV, CH = 0x10000000, 0x20000000, 0x30000000, 0x40000000


@pytest.mark.parametrize("args, why", [
    ((0, 4, 64, CV, CH, 0.5, 3, LBL), "null range"),
    ((R, 4, 64, CV, CH, 0.5, 3, 0), "null labels"),
    ((R, 4, 64, 0, CH, 0.5, 3, LBL), "null cos_v"),
    ((R, 4, 64, CV, 0, 0.5, 3, LBL), "null cos_h"),
    ((R, 0, 64, CV, CH, 0.5, 3, LBL), "H < 1"),
    ((R, 4, 0, CV, CH, 0.5, 3, LBL), "W < 1"),
    ((R, 4, 64, CV, CH, 0.5, 0, LBL), "N < 1"),
    ((R, 4, 64, CV, CH, 0.5, 9, LBL), "N > 8"),
    ((R, 4, 6, CV, CH, 0.5, 3, LBL), "2N >= W"),
    ((R, 65536, 65536, CV, CH, 0.5, 3, LBL), "H*W > INT32_MAX"),
    ((R, 4, 64, CV, CH, float("nan"), 3, LBL), "NaN threshold"),
    ((R, 4, 64, CV, CH, float("inf"), 3, LBL), "inf threshold"),
    ((R, 4, 64, CV, CH, -0.5, 3, LBL), "negative threshold"),
    ((R, 4, 64, CV, CH, 0.5, 3, R + 64), "range/labels overlap"),
    ((R, 4, 64, CV, CH, 0.5, 3, CV), "table/labels overlap"),
])
def test_flic_cluster_rejects_invalid_arguments(L, args, why):
    assert flic.cluster_raw(*args) == flic.FLIC_EINVAL, why
    assert flic.last_error() != ""


def test_null_tables_struct_and_ctx(L):
    assert L.flic_cluster(R, 4, 64, None, 0.5, 3, LBL) == flic.FLIC_EINVAL
    assert flic.cluster_async_raw(None, R, 4, 64, CV, CH, 0.5, 3, LBL, 0) == flic.FLIC_EINVAL
    assert flic.batched_raw(None, [], 0) == flic.FLIC_EINVAL
    assert L.flic_ctx_create(None, 0, 0) == flic.FLIC_EINVAL
    assert L.flic_ctx_create(ctypes.byref(ctypes.c_void_p()), -1, 0) == flic.FLIC_EINVAL
    assert L.flic_plan_launch(None, None, 0, None) == flic.FLIC_EINVAL
    assert L.flic_set_tile_override(None, 64) == flic.FLIC_EINVAL
    L.flic_ctx_destroy(None)
    L.flic_plan_destroy(None)


def test_scan_struct_layout_matches_header(tmp_path):
    """The binding's flic_scan mirror has the header's size and field offsets."""
    import ctypes
    import subprocess
    from paper_2003_00575_amd import flic
    src = tmp_path / "layout.c"
    fields = [f for f, _ in flic._Scan._fields_]
    body = "\n".join(f'    printf("%zu\\n", offsetof(flic_scan, {f}));' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "flic.h"\nint main(void) {\n'
                   f'    printf("%zu\\n", sizeof(flic_scan));\n{body}\n    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(flic._Scan)] + [getattr(flic._Scan, f).offset for f in fields]
    assert got == want


def test_ground_tables_struct_layout_matches_header(tmp_path):
    import ctypes
    import subprocess
    from paper_2003_00575_amd import flic
    src = tmp_path / "glayout.c"
    fields = [f for f, _ in flic._GroundTables._fields_]
    body = "\n".join(f'    printf("%zu\\n", offsetof(flic_ground_tables, {f}));' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "flic.h"\nint main(void) {\n'
                   f'    printf("%zu\\n", sizeof(flic_ground_tables));\n{body}\n    return 0;\n}}\n')
    exe = tmp_path / "glayout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(flic._GroundTables)] + [getattr(flic._GroundTables, f).offset for f in fields]
    assert got == want


def test_ground_remove_rejects_null_ctx(L):
    assert L.flic_ground_remove(None, None, 1, 4, 4, None, None, None, None) == flic.FLIC_EINVAL


def test_noalloc_rejects_before_any_hip_call(L):
    # argument errors as for flic_cluster, and a scan beyond the fixed scratch
    assert flic.cluster_noalloc_raw(0, 4, 64, CV, CH, 0.5, 3, LBL, 0) == flic.FLIC_EINVAL
    assert flic.cluster_noalloc_raw(R, 4, 64, CV, CH, 0.5, 9, LBL, 0) == flic.FLIC_EINVAL
    assert flic.cluster_noalloc_raw(R, 1024, 4096, CV, CH, 0.5, 3, LBL, 0) == flic.FLIC_EINVAL
    assert "scratch" in flic.last_error()


def test_plan_parts_validated(L):
    assert L.flic_ctx_set_plan_parts(None, 3) == flic.FLIC_EINVAL


def test_batched_host_rejects_null_ctx(L):
    arr = (flic._Scan * 1)()
    assert L.flic_cluster_batched_host(None, arr, 1, None, None, None) == flic.FLIC_EINVAL
    assert "ctx" in flic.last_error()
