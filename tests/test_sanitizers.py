"""CPU sanitizer tier: the oracle and the library's host-side code built with
AddressSanitizer and UndefinedBehaviorSanitizer (every finding fatal), then
exercised by the oracle's pins and by the C-ABI validation tests in a child
process that preloads the ASan runtime.  Host code only: no GPU is touched
(the validation tests reject every call before any HIP runtime call)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
ORACLE_PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_ground.py", "tests/test_oracle_maps.py",
               "tests/test_oracle_size_filter.py"]


def _runtime(name):
    path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def _clang_runtime():
    """The ASan runtime (UBSan handlers included) of the ROCm clang that
    hipcc drives."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        pytest.skip("clang ASan runtime not available")
    return hits[-1]


def _sanitized_env(extra, runtime=None):
    env = dict(os.environ)
    env.update(extra)
    env["LD_PRELOAD"] = runtime or _runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def _run(args, env):
    p = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = p.stdout + p.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "libflic_oracle_san.so")
    src = os.path.join(ROOT, "oracle", "flic_oracle.c")
    subprocess.check_call(["gcc", "-O1", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
                           *SAN, "-o", lib, src, "-lm"])
    env = _sanitized_env({"FLIC_ORACLE_LIB": lib})
    # the child really loads the sanitized build
    out = _run(["-c", "import oracle; oracle.lib(); print(oracle._LIB)"], env)
    assert lib in out
    out = _run(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *ORACLE_PINS], env)
    assert " passed" in out


def test_host_api_under_asan_and_ubsan(tmp_path):
    """The host files (flic_api.cpp: argument checks; flic_serve.cpp: the
    serving runtime's scheduler, run on its simulated device) with their host
    halves sanitized, exercised by the C-ABI validation tests and the native
    serving tests; the device code and the kernel objects are the regular
    build's."""
    from paper_2003_00575_amd import build
    host_files = ("flic_api", "flic_serve")
    objs = [os.path.join(build.OBJ_DIR, f) for f in sorted(os.listdir(build.OBJ_DIR))
            if f.endswith(".o") and f[:-2] not in host_files] if os.path.isdir(build.OBJ_DIR) else []
    if not any("flic_kernels" in o for o in objs):
        pytest.skip("kernel objects not built")
    host_san = [a for f in SAN[:2] for a in ("-Xarch_host", f)] + ["-fno-omit-frame-pointer", "-g"]
    san_objs = []
    for name in host_files:
        obj = str(tmp_path / f"{name}_san.o")
        subprocess.check_call([build.HIPCC, *build.FLAGS, *host_san, "-c", "-o", obj,
                               os.path.join(build.CSRC, name + ".cpp")])
        san_objs.append(obj)
    lib = str(tmp_path / "libflic_san.so")
    subprocess.check_call([build.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san,
                           "-o", lib, *san_objs, *objs])
    env = _sanitized_env({"FLIC_LIB": lib}, _clang_runtime())
    out = _run(["-c", "from paper_2003_00575_amd import flic; flic.lib(); print(flic.LIB_PATH)"], env)
    assert lib in out
    out = _run(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi.py",
                "tests/test_serve_native.py"], env)
    assert " passed" in out
