"""Sanitizer builds of the host code (CPU only): the FP64 oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, driven through every entry point; the C ABI's host side (argument
validation, handles) under the same sanitizers, exercised by the ABI tests; and an exhaustive
host check of the bricked addressing the kernels use."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
OUT = os.path.join(ROOT, "_build", "san")
CSRC = os.path.join(ROOT, "paper_1707_00442_amd", "csrc")
# host-only sanitizers: each flag is scoped to the host pass of hipcc
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    out = (r.stdout + r.stderr).strip()
    return r.returncode, out


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _asan_runtime():
    r = subprocess.run(["hipcc", "--print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = found[0] if found else ""
    if not path:
        pytest.skip("clang AddressSanitizer runtime not found")
    return path


def test_oracle_under_address_and_undefined_sanitizers():
    _need("gcc")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_sanitize")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Werror", "-fsanitize=address",
                    "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(NATIVE, "oracle_sanitize.c"), os.path.join(ROOT, "oracle",
                                                                            "oracle.c"),
                    "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe])
    print(out)
    assert rc == 0 and "render calls ok" in out, out


def test_brick_addressing_host_check():
    _need("hipcc")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "brick_bounds")
    rc, out = _run(["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *HOST_SAN,
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(NATIVE, "brick_bounds.hip"), "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe])
    print(out)
    assert rc == 0 and "checked, ok" in out, out


def test_c_abi_host_code_under_sanitizers():
    """libsvr with its C-ABI translation unit (argument validation, ownership of the
    handles) built with AddressSanitizer and UndefinedBehaviorSanitizer on the host, the
    ABI tests run against it in a process that preloads the sanitizer runtime."""
    _need("hipcc")
    objs = [o for o in glob.glob(os.path.join(ROOT, "_build", "*.hip.o"))
            if not o.endswith("api.hip.o")]
    if len(objs) < 5:
        pytest.skip("the library's objects are not built (run __graft_entry__.build())")
    os.makedirs(OUT, exist_ok=True)
    obj = os.path.join(OUT, "api_san.o")
    lib = os.path.join(OUT, "libsvr_san.so")
    rc, out = _run(["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
                    os.path.join(CSRC, "api.hip"), "-o", obj])
    assert rc == 0, out
    rc, out = _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, "-o", lib,
                    obj, *sorted(objs)])
    assert rc == 0, out
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               SVR_LIBRARY=lib)
    rc, out = _run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"),
                    "-q", "-p", "no:cacheprovider"], env=env)
    print(out[-2000:])
    assert rc == 0, out[-4000:]
    assert "passed" in out and "runtime error" not in out and "AddressSanitizer" not in out
