"""The library's host code under AddressSanitizer, on the CPU.

Builds the host side of every source (blob parsing, argument and box validation, workspace
planning, the entry points' error paths) with ASan, with an empty device bundle in place of the
kernels' code objects (so the build takes seconds), and runs the host-only
ABI tests against that build in a child process with the ASan runtime preloaded.  Any heap,
stack or global overflow, use after free or double free in those paths fails the child.  No GPU
is touched: the device side is not built, and the tests it runs reject every request before a
kernel would launch."""

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_17660_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BUNDLER = "/opt/rocm/llvm/bin/clang-offload-bundler"
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def asan_library(tmp_path_factory):
    if not os.path.exists(HIPCC) or not os.path.exists(BUNDLER) or asan_runtime() is None:
        pytest.skip("hipcc, the offload bundler or the clang ASan runtime is not installed")
    out = tmp_path_factory.mktemp("asan")
    empty = str(out / "empty.hipfb")
    r = subprocess.run([BUNDLER, "-type=o", "-targets=host-x86_64-unknown-linux-gnu-", "-input=/dev/null",
                        f"-output={empty}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    base = [HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC", *ASAN_HOST,
            "-Xclang", "-fcuda-include-gpubinary", "-Xclang", empty, "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = str(out / src.replace(".hip", ".o"))
        r = subprocess.run([*base, "-c", os.path.join(CSRC, src), "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(out / "libtensornet_asan.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-shared", "-fPIC", "-Xarch_host",
                        "-fsanitize=address", "-shared-libsan", "-o", lib, *objs], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in syms, "the host code was not instrumented"
    return lib


def test_host_abi_paths_are_clean_under_asan(asan_library):
    env = dict(os.environ)
    env["TN_LIBRARY"] = asan_library
    env["LD_PRELOAD"] = asan_runtime()
    # the interpreter and its extension modules are not instrumented; leaks at exit are theirs
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=97"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_lib_exports.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
