"""The C-ABI layer's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: osann_abi.cpp is compiled again with the
sanitizers on its host pass only (device code unchanged), linked with the
library's other objects, and the ABI's CPU tests (argument checks, error
paths, the allocator hook, struct layouts) run against that build in a child
process with the sanitizer runtime preloaded and every finding fatal."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1509_03453_amd")
OBJDIR = os.path.join(ROOT, "_build")


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def san_lib(tmp_path_factory):
    if os.environ.get("LD_PRELOAD") or os.path.exists("/etc/ld.so.preload"):
        pytest.skip("a library is preloaded already: the sanitizer runtime would have to displace it")
    from paper_1509_03453_amd import build as Bd
    rt = _clang_asan_runtime()
    others = [o for o in glob.glob(os.path.join(OBJDIR, "*.o")) if not o.endswith("osann_abi.cpp.o")]
    if rt is None or not shutil.which(Bd.hipcc()) or len(others) < 10:
        pytest.skip("needs hipcc, clang's ASan runtime and the library's objects (build first)")
    d = tmp_path_factory.mktemp("abi_san")
    obj, lib = str(d / "abi_san.o"), str(d / "libosann_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([Bd.hipcc(), "-x", "hip", "-c", os.path.join(PKG, "csrc", "osann_abi.cpp"), "-o", obj, "-O1", "-g",
                    "-std=c++17", "-fPIC", f"--offload-arch={Bd.ARCH}", "-I", Bd.INCLUDE, "-I", Bd.CSRC]
                   + Bd.DEVICE_FLAGS + san, check=True, capture_output=True)
    subprocess.run([Bd.hipcc(), "-shared", "-fPIC", f"--offload-arch={Bd.ARCH}", "-shared-libsan", "-o", lib, obj]
                   + others + ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"],
                   check=True, capture_output=True)
    return lib, rt


def test_abi_build_is_instrumented(san_lib):
    lib, _ = san_lib
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle" in syms


def test_abi_cpu_tests_pass_under_sanitizers(san_lib):
    lib, rt = san_lib
    env = dict(os.environ, LD_PRELOAD=rt, OSANN_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = ("import sys, pytest; from paper_1509_03453_amd import binding as B; "
            f"assert B.LIB_PATH == {lib!r}; "
            "sys.exit(pytest.main(['tests/test_abi_exports.py', '-x', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu']))")
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
