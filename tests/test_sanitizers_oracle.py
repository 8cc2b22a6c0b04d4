"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (a host
build of its C code, every finding fatal).

The oracle's own pin tests run against the sanitized library in a child
process whose allocator the sanitizer runtime replaces; a deliberate
out-of-bounds read through the C API shows that the sanitizer is live in
such a process."""
import glob
import os
import subprocess
import sys

import pytest

from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def san_env(tmp_path_factory):
    if os.environ.get("LD_PRELOAD") or os.path.exists("/etc/ld.so.preload"):
        pytest.skip("a library is preloaded already: the sanitizer runtime would have to displace it")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = orc.build_sanitized(str(tmp_path_factory.mktemp("san") / "liborc_san.so"))
    return dict(os.environ, LD_PRELOAD=rt, OSANN_ORACLE_LIB=lib,
                ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:halt_on_error=1",
                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def test_sanitizer_catches_an_overflow(san_env):
    # ranks 64 components of a 4-element vector: reads past the buffer
    code = ("import numpy as np; from oracle import oracle as o; L = o.lib(); "
            "v = np.zeros(4, np.float32); out = np.zeros(64, np.int32); "
            "L.orc_rank_order(v.ctypes.data, 64, out.ctypes.data)")
    r = subprocess.run([sys.executable, "-c", code], env=san_env, cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]


def test_oracle_pins_pass_under_sanitizers(san_env):
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert len(files) >= 10
    r = subprocess.run([sys.executable, "-m", "pytest", *files, "-x", "-q", "-p", "no:cacheprovider"],
                       env=san_env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
