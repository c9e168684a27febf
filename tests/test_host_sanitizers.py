"""Host AddressSanitizer / UndefinedBehaviorSanitizer run of the C++ layer
(no GPU needed).

The library is rebuilt into a temporary directory with the host side of
every translation unit instrumented (the gfx950 device code is compiled as
usual), and the CPU tests that call it run against that build in a child
Python with the sanitizer runtime preloaded: argument validation and status
codes before any device work, model-file checks, the exported symbols, the
host eigensolver, and the tuning table's file parsing (including malformed
and over-long lines).  Any sanitizer report fails the run.  The build takes
about a minute and a half on 8 cores."""
import concurrent.futures
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2305_20053_amd"))
import build as libbuild  # noqa: E402

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _runtime():
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return rts[-1] if rts else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    if _runtime() is None or not os.path.exists(libbuild.hipcc()):
        pytest.skip("no hipcc or sanitizer runtime in this image")
    out = tmp_path_factory.mktemp("san")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={libbuild.ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-w"] + SAN + \
            ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]

    def one(src):
        obj = str(out / (src + ".o"))
        r = subprocess.run([libbuild.hipcc()] + flags + ["-x", "hip", "-c", os.path.join(libbuild.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    jobs = max(1, min(len(libbuild.SOURCES), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, libbuild.SOURCES))
    lib = str(out / "libsaa_san.so")
    r = subprocess.run([libbuild.hipcc(), "-shared", "-fPIC", f"--offload-arch={libbuild.ARCH}"] + SAN +
                       ["-shared-libsan", "-o", lib] + objs + ["-lrocblas"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return lib


_CHILD = r'''
import os, sys
sys.path.insert(0, {root!r})
import paper_2305_20053_amd as saa
saa.LIB_PATH = {lib!r}
import numpy as np
# the tuning table: choices, the file they persist in, malformed and long lines
path = {cache!r}
with open(path, "w") as f:
    f.write("not-a-pair\n" + "k" * 2000 + " 3\n" + "x 7 trailing\n\n")
os.environ["SAA_TUNE_CACHE"] = path
saa.tune_set("host/check/key", 5)
assert saa.tune_get("host/check/key") == 5
assert saa.tune_get("host/absent/key") is None
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu",
                      os.path.join({root!r}, "tests", "test_boundary.py"),
                      os.path.join({root!r}, "tests", "test_host_eig.py")]))
'''


def test_cpu_tests_under_address_and_undefined_behaviour_sanitizers(sanitized_lib, tmp_path):
    rt = _runtime()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "LD_LIBRARY_PATH": os.path.dirname(rt) + ":" + env.get("LD_LIBRARY_PATH", ""),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",   # the interpreter and HIP runtime keep their allocations
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    code = _CHILD.format(root=ROOT, lib=sanitized_lib, cache=str(tmp_path / "tune.txt"))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout[-4000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, report
