"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The sources whose work is mostly host code (argument checks, scheme
construction from a node and monomial set, weights, tuning tables, batch
planning, the request server, the allocation-free entry point) are compiled
again with the sanitizers on their host pass only; the device code in them,
and the kernel-only sources, are built as in the library.  The result is
linked with tests/lib_asan_driver.c, which calls every host-only entry point
and every stepping call with arguments its checks reject, so no call reaches
a device and the test runs without a GPU.  The run aborts at the first
out-of-bounds access, leak or undefined operation.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

from paper_1904_04048_amd import build as hipbuild

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_SOURCES = ["api", "batch", "noalloc", "persist_plan", "schemes", "serve"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _clang(name):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        return None
    cand = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", name)
    if os.path.exists(cand):
        return os.path.normpath(cand)  # keep the name: it selects the C or C++ driver
    return shutil.which(name)


def _hipcc(src, obj, extra):
    cmd = ["hipcc"] + hipbuild.COMMON + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return obj


@pytest.mark.skipif(shutil.which("hipcc") is None or _clang("clang++") is None, reason="hipcc / clang++ not available")
def test_library_host_code_clean_under_sanitizers(tmp_path):
    jobs = []
    for src in sorted(glob.glob(os.path.join(hipbuild.CSRC, "*.hip"))):
        name = os.path.basename(src)[: -len(".hip")]
        if name in HOST_SOURCES:
            jobs.append((src, str(tmp_path / (name + ".o")), SAN))
        else:
            built = os.path.join(hipbuild.BUILD, name + ".hip.o")
            if os.path.exists(built) and os.path.getmtime(built) >= os.path.getmtime(src):
                jobs.append((None, built, None))
            else:
                jobs.append((src, str(tmp_path / (name + ".o")), []))
    assert sum(1 for j in jobs if j[2] is SAN) == len(HOST_SOURCES)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(lambda j: j[1] if j[0] is None else _hipcc(*j), jobs))
    for name in HOST_SOURCES:
        with open(tmp_path / (name + ".o"), "rb") as f:
            assert b"__asan_report" in f.read(), f"{name} not instrumented"
    drv = str(tmp_path / "drv.o")
    subprocess.run([_clang("clang"), "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", hipbuild.INCLUDE, "-c",
                    os.path.join(HERE, "lib_asan_driver.c"), "-o", drv], check=True)
    exe = str(tmp_path / "lib_asan")
    rocm_lib = os.path.realpath(os.path.join(os.path.dirname(os.path.realpath(shutil.which("hipcc"))), "..", "lib"))
    subprocess.run([_clang("clang++"), "-fsanitize=address,undefined", "-o", exe, drv] + objs
                   + ["-L", rocm_lib, "-lamdhip64", "-Wl,-rpath," + rocm_lib], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr
    assert "0 failed" in out.stdout, out.stdout
