"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two native drivers (tests/native/) are built with the sanitizers and run:
the library's host code (planner, work-queue and batch planner, statistics,
argument checks; the HIP sources are compiled with the sanitizers on their
host side only, no kernel is launched) and the C oracle (every exported
routine on seeded random small inputs).  A sanitizer report, a leak or a
failed check fails the test.  Builds are cached by source content under
paper_1703_05581_amd/_build/sanitize/."""
import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_05581_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
OUT = os.path.join(ROOT, "paper_1703_05581_amd", "_build", "sanitize")
LLVM = "/opt/rocm/llvm/bin"
LIB_SOURCES = ["ffa_kernels.hip", "ffa_plan.cpp", "ffa_capi.cpp", "ffa_batch.cpp", "ffa_server.cpp",
               "ffa_stats.cpp", "ffa_noalloc.hip"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:halt_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _digest(paths, extra: str) -> str:
    h = hashlib.sha256(extra.encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _cached(name: str, inputs, build) -> str:
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, f"{name}-{_digest(inputs, name)}")
    if not os.path.exists(exe):
        tmp = exe + ".tmp"
        build(tmp)
        os.replace(tmp, exe)
    return exe


def _headers():
    return [os.path.join(ROOT, "include", "ffa.h"), os.path.join(CSRC, "ffa_internal.h")]


def _build_library_driver(exe: str) -> None:
    objdir = exe + ".objs"
    os.makedirs(objdir, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", *SAN,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        subprocess.run(["hipcc", *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, LIB_SOURCES))
    drv = os.path.join(objdir, "driver.o")
    subprocess.run([f"{LLVM}/clang++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(NATIVE, "plan_host_check.cpp"), "-o", drv], check=True)
    subprocess.run([f"{LLVM}/clang++", "-fsanitize=address,undefined", "-o", exe, drv, *objs,
                    "-L/opt/rocm/lib", "-lamdhip64", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    shutil.rmtree(objdir)


def _build_oracle_driver(exe: str) -> None:
    subprocess.run([f"{LLVM}/clang", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
                    os.path.join(NATIVE, "oracle_host_check.c"), os.path.join(ROOT, "oracle", "ffa_oracle.c"),
                    "-lm"], check=True)


needs_toolchain = pytest.mark.skipif(not os.path.exists(f"{LLVM}/clang"), reason="ROCm LLVM toolchain not found")


@needs_toolchain
def test_oracle_under_sanitizers():
    exe = _cached("oracle_host_check", [os.path.join(NATIVE, "oracle_host_check.c"),
                                        os.path.join(ROOT, "oracle", "ffa_oracle.c")], _build_oracle_driver)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and "oracle host check: ok" in r.stdout, r.stdout + r.stderr[-4000:]


@needs_toolchain
def test_library_host_code_under_sanitizers():
    inputs = [os.path.join(CSRC, s) for s in LIB_SOURCES] + _headers() + [
        os.path.join(NATIVE, "plan_host_check.cpp")]
    exe = _cached("plan_host_check", inputs, _build_library_driver)
    # HIP_VISIBLE_DEVICES empty: the runtime sees no GPU even where one exists
    r = subprocess.run([exe], capture_output=True, text=True, env={**ENV, "HIP_VISIBLE_DEVICES": ""},
                       timeout=600)
    assert r.returncode == 0 and "library host check: ok" in r.stdout, r.stdout + r.stderr[-4000:]
