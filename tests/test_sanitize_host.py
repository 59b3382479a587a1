"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU.  The oracle (pvg_oracle.cpp) and the library's host code (argument
validation in api.cpp, the workspace planning, the serving scheduler driven
by its stub launcher, fault injection included) are rebuilt with the
sanitizers, and a set of CPU tests runs against those builds in a child
process with the sanitizer runtime preloaded.  The library's device code is
compiled as usual: every sanitizer option reaches the host pass only.  Any
sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
# host pass only, each option right after -Xarch_host
HOST_SANITIZE = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                 "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()
ORACLE_SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
TESTS = ["tests/test_lib_abi.py", "tests/test_serve_sched.py", "tests/test_host_plan.py",
         "tests/test_oracle_pins.py", "tests/test_oracle_pins_projection.py", "tests/test_oracle_grad_terms.py",
         "tests/test_oracle_sky.py"]


def _runtime():
    if not os.path.exists(CLANG):
        return None
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    rt = _runtime()
    if rt is None:
        pytest.skip("clang's sanitizer runtime is not installed")
    d = tmp_path_factory.mktemp("sanitize")
    sys.path.insert(0, ROOT)
    from paper_2311_18561_amd import build as B
    lib = B.build(out=str(d / "libpvg.so"), objdir=str(d / "obj"), extra_flags=HOST_SANITIZE)
    orc = str(d / "liboracle.so")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                    *ORACLE_SANITIZE, "-o", orc, os.path.join(ROOT, "oracle", "pvg_oracle.cpp")], check=True)
    return rt, lib, orc


def test_builds_are_instrumented(builds):
    _, lib, orc = builds
    for path in (lib, orc):
        syms = subprocess.run(["nm", "-D", path], capture_output=True, text=True, check=True).stdout
        assert "__asan_report" in syms and "__ubsan_handle" in syms, path


def test_host_code_under_sanitizers(builds):
    rt, lib, orc = builds
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "PVG_LIB": lib,
        "PVG_ORACLE_LIB": orc,
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *TESTS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert r.returncode == 0, out[-6000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert " passed" in out
