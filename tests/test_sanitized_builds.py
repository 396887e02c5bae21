"""CPU checks under AddressSanitizer and UndefinedBehaviorSanitizer.

* The C oracles, built with both sanitizers (gcc), run the oracle's pin
  tests in a child process with the sanitizer runtimes preloaded.
* The HIP library's host code (argument validation, workspace layout, the
  entry points' early returns), built with both sanitizers on the host pass
  only, runs the C-ABI tests without a GPU in a child process.
* The mesh fine pass's LDS index arithmetic (chunk compaction, per-lane
  lists, fragment staging) replayed by a bounds-checked model built with
  both sanitizers, with the kernel's block sizes: in bounds for the kernel's
  64-face chunks; a 48-face chunk gathered by a 64-lane wave writes records
  past its block (the cause of an earlier GPU memory fault of such a
  variant, shown here on the CPU).

Each child asserts that the sanitized library, not the in-tree one, was
mapped into it.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def clang_asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def run_child(code, env_extra, timeout=900):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    return p.returncode, p.stdout + p.stderr


CHILD = """
import sys, pytest
rc = pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu and not slow"] + {tests!r})
maps = open("/proc/self/maps").read()
assert {lib!r} in maps, "the sanitized library was not loaded"
sys.exit(int(rc))
"""


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = gcc_runtime("libasan.so"), gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    import oracle
    lib = oracle.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    tests = ["tests/test_oracle_pins.py", "tests/test_oracle_margins.py", "tests/test_oracle_options.py",
             "tests/test_oracle_points.py", "tests/test_oracle_fd.py"]
    rc, out = run_child(CHILD.format(tests=tests, lib=lib), {"LD_PRELOAD": f"{asan}:{ubsan}", "ORACLE_LIB_PATH": lib})
    assert rc == 0, out[-4000:]
    assert "passed" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    asan = clang_asan_runtime()
    if asan is None or shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or its sanitizer runtime not installed")
    from paper_2007_08501_amd import build
    lib = build.build(sanitize_host=True, out=str(tmp_path / "librast_san.so"))
    rc, out = run_child(CHILD.format(tests=["tests/test_abi_cpu.py"], lib=lib),
                        {"LD_PRELOAD": asan, "RAST_LIB_PATH": lib})
    assert rc == 0, out[-4000:]
    assert "passed" in out


def test_tile_pass_lds_indexing_model(tmp_path):
    exe = str(tmp_path / "tile_lds_model")
    src = os.path.join(ROOT, "tests", "cpu_models", "tile_lds_model.cpp")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", src, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    ok = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert ok.returncode == 0, ok.stdout + ok.stderr
    assert "every offset in bounds" in ok.stdout
    # a 48-face chunk: the 64-lane gather ranks up to 64 kept faces into 48 records
    bad = subprocess.run([exe, "48"], capture_output=True, text=True, env=env)
    assert bad.returncode == 1, bad.stdout + bad.stderr
    assert "OUT OF BOUNDS: chunk record index 48, limit 48" in bad.stdout
