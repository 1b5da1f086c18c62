"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

  * the library with every host source (tables, problem, C-ABI, server) compiled with both
    sanitizers runs the C-ABI tests (symbol table, host tables, validation, server and
    allocation-free refusals) through VPS_LIB with the ASan runtime preloaded, and must finish
    without a sanitizer report;
  * the table generator (host tables.cpp + gen_tables.cpp) built with both sanitizers emits the
    same header as the regular build.
GPU kernels are not instrumented (no device sanitizer is used here)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")),
                                 reason="needs hipcc")]


def _fail_markers(text):
    return [m for m in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer") if m in text]


def test_c_abi_tests_pass_with_sanitized_host_code():
    from paper_2405_19004_amd import build
    lib = build.build_sanitized()
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("no shared ASan runtime found")
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("another preload library is set; the ASan runtime must be loaded first")
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, VPS_LIB=lib, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and not _fail_markers(out), out[-4000:]
    assert " passed" in out


def test_table_generator_under_sanitizers(tmp_path):
    from paper_2405_19004_amd import build
    gen = os.path.join(build.GEN_DIR, "patch_tables_gen.hpp")
    if not os.path.exists(gen):
        build.build()
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "gen_tables_san")
    cmd = [cxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I" + build.CSRC, os.path.join(build.CSRC, "gen_tables.cpp"), os.path.join(build.CSRC, "tables.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and not _fail_markers(r.stderr), r.stderr[-4000:]
    assert r.stdout == open(gen).read()
