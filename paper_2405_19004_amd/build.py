"""Build libvps.so (HIP for gfx950 + host C++) in-tree.

Usage: python -m paper_2405_19004_amd.build  (or paper_2405_19004_amd.build.build()).
Compiles every source under csrc/ with hipcc into csrc/../_build/*.o in parallel
and links paper_2405_19004_amd/libvps.so.  Always recompiles (the build check
must exercise the compiler).
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvps.so")

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed FP32 instructions are disabled for every device function
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + os.path.join(HERE, "_build", "gen"),
    "-Wno-unused-command-line-argument",
]
SOURCES = ["smoother.hip", "grid.hip", "vector.hip", "tables.cpp", "problem.cpp", "capi.cpp", "server.cpp"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src, verbose):
    out = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + COMMON + ["-c", os.path.join(CSRC, src), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, r.stderr[-8000:]))
    return out


GEN_DIR = os.path.join(BUILD, "gen")


def _generate_tables(verbose):
    """Compile and run gen_tables.cpp (host) to write the constexpr patch tables header."""
    os.makedirs(GEN_DIR, exist_ok=True)
    exe = os.path.join(BUILD, "gen_tables")
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        raise RuntimeError("a host C++ compiler is needed to generate the patch tables")
    cmd = [cxx, "-O2", "-std=c++17", "-I" + CSRC, os.path.join(CSRC, "gen_tables.cpp"), os.path.join(CSRC, "tables.cpp"),
           "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("table generator failed to build:\n" + r.stderr[-4000:])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    with open(os.path.join(GEN_DIR, "patch_tables_gen.hpp"), "w") as f:
        f.write(out)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    _generate_tables(verbose)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-8000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
