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


SAN_DIR = os.path.join(BUILD, "sanitize")
HOST_SOURCES = ["tables.cpp", "problem.cpp", "capi.cpp", "server.cpp"]


def asan_runtime():
    """Path of the compiler's shared AddressSanitizer runtime (host), or None."""
    r = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    base = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(_hipcc()))), "llvm", "lib", "clang")
    for ver in sorted(os.listdir(base)) if os.path.isdir(base) else []:
        cand = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return cand
    return None


def build_sanitized(verbose=False):
    """libvps with its host code under AddressSanitizer and UndefinedBehaviorSanitizer.

    The host sources are recompiled with the sanitizers (host compilation only: the device code of
    every kernel is the regular build's), then linked with the regular objects of the kernel
    sources.  For host-side tests without a GPU: load it through VPS_LIB with the ASan runtime
    preloaded.  Returns the library path."""
    for src in SOURCES:
        if not os.path.exists(os.path.join(BUILD, os.path.splitext(src)[0] + ".o")):
            build(verbose)
            break
    os.makedirs(SAN_DIR, exist_ok=True)
    flags = ["-O1", "-g", "-fno-omit-frame-pointer"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]

    def one(src):
        out = os.path.join(SAN_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [_hipcc()] + [f for f in COMMON if f != "-O3"] + flags + san + ["-c", os.path.join(CSRC, src), "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("sanitized compile failed: %s\n%s" % (src, r.stderr[-8000:]))
        return out

    with cf.ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(one, HOST_SOURCES))
    objs += [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES if s not in HOST_SOURCES]
    lib = os.path.join(SAN_DIR, "libvps_sanitized.so")
    # host link (clang++ of the same toolchain): the kernel objects carry their device code
    clangxx = os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = shutil.which("clang++") or clangxx
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(_hipcc()))), "lib")
    cmd = [clangxx, "-shared", "-fPIC", "-shared-libsan", "-fsanitize=address,undefined", "-o", lib] + objs + \
        ["-L" + rocm_lib, "-Wl,-rpath," + rocm_lib, "-lamdhip64"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stderr[-8000:])
    return lib


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
