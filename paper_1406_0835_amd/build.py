"""Build libofdft.so (HIP kernels for gfx950 + host C ABI) in-tree with hipcc.

Usage: python -m paper_1406_0835_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libofdft.so")
ARCH = os.environ.get("OFDFT_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-munsafe-fp-atomics"]
SOURCES = [("ofdft_kernels.hip", True), ("ofdft_api.cpp", False), ("ofdft_ewald.cpp", False)]


def _compile(src, device):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + (DEVICE if device else ["-D__HIP_PLATFORM_AMD__"]) + [
        "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


SAN_LIB = os.path.join(BUILD, "san", "libofdft_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(verbose: bool = False) -> str:
    """Host code under AddressSanitizer and UBSan: the C ABI and the Ewald sums compiled by
    g++ with the sanitizers, linked with the unchanged device object of build().  For CPU runs
    of the host paths (argument checks, option validation, Ewald), with libasan preloaded:
        LD_PRELOAD=$(g++ -print-file-name=libasan.so) ASAN_OPTIONS=detect_leaks=0 \
        OFDFT_LIBRARY=<SAN_LIB> python -m pytest tests/test_abi_cpu.py tests/test_ewald_cpu.py"""
    kobj = os.path.join(BUILD, "ofdft_kernels.o")
    if not os.path.exists(kobj):
        build()
    out = os.path.dirname(SAN_LIB)
    os.makedirs(out, exist_ok=True)
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    objs = [kobj]
    for src in ("ofdft_api.cpp", "ofdft_ewald.cpp"):
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        cmd = ["g++", "-std=c++17", "-O1", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include"] + SAN_FLAGS + [
            "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        objs.append(obj)
    cmd = ["g++", "-shared", "-o", SAN_LIB] + objs + SAN_FLAGS + [f"-L{rocm}/lib", "-lamdhip64", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
