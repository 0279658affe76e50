"""Build libbem.so (HIP kernels for gfx950 + host runtime) in-tree with hipcc.

Device code is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); host C++ (trees, ACA,
server) without floating-point contraction so that tree decisions follow the
plain IEEE expressions written in the source.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libbem.so")
ARCH = os.environ.get("BEM_OFFLOAD_ARCH", "gfx950")

DEVICE_SOURCES = ["entries.hip", "geometry.hip", "near.hip"]
HOST_SOURCES = ["mesh_expand.cpp", "server.cpp", "hmat.cpp", "tree.cpp", "capi.cpp", "aca_kernels.cpp", "dense.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall",
          "-Wno-unused-result"]
DEVICE_FLAGS = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics"]
HOST_FLAGS = ["-x", "hip", "--offload-arch=" + ARCH, "-ffp-contract=off", "-fcx-limited-range", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src, flags, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc"] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(s, DEVICE_FLAGS) for s in DEVICE_SOURCES] + [(s, HOST_FLAGS) for s in HOST_SOURCES]
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], j[1], verbose), jobs))
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
