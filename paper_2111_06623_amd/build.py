"""Build the HIP library (gfx950) in-tree: paper_2111_06623_amd/liblz.so.

Each translation unit compiles in its own hipcc process (in parallel), then
one hipcc call links the shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/lz_fft_f64.hip", "csrc/lz_fft_f32.hip", "csrc/lz_linalg.hip", "csrc/lz_api.hip"]
LIB = os.path.join(HERE, "liblz.so")
OBJDIR = os.path.join(HERE, "_build")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed-fp32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def _compile(src):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    return src, obj, r


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(len(os.sched_getaffinity(0)), 16)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    errors = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, r in errors:
        sys.stderr.write(f"--- {s}\n{r.stdout}{r.stderr}")
    if errors:
        raise RuntimeError("hipcc failed")
    if verbose:
        for s, _, r in results:
            sys.stderr.write(r.stderr)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results]
    r = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
