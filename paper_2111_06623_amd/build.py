"""Build the HIP library (gfx950) in-tree: paper_2111_06623_amd/liblz.so.

Each translation unit compiles in its own hipcc process (in parallel), then
one hipcc call links the shared library.  A second library,
liblz_asan.so, holds the same objects except the API unit (argument
validation, context set-up, checkpoints), whose host code is compiled with
AddressSanitizer for host-only checks (tests/test_asan_host.py); device code
is never instrumented.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/lz_fft_f64.hip", "csrc/lz_fft_f32.hip", "csrc/lz_linalg.hip", "csrc/lz_api.hip"]
LIB = os.path.join(HERE, "liblz.so")
LIB_ASAN = os.path.join(HERE, "liblz_asan.so")
OBJDIR = os.path.join(HERE, "_build")
# host code only: each -fsanitize flag applies to the host compilation
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
ASAN_SOURCES = ["csrc/lz_api.hip"]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed-fp32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def _compile(src, asan=False):
    obj = os.path.join(OBJDIR, os.path.basename(src) + (".asan.o" if asan else ".o"))
    cmd = ["hipcc", *FLAGS, *(ASAN_FLAGS if asan else []), "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    return src, obj, r


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, lib)


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = min(len(SOURCES) + len(ASAN_SOURCES), max(1, min(len(os.sched_getaffinity(0)), 16)))
    tasks = [(src, False) for src in SOURCES] + [(src, True) for src in ASAN_SOURCES]
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda t: _compile(*t), tasks))
    errors = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, r in errors:
        sys.stderr.write(f"--- {s}\n{r.stdout}{r.stderr}")
    if errors:
        raise RuntimeError("hipcc failed")
    if verbose:
        for s, _, r in results:
            sys.stderr.write(r.stderr)
    plain = [o for (_, a), (_, o, _) in zip(tasks, results) if not a]
    _link(plain, LIB)
    sanitized = {src: o for (src, a), (_, o, _) in zip(tasks, results) if a}
    _link([sanitized.get(src, o) for src, o in zip(SOURCES, plain)], LIB_ASAN)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
