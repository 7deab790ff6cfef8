"""Build the HIP library (gfx950) in-tree: paper_2111_06623_amd/liblz.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/lz_kernels.hip", "csrc/lz_api.hip"]
LIB = os.path.join(HERE, "liblz.so")


def hipcc_cmd(out=LIB, extra=()):
    return ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # no packed-fp32 instructions anywhere in the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result",
            *extra, "-o", out] + [os.path.join(HERE, s) for s in SOURCES]


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    r = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
