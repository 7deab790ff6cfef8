"""The library's host code under AddressSanitizer (no GPU needed).

`liblz_asan.so` is built beside `liblz.so` with the host code of the API unit
(argument validation, context set-up, checkpoint parsing, spectrum arguments)
compiled with -fsanitize=address; device code is not instrumented.  A child
process with the sanitizer runtime preloaded drives every entry point down
the paths that run before any device work: malformed options and systems,
null arguments, bad checkpoint buffers, and the host-only launch plan over
grids and sizes from the smallest to the large cell's.  Any heap or stack overflow, use
after free or similar error aborts the child with the sanitizer's report.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_ASAN = os.path.join(ROOT, "paper_2111_06623_amd", "liblz_asan.so")


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


CHILD = textwrap.dedent(r"""
    import ctypes, sys
    sys.path.insert(0, sys.argv[2])
    import numpy as np
    import paper_2111_06623_amd as lz
    from synth import config_system

    lib = ctypes.CDLL(sys.argv[1])
    lib.lz_last_error.restype = ctypes.c_char_p
    vp = ctypes.c_void_p
    ERR_ARG = lz.LZ_ERR_ARG

    def expect(st, word=None):
        assert st == ERR_ARG, (st, lib.lz_last_error())
        msg = lib.lz_last_error().decode()
        assert msg and (word is None or word in msg), msg

    sysarr, keep = lz.make_system(config_system("micro"))
    out = vp()
    base = dict(prec=lz.LZ_FP64, approx=0, max_steps=8)
    bad = [dict(prec=7), dict(max_steps=0), dict(autotune=2), dict(algorithm=5), dict(streams=65),
           dict(projector_gemm=9), dict(density_group_bands=-1), dict(projector_chunk=96),
           dict(fft_planes=3), dict(batched=2), dict(approx=9)]
    for b in bad:
        opt = lz.LzOptions(**{**base, **b})
        expect(lib.lz_init(ctypes.byref(sysarr), 1, ctypes.byref(opt), 0, None, ctypes.byref(out)))
        assert not out.value
    opt = lz.LzOptions(**base)
    expect(lib.lz_init(None, 1, ctypes.byref(opt), 0, None, ctypes.byref(out)))
    expect(lib.lz_init(ctypes.byref(sysarr), 0, ctypes.byref(opt), 0, None, ctypes.byref(out)))
    expect(lib.lz_ground_state(None, 4, ctypes.c_double(1e-9), 10, 0, None, None, None, None, None))
    expect(lib.lz_ground_density(None, 1, 0, None, None, None))
    w = np.linspace(0.0, 1.0, 8)
    res = np.zeros(16)
    for f in (lib.lz_spectrum_ext, lib.lz_spectrum_ext_noalloc):
        expect(f(None, 0, 4, 4, 0, w.ctypes.data_as(vp), 8, ctypes.c_double(0.01),
                 res.ctypes.data_as(vp), res.ctypes.data_as(vp), res.ctypes.data_as(vp)))
    junk = ctypes.create_string_buffer(b"\x07" * 4096)
    n = ctypes.c_uint64()
    expect(lib.lz_checkpoint_load(None, 0, junk, ctypes.c_uint64(4096)))
    expect(lib.lz_checkpoint_size(None, 0, ctypes.byref(n)))
    expect(lib.lz_step(None, 1, None))
    plan = (ctypes.c_int32 * 15)()
    for n in (2, 12, 24, 40, 48, 72, 96):
        for prec in (0, 1, 2):
            for sizes in ((1, 1, 1, 0, 0), (16, 8, 6500, 32, 768), (128, 4, 51443, 256, 256)):
                assert lib.lz_launch_plan(n, prec, *sizes, plan) == lz.LZ_OK, lib.lz_last_error()
    expect(lib.lz_launch_plan(97, 0, 4, 1, 100, 0, 0, plan))
    assert lib.lz_free(None) == lz.LZ_OK
    print("asan-host-ok", flush=True)
""")


@pytest.mark.skipif(not os.path.exists(LIB_ASAN) or _asan_runtime() is None,
                    reason="the sanitized host library or the sanitizer runtime is missing")
def test_host_entry_points_under_address_sanitizer():
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD, LIB_ASAN, ROOT], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "asan-host-ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
