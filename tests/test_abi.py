"""The C ABI library loads on a machine without a GPU and exports every entry
point include/lz.h declares; argument checks that precede any device call
report LZ_ERR_ARG."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2111_06623_amd", "liblz.so")


def _declared():
    with open(os.path.join(ROOT, "include", "lz.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\S.*?\b(lz_[a-z_]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_four_core_calls():
    names = _declared()
    for n in ("lz_init", "lz_apply_liouvillian", "lz_step", "lz_spectrum"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_rejected_before_device_work():
    import paper_2111_06623_amd as lz
    lib = lz.load()
    out = ctypes.c_void_p()
    assert lib.lz_init(None, 1, None, 0, None, ctypes.byref(out)) == lz.LZ_ERR_ARG
    assert out.value is None
    assert "null" in lz.lz_last_error()
    assert lib.lz_step(None, 1, None) == lz.LZ_ERR_ARG
    assert lib.lz_free(None) == lz.LZ_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_unknown_precision_rejected_before_device_work():
    import paper_2111_06623_amd as lz
    from synth import config_system
    lib = lz.load()
    sysarr, keep = lz.make_system(config_system("micro"))
    opt = lz.LzOptions(3, 0, 8, 0, 0)
    out = ctypes.c_void_p()
    assert lib.lz_init(ctypes.byref(sysarr), 1, ctypes.byref(opt), 0, None,
                       ctypes.byref(out)) == lz.LZ_ERR_ARG
    assert "precision" in lz.lz_last_error()


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2111_06623_amd as lz
    with pytest.raises(ImportError):
        lz.load(str(tmp_path / "missing.so"))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_unknown_algorithm_rejected_before_device_work():
    import paper_2111_06623_amd as lz
    from synth import config_system
    lib = lz.load()
    sysarr, keep = lz.make_system(config_system("micro"))
    opt = lz.LzOptions(lz.LZ_FP64, 0, 8, 0, 0, 7)
    out = ctypes.c_void_p()
    assert lib.lz_init(ctypes.byref(sysarr), 1, ctypes.byref(opt), 0, None,
                       ctypes.byref(out)) == lz.LZ_ERR_ARG
    assert "algorithm" in lz.lz_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_stream_count_checked_before_device_work():
    import paper_2111_06623_amd as lz
    from synth import config_system
    lib = lz.load()
    sysarr, keep = lz.make_system(config_system("micro"))
    opt = lz.LzOptions(lz.LZ_FP64, 0, 8, 0, 0, 0, 65)
    out = ctypes.c_void_p()
    assert lib.lz_init(ctypes.byref(sysarr), 1, ctypes.byref(opt), 0, None,
                       ctypes.byref(out)) == lz.LZ_ERR_ARG
    assert "streams" in lz.lz_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_autotune_flag_checked_before_device_work():
    import paper_2111_06623_amd as lz
    from synth import config_system
    lib = lz.load()
    sysarr, keep = lz.make_system(config_system("micro"))
    opt = lz.LzOptions(lz.LZ_FP64, 0, 8, 0, 2)
    out = ctypes.c_void_p()
    assert lib.lz_init(ctypes.byref(sysarr), 1, ctypes.byref(opt), 0, None,
                       ctypes.byref(out)) == lz.LZ_ERR_ARG
    assert "autotune" in lz.lz_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_ground_state_arguments_checked_before_device_work():
    import paper_2111_06623_amd as lz
    lib = lz.load()
    assert lib.lz_ground_state(None, 4, 1e-9, 10, 0, None, None, None, None, None) == lz.LZ_ERR_ARG
    assert "null" in lz.lz_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("field,value,word", [("density_group_bands", -1, "density_group_bands"),
                                              ("projector_chunk", 96, "projector_chunk"),
                                              ("fft_planes", 3, "fft_planes"),
                                              ("batched", 2, "batched")])
def test_fixed_launch_parameters_checked_before_device_work(field, value, word):
    import paper_2111_06623_amd as lz
    from synth import config_system
    lib = lz.load()
    sysarr, keep = lz.make_system(config_system("micro"))
    opt = lz.LzOptions(lz.LZ_FP64, 0, 8, 0, 0, 0, 0, 0)
    setattr(opt, field, value)
    out = ctypes.c_void_p()
    assert lib.lz_init(ctypes.byref(sysarr), 1, ctypes.byref(opt), 0, None,
                       ctypes.byref(out)) == lz.LZ_ERR_ARG
    assert word in lz.lz_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_noalloc_spectrum_checks_arguments_before_device_work():
    import paper_2111_06623_amd as lz
    lib = lz.load()
    assert lib.lz_spectrum_ext_noalloc(None, 0, 1, 1, 0, None, 1, 0.01, None, None,
                                       None) == lz.LZ_ERR_ARG
