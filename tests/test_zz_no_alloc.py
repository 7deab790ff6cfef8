"""The allocation-free spectrum entry point (lz_spectrum_ext_noalloc) against
lz_spectrum_ext on the same context, through the C ABI: the two share the
spectrum kernel, so the results agree bit for bit (the test asks for 1e-14
relative, within the 1e-12 bar of the FP64 path), on two calls in a row, the
second with a smaller frequency grid, with and without extrapolation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import config_system  # noqa: E402


def _lz():
    import paper_2111_06623_amd as lz
    lz.load()
    return lz


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("scheme,m_total", [("no", None), ("osc", 5000), ("constant", 5000)])
def test_noalloc_spectrum_equals_allocating_one(scheme, m_total):
    lz = _lz()
    s = config_system("cfg1")
    print(f"[noalloc] cfg1 {scheme}", flush=True)
    ctx = lz.lz_init(s, prec="fp64", max_steps=120)
    ctx.step(120)
    for n in (3000, 257):
        om = np.linspace(0.0, 2.0, n)
        ref = ctx.spectrum(om, 0.01, m=120, m_total=m_total, extrapolation=scheme)
        got = ctx.spectrum_noalloc(om, 0.01, m=120, m_total=m_total, extrapolation=scheme)
        for a, b in zip(got, ref):
            assert _rel(a, b) <= 1e-14
    with pytest.raises(lz.LzError) as e:
        ctx.spectrum_noalloc(np.zeros(65537), 0.01, m=120)
    assert e.value.status == lz.LZ_ERR_ARG
    ctx.free()


def test_noalloc_spectrum_on_two_contexts():
    """Two contexts on one device, called one after the other, each see their
    own coefficients through the shared staging area."""
    lz = _lz()
    a = lz.lz_init(config_system("cfg1"), prec="fp64", max_steps=60)
    b = lz.lz_init(config_system("micro"), prec="fp64", max_steps=60)
    a.step(60)
    b.step(40)
    om = np.linspace(0.0, 2.0, 1000)
    ra, rb = a.spectrum(om, 0.02), b.spectrum(om, 0.02)
    ga, gb = a.spectrum_noalloc(om, 0.02), b.spectrum_noalloc(om[:500], 0.02)
    assert _rel(ga[0], ra[0]) <= 1e-14 and _rel(gb[0], rb[0][:500]) <= 1e-14
    a.free()
    b.free()
