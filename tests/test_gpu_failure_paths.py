"""Failure paths of the C ABI on the GPU: an indefinite metric (a system
without a gap) ends the recursion with LZ_ERR_NOT_PD where the oracle's
recursion reports not_pd (Sec. 2.5: the pseudo-Hermitian recursion needs a
positive-definite metric diag(D+K, D)); checkpoints of another operator of
the same shape are refused; non-cubic grids are refused."""
import copy

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import lanczos  # noqa: E402
from oracle.liouvillian import Liouvillian  # noqa: E402
from synth import config_system, q_sweep  # noqa: E402


def _lz():
    import paper_2111_06623_amd as lz
    lz.load()
    return lz


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gapless_system_stops_with_not_pd(prec):
    lz = _lz()
    s = config_system("gapless")
    print(f"[not_pd] gapless {prec}", flush=True)
    ref = lanczos.run(Liouvillian(s), 300)
    assert ref.status == "not_pd"
    ctx = lz.lz_init(s, prec=prec, max_steps=300)
    with pytest.raises(lz.LzError) as e:
        ctx.step(300)
    assert e.value.status == lz.LZ_ERR_NOT_PD
    done, status = ctx.state()
    assert status == lz.LZ_ERR_NOT_PD
    if prec == "fp64":
        # the same step fails on both sides, and the coefficients before it agree
        assert done == ref.steps
        beta, _, z = ctx.coefficients()
        assert np.max(np.abs(beta - ref.beta) / ref.beta) < 1e-10
    else:
        assert abs(done - ref.steps) <= 2
    # a stopped recursion takes no further steps and keeps its status
    with pytest.raises(lz.LzError) as e:
        ctx.step(5)
    assert e.value.status == lz.LZ_ERR_NOT_PD and ctx.state()[0] == done
    ctx.free()


def test_checkpoint_of_a_sibling_q_is_refused():
    """Two members of a q sweep have the same shapes (grid, k-points, bands,
    padded stride) but different operators: the fingerprint refuses the load."""
    lz = _lz()
    a_sys, b_sys = q_sweep("cfg2lo")[:2]
    assert a_sys.npwx == b_sys.npwx and a_sys.nks == b_sys.nks
    a = lz.lz_init(a_sys, prec="fp64", max_steps=32)
    a.step(11)
    blob = a.checkpoint()
    b = lz.lz_init(b_sys, prec="fp64", max_steps=32)
    with pytest.raises(lz.LzError) as e:
        b.restore(blob)
    assert e.value.status == lz.LZ_ERR_ARG and "another system" in str(e.value)
    # the same operator in a fresh context loads and continues
    c = lz.lz_init(a_sys, prec="fp64", max_steps=32)
    c.restore(blob)
    assert c.state()[0] == 11
    for x in (a, b, c):
        x.free()


def test_checkpoint_of_another_level_of_theory_is_refused():
    lz = _lz()
    s = config_system("cfg1")
    rpa = lz.lz_init(s, prec="fp64", approx="rpa", max_steps=32)
    rpa.step(9)
    blob = rpa.checkpoint()
    tddft = lz.lz_init(s, prec="fp64", approx="tddft", max_steps=32)
    with pytest.raises(lz.LzError) as e:
        tddft.restore(blob)
    assert e.value.status == lz.LZ_ERR_ARG and "level of theory" in str(e.value)
    rpa.free()
    tddft.free()


def test_non_cubic_grid_is_refused():
    lz = _lz()
    s = copy.copy(config_system("micro"))
    s.nr = np.array([12, 12, 15], dtype=np.int32)
    with pytest.raises(lz.LzError) as e:
        lz.lz_init(s, prec="fp64", max_steps=4)
    assert e.value.status == lz.LZ_ERR_ARG and "cubic" in str(e.value)
