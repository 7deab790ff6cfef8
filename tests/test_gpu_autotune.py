"""Autotuned launch configurations: whatever the tuner picks (projector
products on the vector ALU or the matrix cores, density band-group size),
results meet the oracle's tolerances, and a path asked for is kept."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import lanczos  # noqa: E402
from oracle.liouvillian import Liouvillian  # noqa: E402
from synth import config_system, random_batch  # noqa: E402


def _lz():
    import paper_2111_06623_amd as lz
    lz.load()
    return lz


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name,prec,tol,kw", [("cfg2lo", "fp64", 1e-12, {}),
                                              ("cfg1", "fp32", 2e-5, {}),
                                              ("uneven", "fp32", 2e-5,
                                               dict(index=7, grid=48, nbnd=48, nk=2))])
def test_autotuned_apply_matches_oracle(name, prec, tol, kw):
    lz = _lz()
    s = config_system(name, **kw)
    ctx = lz.lz_init(s, prec=prec, max_steps=4, autotune=True)
    gemm, bands, chunks, planes = ctx.tuning()
    print(f"[autotune] {name} {prec}: {gemm} groups of {bands} bands, {chunks} chunks, "
          f"{planes} planes", flush=True)
    assert gemm in ("valu", "mfma") and bands >= 1 and chunks >= 1 and planes in ("registers", "lds")
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    p = torch.from_numpy(random_batch(s, 5)).to("cuda", dt)
    q = torch.from_numpy(random_batch(s, 6)).to("cuda", dt)
    qo, po = torch.zeros_like(p), torch.zeros_like(p)
    ctx.apply_liouvillian(q, p, qo, po)
    torch.cuda.synchronize()
    L = Liouvillian(s)
    assert _rel(qo.cpu().numpy(), L.apply_D(random_batch(s, 5))) < tol
    assert _rel(po.cpu().numpy(), L.apply_DK(random_batch(s, 6))) < tol
    ctx.free()


@pytest.mark.parametrize("alg", ["ph", "nh"])
def test_autotuned_recursion_matches_oracle(alg):
    lz = _lz()
    s = config_system("cfg2lo")
    ctx = lz.lz_init(s, prec="fp64", max_steps=64, autotune=True, algorithm=alg)
    done, _ = ctx.step(50)
    ref = lanczos.run(Liouvillian(s), 50, variant=alg)
    assert done == ref.steps == 50
    beta, gamma, z = ctx.coefficients()
    assert np.max(np.abs(beta - ref.beta) / ref.beta) < 1e-10
    assert np.abs(z - ref.z).max() < 1e-10 * np.abs(ref.z).max()
    ctx.free()


def test_asked_for_path_is_kept():
    lz = _lz()
    s = config_system("cfg2lo")
    for g in ("valu", "mfma"):
        ctx = lz.lz_init(s, prec="fp32", max_steps=4, autotune=True, projector_gemm=g)
        assert ctx.tuning()[0] == g
        ctx.free()
    ctx = lz.lz_init(s, prec="fp32", max_steps=4)
    assert ctx.tuning()[0] == "valu"   # the heuristic for 16 bands
    ctx.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_launch_plan_matches_the_context(prec):
    """lz_launch_plan (the host helpers alone) gives the launch parameters an
    lz_init without autotuning takes on the benchmark cell: the density
    band groups (for the LDS form, the round rule at some number of resident
    blocks per compute unit, which the device decides) and the dot chunks."""
    lz = _lz()
    s = config_system("cfg2")
    ctx = lz.lz_init(s, prec=prec, max_steps=4, autotune=False)
    gemm, bands, chunks, planes = ctx.tuning()
    ctx.free()
    nbnd, nks, npwx, nproj = int(s.nbnd), int(s.nks), int(s.nl_kq.shape[1]), int(s.nproj)
    n = int(s.nr[0])
    plan0 = lz.lz_launch_plan(n, prec, nbnd, nks, npwx, nproj, 0)
    assert chunks == (plan0["valu_nchunk"] if gemm == "valu" else plan0["mfma_nchunk"])
    if plan0["reg_plane"]:
        assert planes == "registers" and bands == plan0["gsize"]
    else:
        # LDS passes: the round rule at 1 to 8 resident blocks per compute unit
        options = {lz.lz_launch_plan(n, prec, nbnd, nks, npwx, nproj, 256 * b)["gsize"]
                   for b in range(1, 9)}
        assert bands in options, (bands, options)
