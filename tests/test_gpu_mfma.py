"""Projector products on the matrix cores (MFMA) against the oracle: forced
on the small cells (so that tiles are mostly padding: ragged rows, bands and
plane waves), chosen automatically on batched-workload members with many
bands, and through the recursion (pseudo-Hermitian and non-Hermitian).
Tolerances as for the vector-ALU path: FP64 applications 1e-12 relative to
the largest output element, FP32 2e-5; Lanczos beta 1e-10 (FP64)."""
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


def _apply(ctx, s, dt, seed=11):
    p = torch.from_numpy(random_batch(s, seed)).to(device="cuda", dtype=dt)
    q = torch.from_numpy(random_batch(s, seed + 1)).to(device="cuda", dtype=dt)
    qo = torch.zeros_like(p)
    po = torch.zeros_like(p)
    ctx.apply_liouvillian(q, p, qo, po)
    torch.cuda.synchronize()
    return qo.cpu().numpy(), po.cpu().numpy()


@pytest.mark.parametrize("name", ["micro", "cfg1", "cfg2lo"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_forced_mfma_apply_matches_oracle(name, prec, tol):
    lz = _lz()
    s = config_system(name)
    print(f"[mfma apply] {name} {prec}", flush=True)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    ctx = lz.lz_init(s, prec=prec, max_steps=4, projector_gemm="mfma")
    qo, po = _apply(ctx, s, dt)
    L = Liouvillian(s)
    assert _rel(qo, L.apply_D(random_batch(s, 11))) < tol
    assert _rel(po, L.apply_DK(random_batch(s, 12))) < tol
    ctx.free()


def test_mfma_and_vector_alu_agree_on_cfg2():
    """The 48^3 benchmark cell in FP64 with both product paths: the same
    application to rounding (1e-13)."""
    lz = _lz()
    s = config_system("cfg2")
    out = []
    for g in ("valu", "mfma"):
        ctx = lz.lz_init(s, prec="fp64", max_steps=4, projector_gemm=g)
        out.append(_apply(ctx, s, torch.complex128))
        ctx.free()
    assert _rel(out[1][0], out[0][0]) < 1e-13
    assert _rel(out[1][1], out[0][1]) < 1e-13


@pytest.mark.parametrize("grid,nbnd,nk", [(48, 48, 2), (32, 40, 1)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_many_band_members_take_mfma(grid, nbnd, nk, prec, tol):
    """Members of the batched workload with many bands (projector rows
    nbnd + 2 nbnd, bands not a multiple of the 64-wide tile)."""
    lz = _lz()
    s = config_system("uneven", index=7, grid=grid, nbnd=nbnd, nk=nk)
    print(f"[mfma auto] {grid}^3 nbnd={nbnd} nk={nk} {prec}", flush=True)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    ctx = lz.lz_init(s, prec=prec, max_steps=4)
    qo, po = _apply(ctx, s, dt, seed=21)
    L = Liouvillian(s)
    assert _rel(qo, L.apply_D(random_batch(s, 21))) < tol
    assert _rel(po, L.apply_DK(random_batch(s, 22))) < tol
    ctx.free()


@pytest.mark.parametrize("alg", ["ph", "nh"])
def test_forced_mfma_recursion_matches_oracle(alg):
    lz = _lz()
    s = config_system("cfg2lo")
    ctx = lz.lz_init(s, prec="fp64", max_steps=64, projector_gemm="mfma", algorithm=alg)
    done, st = ctx.step(50)
    ref = lanczos.run(Liouvillian(s), 50, variant=alg)
    assert done == ref.steps == 50 and st == lz.LZ_OK
    beta, gamma, z = ctx.coefficients()
    assert np.max(np.abs(beta - ref.beta) / ref.beta) < 1e-10
    assert np.max(np.abs(gamma - ref.gamma) / np.abs(ref.gamma)) < 1e-10
    assert np.abs(z - ref.z).max() < 1e-10 * np.abs(ref.z).max()
    ctx.free()


@pytest.mark.parametrize("name", ["micro", "cfg1", "cfg2lo"])
def test_split_bf16_apply_matches_oracle(name):
    """Split-bf16 projector products: each real product carries about 2^-16
    relative error (the dropped lo*lo term and the bf16 rounding of lo), on
    terms no larger than the output: 5e-5 of the largest output element
    (measured 1e-5 at most, against 2e-7 in FP32)."""
    lz = _lz()
    s = config_system(name)
    ctx = lz.lz_init(s, prec="splitbf16", max_steps=4)
    qo, po = _apply(ctx, s, torch.complex64)
    L = Liouvillian(s)
    e = (_rel(qo, L.apply_D(random_batch(s, 11))), _rel(po, L.apply_DK(random_batch(s, 12))))
    print(f"[split-bf16 apply] {name} {e[0]:.2e} {e[1]:.2e}", flush=True)
    assert max(e) < 5e-5
    ctx.free()


def test_split_bf16_recursion_tracks_oracle():
    """cfg2lo, 150 steps: beta within 2e-5 over the first 50 steps and the
    loss function within the 1e-4 gate of the mixed path (measured 3.8e-6
    and 2.7e-5)."""
    lz = _lz()
    from oracle import spectrum
    s = config_system("cfg2lo")
    ctx = lz.lz_init(s, prec="splitbf16", max_steps=152)
    done, _ = ctx.step(150)
    assert done == 150
    beta, _, _ = ctx.coefficients()
    L = Liouvillian(s)
    ref = lanczos.run(L, 150)
    assert np.max(np.abs(beta[:50] - ref.beta[:50]) / ref.beta[:50]) < 2e-5
    om = np.linspace(0.0, 2.0, 2000)
    _, _, loss = ctx.spectrum(om, 0.01)
    _, _, loss_r, _ = spectrum.spectrum(ref.beta, ref.z, om, 0.01, L.cell.omega, L.Q)
    floor = 1e-6 * np.abs(loss_r).max()
    assert np.max(np.abs(loss - loss_r) / np.maximum(np.abs(loss_r), floor)) < 1e-4
    ctx.free()
