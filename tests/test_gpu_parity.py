"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the
same seeded inputs.  Tolerances (FP64 path): operator applications 1e-12
relative to the largest output element; Lanczos beta/gamma 1e-10 relative and
z 1e-10 of max|z| over the first 50 steps; loss function 1e-6 relative with
the denominator floored at 1e-6 of its maximum."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import lanczos, spectrum  # noqa: E402
from oracle.liouvillian import Liouvillian  # noqa: E402
from synth import config_system, random_batch  # noqa: E402


def _lz():
    import paper_2111_06623_amd as lz
    lz.load()
    return lz


def _to_dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _loss_err(loss, ref):
    floor = 1e-6 * np.abs(ref).max()
    return np.max(np.abs(loss - ref) / np.maximum(np.abs(ref), floor))


CASES = [("micro", {}), ("cfg1", {}), ("cfg2lo", {}), ("free", {})]


@pytest.mark.parametrize("name,kw", CASES)
@pytest.mark.parametrize("approx", ["tddft", "rpa", "ipa"])
def test_apply_liouvillian_matches_oracle(name, kw, approx):
    lz = _lz()
    s = config_system(name, **kw)
    print(f"[apply] {name} {approx} nr={tuple(s.nr)} nks={s.nks} nbnd={s.nbnd}", flush=True)
    ctx = lz.lz_init(s, prec="fp64", approx=approx, max_steps=8)
    L = Liouvillian(s, approx)
    p = random_batch(s, 11)
    q = random_batch(s, 12)
    qo = torch.zeros_like(_to_dev(p))
    po = torch.zeros_like(qo)
    ctx.apply_liouvillian(_to_dev(q), _to_dev(p), qo, po)
    torch.cuda.synchronize()
    d_ref = L.apply_D(p)
    dk_ref = L.apply_DK(q)
    assert _rel(qo.cpu().numpy(), d_ref) < 1e-12
    assert _rel(po.cpu().numpy(), dk_ref) < 1e-12
    ctx.free()


@pytest.mark.parametrize("name", ["micro", "cfg1", "cfg2lo", "free"])
def test_rhs_matches_oracle(name):
    lz = _lz()
    s = config_system(name)
    ctx = lz.lz_init(s, prec="fp64", max_steps=4)
    y = ctx.rhs().cpu().numpy()
    assert _rel(y, Liouvillian(s).rhs()) < 1e-12
    ctx.free()


@pytest.mark.parametrize("name,approx", [("cfg1", "tddft"), ("micro", "tddft"), ("micro", "rpa"),
                                         ("micro", "ipa"), ("cfg2lo", "tddft")])
def test_lanczos_coefficients_first_50_steps(name, approx):
    lz = _lz()
    s = config_system(name)
    print(f"[lanczos] {name} {approx}", flush=True)
    ctx = lz.lz_init(s, prec="fp64", approx=approx, max_steps=64)
    done, st = ctx.step(50)
    ref = lanczos.run(Liouvillian(s, approx), 50)
    assert done == ref.steps == 50 and st == lz.LZ_OK
    beta, gamma, z = ctx.coefficients()
    assert np.max(np.abs(beta - ref.beta) / ref.beta) < 1e-10
    assert np.array_equal(beta, gamma)
    assert np.abs(z - ref.z).max() < 1e-10 * np.abs(ref.z).max()
    ctx.free()


def test_spectrum_cfg1_full_run():
    """cfg1: 200 steps, 2000 frequencies in [0, 2] Ha, eta = 0.01 Ha."""
    lz = _lz()
    s = config_system("cfg1")
    ctx = lz.lz_init(s, prec="fp64", max_steps=200)
    done, _ = ctx.step(200)
    assert done == 200
    om = np.linspace(0.0, 2.0, 2000)
    chi, einv, loss = ctx.spectrum(om, 0.01)
    L = Liouvillian(s)
    ref = lanczos.run(L, 200)
    chi_r, einv_r, loss_r, _ = spectrum.spectrum(ref.beta, ref.z, om, 0.01, L.cell.omega, L.Q)
    assert _loss_err(loss, loss_r) < 1e-6
    assert _rel(chi, chi_r) < 1e-6
    # the spectrum kernel on the oracle's own coefficients isolates the solve
    beta, _, z = ctx.coefficients()
    chi_same = spectrum.chi_from_coefficients(beta, z, om, 0.01, L.cell.omega)
    assert _rel(chi, chi_same) < 1e-12
    ctx.free()


def test_free_electron_lucky_breakdown_on_gpu(free):
    lz = _lz()
    ctx = lz.lz_init(free, prec="fp64", max_steps=40)
    done, st = ctx.step(30)
    ref = lanczos.run(Liouvillian(free), 30)
    assert st == lz.LZ_BREAKDOWN and ref.status == "breakdown"
    assert done == ref.steps
    beta, _, z = ctx.coefficients()
    assert np.max(np.abs(beta - ref.beta) / ref.beta) < 1e-10
    ctx.free()


def test_pauli_blocked_rhs_gives_zero_spectrum():
    lz = _lz()
    s = config_system("free", g0=(0, 0, 0))
    ctx = lz.lz_init(s, prec="fp64", max_steps=8)
    done, st = ctx.step(5)
    assert st == lz.LZ_BREAKDOWN and done == 0
    chi, einv, loss = ctx.spectrum(np.linspace(0, 1, 11), 0.02, m=0)
    assert np.all(chi == 0) and np.all(loss == 0)
    ctx.free()


def test_recursion_is_deterministic(cfg1):
    lz = _lz()
    out = []
    for _ in range(2):
        ctx = lz.lz_init(cfg1, prec="fp64", max_steps=40)
        ctx.step(40)
        out.append(ctx.coefficients())
        ctx.free()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][2], out[1][2])


def test_steps_in_pieces_equal_one_call(cfg1):
    lz = _lz()
    a = lz.lz_init(cfg1, prec="fp64", max_steps=30)
    a.step(30)
    b = lz.lz_init(cfg1, prec="fp64", max_steps=30)
    for n in (1, 2, 7, 20):
        b.step(n)
    assert np.array_equal(a.coefficients()[0], b.coefficients()[0])
    with pytest.raises(lz.LzError) as e:
        b.step(1)
    assert e.value.status == lz.LZ_ERR_STATE
    a.free()
    b.free()


def test_argument_errors_are_reported(cfg1):
    lz = _lz()
    import copy
    bad = copy.copy(cfg1)
    bad.wk = np.array([0.5])
    with pytest.raises(lz.LzError) as e:
        lz.lz_init(bad)
    assert e.value.status == lz.LZ_ERR_ARG and "weights" in str(e.value)
    bad = copy.copy(cfg1)
    bad.nr = np.array([24, 24, 7 * 3])
    with pytest.raises(lz.LzError) as e:
        lz.lz_init(bad)
    assert e.value.status == lz.LZ_ERR_ARG
    ctx = lz.lz_init(cfg1, max_steps=10)
    ctx.step(10)
    with pytest.raises(lz.LzError) as e:
        ctx.spectrum(np.zeros(3), 0.01, m=11)
    assert e.value.status == lz.LZ_ERR_STATE
    ctx.free()


@pytest.fixture(scope="module")
def cfg2_oracle_50():
    """The oracle's first 50 steps on the benchmark workload (48^3, 16 bands, 8 k)."""
    s = config_system("cfg2")
    print("[cfg2] oracle", flush=True)
    return s, lanczos.run(Liouvillian(s), 50)


@pytest.mark.slow
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_cfg2_first_50_steps_full_size(cfg2_oracle_50, prec, tol):
    """The benchmark workload at its full size, in both precisions: FP64 to
    the parity bar, the mixed path (FP32 bulk, FP64 scalars) to 2e-5."""
    lz = _lz()
    s, ref = cfg2_oracle_50
    print(f"[cfg2] {prec}", flush=True)
    ctx = lz.lz_init(s, prec=prec, max_steps=64)
    done, st = ctx.step(50)
    assert done == 50
    beta, _, z = ctx.coefficients()
    assert np.max(np.abs(beta - ref.beta) / ref.beta) < tol
    assert np.abs(z - ref.z).max() < tol * np.abs(ref.z).max()
    ctx.free()


@pytest.mark.parametrize("name", ["cfg1", "cfg2lo", "cfg2"])
@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("splitbf16", 5e-5)])
def test_apply_liouvillian_fp32_matches_oracle(name, prec, tol):
    """Single-precision applications (the kernels of the mixed path, at the
    benchmark grid for cfg2; projector products on the vector ALU or as split
    bf16 products on the matrix cores) against the FP64 oracle: 2e-5 (5e-5
    for split bf16) of the largest output element."""
    lz = _lz()
    s = config_system(name)
    print(f"[apply32] {name} {prec}", flush=True)
    ctx = lz.lz_init(s, prec=prec, max_steps=8)
    L = Liouvillian(s)
    p = random_batch(s, 21)
    q = random_batch(s, 22)
    qo = torch.zeros(p.shape, dtype=torch.complex64, device="cuda")
    po = torch.zeros_like(qo)
    ctx.apply_liouvillian(_to_dev(q, torch.complex64), _to_dev(p, torch.complex64), qo, po)
    torch.cuda.synchronize()
    assert _rel(qo.cpu().numpy(), L.apply_D(p)) < tol
    assert _rel(po.cpu().numpy(), L.apply_DK(q)) < tol
    ctx.free()


@pytest.fixture(scope="module")
def cfg2_apply_ref():
    """The oracle's D p and (D+K) q on the 48^3 benchmark cell."""
    import oracle.pw as opw
    opw.FFT_WORKERS = min(len(__import__("os").sched_getaffinity(0)), 16)
    s = config_system("cfg2")
    print("[cfg2] oracle applications", flush=True)
    L = Liouvillian(s)
    p = random_batch(s, 61)
    q = random_batch(s, 62)
    return s, p, q, L.apply_D(p), L.apply_DK(q)


def _apply_case(lz, s, p, q, d_ref, dk_ref, prec, tol, **opts):
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    ctx = lz.lz_init(s, prec=prec, max_steps=4, **opts)
    qo = torch.zeros(p.shape, dtype=dt, device="cuda")
    po = torch.zeros_like(qo)
    ctx.apply_liouvillian(_to_dev(q, dt), _to_dev(p, dt), qo, po)
    torch.cuda.synchronize()
    tuning = ctx.tuning()
    assert _rel(qo.cpu().numpy(), d_ref) < tol
    assert _rel(po.cpu().numpy(), dk_ref) < tol
    ctx.free()
    return tuning


# every launch configuration the autotuner can pick, forced: density band
# groups of the heuristic size and twice it (4 takes the quad kernel on 48^2
# single-precision planes, 8 the line kernel), ragged groups (3, 5), and the
# three plane-wave chunks of the vector-ALU projector dot, and both schedules
# of the plane transforms (register lines / lane pairs, LDS Stockham passes)
@pytest.mark.parametrize("prec,tol,gsize,chunk,gemm,planes", [
    ("fp32", 2e-5, 4, 64, "valu", "registers"), ("fp32", 2e-5, 8, 64, "valu", "registers"),
    ("fp32", 2e-5, 3, 128, "valu", "registers"), ("fp32", 2e-5, 1, 256, "valu", "registers"),
    ("fp32", 2e-5, 16, 64, "mfma", "registers"), ("fp32", 2e-5, 5, 64, "mfma", "registers"),
    ("fp32", 2e-5, 6, 64, "valu", "lds"), ("fp32", 2e-5, 4, 64, "valu", "lds"),
    ("fp64", 1e-12, 6, 64, "valu", "registers"), ("fp64", 1e-12, 12, 128, "valu", "registers"),
    ("fp64", 1e-12, 5, 256, "valu", "registers"), ("fp64", 1e-12, 6, 64, "mfma", "registers"),
    ("fp64", 1e-12, 6, 64, "valu", "lds")])
def test_every_launch_candidate_on_the_benchmark_cell(cfg2_apply_ref, prec, tol, gsize, chunk, gemm,
                                                      planes):
    lz = _lz()
    s, p, q, d_ref, dk_ref = cfg2_apply_ref
    print(f"[candidate] cfg2 {prec} groups of {gsize}, chunk {chunk}, {gemm}, {planes} planes",
          flush=True)
    got = _apply_case(lz, s, p, q, d_ref, dk_ref, prec, tol, density_group_bands=gsize,
                      projector_chunk=chunk, projector_gemm=gemm, fft_planes=planes)
    assert got[0] == gemm and got[1] == gsize and got[3] == planes
    if gemm == "valu":
        assert got[2] == -(-int(s.npwx) // chunk)


def test_reset_restarts_the_recursion(cfg1):
    lz = _lz()
    ctx = lz.lz_init(cfg1, prec="fp64", max_steps=40)
    ctx.step(30)
    first = ctx.coefficients()
    ctx.reset()
    assert ctx.state()[0] == 0
    ctx.step(30)
    again = ctx.coefficients()
    assert np.array_equal(first[0], again[0]) and np.array_equal(first[2], again[2])
    ctx.free()


@pytest.mark.parametrize("name,steps", [("cfg1", 150), ("cfg2lo", 150)])
def test_mixed_precision_tracks_the_oracle(name, steps):
    """FP32 bulk with FP64 scalars: beta within 1e-5 over the first 50 steps and
    the loss function of the whole recursion within 1e-4 (floored)."""
    lz = _lz()
    s = config_system(name)
    ctx = lz.lz_init(s, prec="fp32", max_steps=steps + 2)
    done, _ = ctx.step(steps)
    assert done == steps
    beta, _, z = ctx.coefficients()
    L = Liouvillian(s)
    ref = lanczos.run(L, steps)
    assert np.max(np.abs(beta[:50] - ref.beta[:50]) / ref.beta[:50]) < 1e-5
    om = np.linspace(0.0, 2.0, 2000)
    _, _, loss = ctx.spectrum(om, 0.01)
    _, _, loss_r, _ = spectrum.spectrum(ref.beta, ref.z, om, 0.01, L.cell.omega, L.Q)
    assert _loss_err(loss, loss_r) < 1e-4
    ctx.free()


@pytest.mark.parametrize("name,prec", [("cfg1", "fp64"), ("cfg2lo", "fp32")])
def test_graph_replay_equals_eager(name, prec):
    """Pairs of steps replayed from a captured graph, interleaved with eager
    steps and with operator applications on the same context, give the
    coefficients of the eager recursion bit for bit, on every replay."""
    lz = _lz()
    s = config_system(name)
    eager = lz.lz_init(s, prec=prec, max_steps=64)
    eager.step(41)
    ref = eager.coefficients()
    eager.free()
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    p = _to_dev(random_batch(s, 3), dt)
    g = lz.lz_init(s, prec=prec, max_steps=64, use_graph=True)
    for rep in range(3):
        g.reset()
        for n in (1, 6, 3, 31):
            g.step(n)
            qo = torch.zeros_like(p)
            po = torch.zeros_like(p)
            g.apply_liouvillian(p, p, qo, po)
            torch.cuda.synchronize()
        got = g.coefficients()
        print(f"[graph] {name} {prec} replay {rep}", flush=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])
    g.free()


@pytest.fixture(scope="module")
def cfg5r_ref():
    """The large cell (96^3, 128 bands, 4 k, 256 projectors; random
    orthonormal orbitals) and the oracle's D p and (D+K) q on it."""
    import oracle.pw as opw
    opw.FFT_WORKERS = min(len(__import__("os").sched_getaffinity(0)), 16)
    s = config_system("cfg5r")
    print("[cfg5r] oracle", flush=True)
    L = Liouvillian(s)
    p = random_batch(s, 31)
    q = random_batch(s, 32)
    return s, p, q, L.apply_D(p), L.apply_DK(q)


@pytest.mark.slow
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5), ("splitbf16", 5e-5)])
def test_large_cell_apply_full_size(cfg5r_ref, prec, tol):
    """Every kernel at the large-cell size (general 96^3 transforms, projector
    products spanning several tiles) against the oracle."""
    lz = _lz()
    s, p, q, d_ref, dk_ref = cfg5r_ref
    print(f"[cfg5r] {prec}", flush=True)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    ctx = lz.lz_init(s, prec=prec, max_steps=4)
    qo = torch.zeros(p.shape, dtype=dt, device="cuda")
    po = torch.zeros_like(qo)
    ctx.apply_liouvillian(_to_dev(q, dt), _to_dev(p, dt), qo, po)
    torch.cuda.synchronize()
    assert _rel(qo.cpu().numpy(), d_ref) < tol
    assert _rel(po.cpu().numpy(), dk_ref) < tol
    ctx.free()


@pytest.mark.slow
@pytest.mark.parametrize("prec,tol,gsize", [("fp32", 2e-5, 16), ("fp32", 2e-5, 5),
                                            ("fp64", 1e-12, 16), ("fp64", 1e-12, 3)])
def test_large_cell_density_groups(cfg5r_ref, prec, tol, gsize):
    """The large cell with density band groups other than the heuristic 8
    (twice it, and ragged groups whose last one is shorter)."""
    lz = _lz()
    s, p, q, d_ref, dk_ref = cfg5r_ref
    print(f"[cfg5r] {prec} groups of {gsize}", flush=True)
    got = _apply_case(lz, s, p, q, d_ref, dk_ref, prec, tol, density_group_bands=gsize)
    assert got[1] == gsize


@pytest.mark.parametrize("grid,nbnd,nk", [(40, 8, 2), (72, 8, 1), (64, 16, 1), (48, 5, 1)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_uneven_grid_apply(grid, nbnd, nk, prec, tol):
    """Members of the batched workload: runtime-plan grids (40 = 8 x 5,
    72 = 8 x 9), the compile-time 64^3 grid, and a 48^3 member of five
    orbitals, whose density pass has a last band group of one (three idle
    lanes of each quad in single precision)."""
    lz = _lz()
    s = config_system("uneven", index=grid, grid=grid, nbnd=nbnd, nk=nk)
    print(f"[uneven] {grid} {prec}", flush=True)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    L = Liouvillian(s)
    p = random_batch(s, 41)
    q = random_batch(s, 42)
    ctx = lz.lz_init(s, prec=prec, max_steps=4)
    qo = torch.zeros(p.shape, dtype=dt, device="cuda")
    po = torch.zeros_like(qo)
    ctx.apply_liouvillian(_to_dev(q, dt), _to_dev(p, dt), qo, po)
    torch.cuda.synchronize()
    assert _rel(qo.cpu().numpy(), L.apply_D(p)) < tol
    assert _rel(po.cpu().numpy(), L.apply_DK(q)) < tol
    ctx.free()


def test_instances_in_one_context_match_single_contexts():
    """Three instances of different grids (24^3, 12^3, 32^3) in one context:
    every instance's recursion is bit for bit the one of a context of its
    own, and applications on the concatenated layout are the instances'."""
    lz = _lz()
    names = ["cfg1", "micro", "cfg2lo"]
    systems = [config_system(n) for n in names]
    single = []
    for s in systems:
        c = lz.lz_init(s, prec="fp64", max_steps=40)
        c.step(30)
        single.append(c.coefficients())
        c.free()
    ctx = lz.lz_init(systems, prec="fp64", max_steps=40)
    done, st = ctx.step(30)
    assert done == 30
    for i in range(3):
        beta, _, z = ctx.coefficients(inst=i)
        assert np.array_equal(beta, single[i][0]) and np.array_equal(z, single[i][2])
    ps = [random_batch(s, 51) for s in systems]
    flat = np.concatenate([x.ravel() for x in ps])
    qo = torch.zeros(flat.shape, dtype=torch.complex128, device="cuda")
    po = torch.zeros_like(qo)
    ctx.apply_liouvillian(_to_dev(flat), _to_dev(flat), qo, po)
    torch.cuda.synchronize()
    off = 0
    for s, x in zip(systems, ps):
        L = Liouvillian(s)
        n = x.size
        assert _rel(qo.cpu().numpy()[off:off + n].reshape(x.shape), L.apply_D(x)) < 1e-12
        assert _rel(po.cpu().numpy()[off:off + n].reshape(x.shape), L.apply_DK(x)) < 1e-12
        off += n
    ctx.free()


@pytest.mark.parametrize("scheme", ["constant", "osc"])
def test_extrapolated_spectrum_matches_oracle(scheme):
    """cfg1, 200 computed steps extended to 20000 (the paper's use of the
    extrapolation): the device sweep against the oracle's banded solve on the
    same coefficients, and against the oracle's own recursion."""
    lz = _lz()
    s = config_system("cfg1")
    ctx = lz.lz_init(s, prec="fp64", max_steps=200)
    ctx.step(200)
    om = np.linspace(0.0, 2.0, 400)
    chi, _, loss = ctx.spectrum(om, 0.01, m=200, m_total=20000, extrapolation=scheme)
    L = Liouvillian(s)
    beta, _, z = ctx.coefficients()
    same = spectrum.spectrum(beta, z, om, 0.01, L.cell.omega, L.Q, m=200, m_total=20000,
                             scheme=scheme)
    assert _rel(chi, same[0]) < 1e-10
    ref = lanczos.run(L, 200)
    chi_r, _, loss_r, _ = spectrum.spectrum(ref.beta, ref.z, om, 0.01, L.cell.omega, L.Q, m=200,
                                            m_total=20000, scheme=scheme)
    assert _loss_err(loss, loss_r) < 1e-6
    plain, _, _ = ctx.spectrum(om, 0.01, m=200)
    assert _rel(chi, plain) > 1e-8  # the tail changes the spectrum
    with pytest.raises(lz.LzError) as e:
        ctx.spectrum(om, 0.01, m=200, m_total=100, extrapolation=scheme)
    assert e.value.status == lz.LZ_ERR_ARG
    ctx.free()


@pytest.mark.parametrize("name,prec", [("cfg1", "fp64"), ("cfg2lo", "fp32")])
def test_checkpoint_restart_continues_bit_for_bit(name, prec):
    """30 steps, checkpoint, 20 more in the same context; a fresh context
    loaded from the checkpoint runs the same 20 steps to the same bits."""
    lz = _lz()
    s = config_system(name)
    a = lz.lz_init(s, prec=prec, max_steps=64)
    a.step(31)
    blob = a.checkpoint()
    a.step(20)
    ref = a.coefficients()
    b = lz.lz_init(s, prec=prec, max_steps=64)
    b.restore(blob)
    assert b.state()[0] == 31
    b.step(20)
    got = b.coefficients()
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])
    # a checkpoint of another system is refused
    other = lz.lz_init(config_system("micro"), prec=prec, max_steps=64)
    with pytest.raises(lz.LzError) as e:
        other.restore(blob)
    assert e.value.status == lz.LZ_ERR_ARG
    with pytest.raises(lz.LzError):
        b.restore(blob[:100])
    for c in (a, b, other):
        c.free()
