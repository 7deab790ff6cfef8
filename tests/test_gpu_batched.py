"""Several instances in one context advanced side by side: a q-dispersion
sweep (the crystal of the 32^3 cell at eight transferred momenta) and
instances of different grids, run on several streams, against the same
instances one after another on one stream and against contexts of their own
(bit for bit: the arithmetic of an instance does not depend on what runs
beside it), and the sweep's end points against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import lanczos, spectrum  # noqa: E402
from oracle.liouvillian import Liouvillian  # noqa: E402
from synth import config_system, q_sweep  # noqa: E402


def _lz():
    import paper_2111_06623_amd as lz
    lz.load()
    return lz


def _coefs(ctx, n):
    return [ctx.coefficients(inst=i) for i in range(n)]


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.fixture(scope="module")
def sweep():
    return q_sweep("cfg2lo")


@pytest.mark.parametrize("prec,graph", [("fp64", False), ("fp32", True), ("fp32", False)])
def test_q_sweep_side_by_side_equals_one_after_another(sweep, prec, graph):
    lz = _lz()
    n = len(sweep)
    print(f"[sweep] {prec} graph={graph} instances={n}", flush=True)
    seq = lz.lz_init(sweep, prec=prec, max_steps=64, use_graph=graph, streams=1)
    seq.step(7)
    seq.step(40)
    ref = _coefs(seq, n)
    seq.free()
    par = lz.lz_init(sweep, prec=prec, max_steps=64, use_graph=graph)
    par.step(7)
    done, st = par.step(40)
    assert done == 47 and st == lz.LZ_OK
    got = _coefs(par, n)
    for i in range(n):
        assert _same(got[i], ref[i]), i
    # a context of its own for two of the instances
    for i in (0, n - 1):
        one = lz.lz_init(sweep[i], prec=prec, max_steps=64, use_graph=graph)
        one.step(47)
        assert _same(_coefs(one, 1)[0], ref[i])
        one.free()
    par.free()


def test_q_sweep_end_points_match_oracle(sweep):
    """FP64: beta and z of the smallest and largest q over 50 steps to 1e-10,
    and the loss functions of the two (the dispersion's end points) to 1e-6."""
    lz = _lz()
    ctx = lz.lz_init(sweep, prec="fp64", max_steps=64)
    ctx.step(50)
    om = np.linspace(0.0, 2.0, 2000)
    for i in (0, len(sweep) - 1):
        L = Liouvillian(sweep[i])
        ref = lanczos.run(L, 50)
        beta, _, z = ctx.coefficients(inst=i)
        assert np.max(np.abs(beta - ref.beta) / ref.beta) < 1e-10
        assert np.abs(z - ref.z).max() < 1e-10 * np.abs(ref.z).max()
        _, _, loss = ctx.spectrum(om, 0.01, inst=i)
        _, _, loss_r, _ = spectrum.spectrum(ref.beta, ref.z, om, 0.01, L.cell.omega, L.Q)
        floor = 1e-6 * np.abs(loss_r).max()
        assert np.max(np.abs(loss - loss_r) / np.maximum(np.abs(loss_r), floor)) < 1e-6
    ctx.free()


def test_breakdown_of_one_instance_leaves_the_others_running():
    """Free electrons break down after a few steps; the other instances of
    the context, on other streams and on the same one, run on unchanged."""
    lz = _lz()
    systems = [config_system("cfg1"), config_system("free"), config_system("micro"),
               config_system("cfg1"), config_system("free")]
    alone = []
    for s in systems:
        c = lz.lz_init(s, prec="fp64", max_steps=48)
        c.step(40)
        alone.append((_coefs(c, 1)[0], c.state()))
        c.free()
    ctx = lz.lz_init(systems, prec="fp64", max_steps=48, streams=2)
    _, st = ctx.step(40)
    assert st == lz.LZ_BREAKDOWN
    for i in range(len(systems)):
        assert ctx.state(i) == alone[i][1]
        assert _same(_coefs(ctx, len(systems))[i], alone[i][0])
    ctx.free()


def test_non_hermitian_instances_side_by_side():
    lz = _lz()
    systems = [config_system("cfg1"), config_system("micro"), config_system("cfg2lo")]
    seq = lz.lz_init(systems, prec="fp64", max_steps=40, streams=1, algorithm="nh")
    seq.step(30)
    ref = _coefs(seq, 3)
    seq.free()
    par = lz.lz_init(systems, prec="fp64", max_steps=40, algorithm="nh", use_graph=True)
    par.step(30)
    got = _coefs(par, 3)
    for i in range(3):
        assert _same(got[i], ref[i])
    par.free()



# members of the batched uneven workload (seeded; grid, bands, k-points): the
# eight smallest by bands x grid points and the two largest
SMALLEST = (60, 58, 49, 32, 62, 16, 3, 22)   # 32^3..48^3, 8-48 bands, 1-8 k
LARGEST = (29, 12)                            # 72^3: 40 bands x 9 k, 48 bands x 16 k


@pytest.mark.slow
def test_uneven_members_recursions_in_one_context():
    """Ten members of the batched uneven workload (grids 32^3 to 72^3, up to
    768 band-k products) advance their recursions side by side in one
    context; the eight smallest members' first 40 coefficients and the two
    largest members' first 6 against the oracle: beta to 1e-10 relative and z
    to 1e-10 of max|z| at every step.  These members' orbitals are seeded
    orthonormal sets with energies below the spectrum of H (not eigenstates:
    D is positive definite by construction), so the check runs in the RPA,
    whose Hartree kernel keeps D + K positive definite too; with the ALDA
    kernel of their random densities the metric of several members is close
    to indefinite and their recursions amplify rounding (by about 10 per step
    on three of them, where the oracle's own Im z, zero in exact arithmetic,
    grows at the same rate), which no two implementations reproduce alike."""
    import os

    import oracle.pw as opw
    lz = _lz()
    opw.FFT_WORKERS = min(len(os.sched_getaffinity(0)), 16)
    idx = SMALLEST + LARGEST
    systems = [config_system("uneven", index=i) for i in idx]
    print("[uneven] members built", flush=True)
    ctx = lz.lz_init(systems, prec="fp64", approx="rpa", max_steps=48)
    done, st = ctx.step(40)
    assert st == lz.LZ_OK
    worst_b, worst_z = 0.0, 0.0
    for j, (i, s) in enumerate(zip(idx, systems)):
        n = 40 if i in SMALLEST else 6
        ref = lanczos.run(Liouvillian(s, "rpa"), n)
        beta, _, z = ctx.coefficients(inst=j)
        assert ctx.state(j)[0] == 40
        eb = float(np.max(np.abs(beta[:n] - ref.beta) / ref.beta))
        ez = float(np.abs(z[:n] - ref.z).max() / np.abs(ref.z).max())
        print(f"[uneven] member {i}: grid {int(s.nr[0])}, {s.nbnd} bands, {s.nks} k, {n} steps: "
              f"beta {eb:.1e}, z {ez:.1e}", flush=True)
        worst_b, worst_z = max(worst_b, eb), max(worst_z, ez)
    ctx.free()
    assert worst_b < 1e-10
    assert worst_z < 1e-10
