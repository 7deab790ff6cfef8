"""Several instances in one context advanced side by side: a q-dispersion
sweep (the crystal of the 32^3 cell at eight transferred momenta) and
instances of different grids, run on several streams, against the same
instances one after another on one stream and against contexts of their own
(bit for bit: the arithmetic of an instance does not depend on what runs
beside it), and the sweep's end points against the oracle."""
import dataclasses
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


@pytest.mark.parametrize("prec,graph", [("fp64", False), ("fp32", False), ("splitbf16", False),
                                        ("fp32", True)])
def test_q_sweep_one_launch_per_kernel_equals_per_instance(sweep, prec, graph):
    """With batched=True every kernel of a step runs once over the eight
    instances (a work list of (instance, block) items); the coefficients equal
    those of the per-instance launches bit for bit, since each block runs the
    same code on the same data (also with the pairs of steps replayed as one
    captured graph)."""
    lz = _lz()
    n = len(sweep)
    print(f"[sweep] {prec} batched, graph={graph}, instances={n}", flush=True)
    seq = lz.lz_init(sweep, prec=prec, max_steps=64, streams=1)
    seq.step(7)
    seq.step(40)
    ref = _coefs(seq, n)
    seq.free()
    bat = lz.lz_init(sweep, prec=prec, max_steps=64, batched=True, use_graph=graph)
    bat.step(7)
    done, st = bat.step(40)
    assert done == 47 and st == lz.LZ_OK
    got = _coefs(bat, n)
    for i in range(n):
        assert _same(got[i], ref[i]), i
    bat.free()


def test_one_launch_per_kernel_groups_and_breakdown():
    """Instances of three grids (24^3, 32^3 and a general 12^3 grid) and free
    electrons that break down after a few steps, batched: the instances form
    one group per kernel sequence, each group launched as one; every instance
    equals a context of its own bit for bit, also after the breakdown of the
    free-electron members (their blocks return at once from then on), and
    after a reset."""
    lz = _lz()
    systems = [config_system("cfg1"), config_system("free"), config_system("micro"),
               config_system("cfg2lo"), config_system("cfg1"), config_system("free")]
    alone = []
    for s in systems:
        c = lz.lz_init(s, prec="fp64", max_steps=48)
        c.step(40)
        alone.append((_coefs(c, 1)[0], c.state()))
        c.free()
    for streams, graph in ((1, False), (0, False), (0, True)):
        print(f"[groups] batched, streams={streams}, graph={graph}", flush=True)
        ctx = lz.lz_init(systems, prec="fp64", max_steps=48, batched=True, streams=streams,
                         use_graph=graph)
        for rep in range(2):
            _, st = ctx.step(15)
            _, st = ctx.step(25)
            assert st == lz.LZ_BREAKDOWN
            for i in range(len(systems)):
                assert ctx.state(i) == alone[i][1]
                assert _same(_coefs(ctx, len(systems))[i], alone[i][0]), i
            ctx.reset()
        ctx.free()


def test_uneven_members_one_launch_per_kernel():
    """The ten members of the uneven batch (grids 32^3 to 72^3; vector-ALU and
    matrix-core projector paths; 8 to 768 band-k products) batched equal the
    per-instance launches bit for bit over 12 steps, in both precisions."""
    lz = _lz()
    idx = SMALLEST + LARGEST
    systems = [config_system("uneven", index=i) for i in idx]
    for prec in ("fp64", "fp32"):
        print(f"[uneven] {prec} batched", flush=True)
        seq = lz.lz_init(systems, prec=prec, max_steps=16, streams=1)
        seq.step(12)
        ref = _coefs(seq, len(systems))
        seq.free()
        bat = lz.lz_init(systems, prec=prec, max_steps=16, batched=True)
        done, st = bat.step(12)
        assert done == 12 and st == lz.LZ_OK
        got = _coefs(bat, len(systems))
        for i in range(len(systems)):
            assert _same(got[i], ref[i]), idx[i]
        bat.free()


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


def _horizon(s, n, ref):
    """Steps over which the oracle's recursion of s is determined to rounding:
    the oracle run again with the local potential scaled by 1 + 1e-13 (a
    perturbation of the size of a rounding difference between two FP64
    implementations) agrees with ref to 1e-11 in beta and in z."""
    s2 = dataclasses.replace(s, vloc_r=s.vloc_r * (1.0 + 1e-13))
    alt = lanczos.run(Liouvillian(s2), n)
    zmax = np.abs(ref.z).max()
    bad = (np.abs(alt.beta - ref.beta) > 1e-11 * ref.beta) | (np.abs(alt.z - ref.z) > 1e-11 * zmax)
    return int(np.argmax(bad)) if bad.any() else n


@pytest.mark.slow
def test_uneven_members_recursions_in_one_context():
    """Ten members of the batched uneven workload (grids 32^3 to 72^3, up to
    768 band-k products) advance their recursions side by side in one
    context; the eight smallest members' first 40 coefficients and the two
    largest members' first 6 are compared with the oracle's, beta to 1e-10
    relative and z to 1e-10 of max|z|, over the steps where the oracle's own
    recursion is determined to rounding (_horizon).  These members' orbitals
    are seeded orthonormal sets with energies below the spectrum of H, not
    eigenstates; where |q| is small the Hartree term gives L an isolated large
    eigenvalue, the recursion converges to it within a few steps and from
    then on amplifies every rounding difference (a 1e-13 change of V_loc moves
    beta by 1e-2 within 30 steps on three of them, in the oracle alone: their
    horizons are 9 to 11 steps), so coefficients past that point are not a
    property of the operator."""
    import os

    import oracle.pw as opw
    lz = _lz()
    opw.FFT_WORKERS = min(len(os.sched_getaffinity(0)), 16)
    idx = SMALLEST + LARGEST
    systems = [config_system("uneven", index=i) for i in idx]
    print("[uneven] members built", flush=True)
    ctx = lz.lz_init(systems, prec="fp64", max_steps=48)
    done, st = ctx.step(40)
    assert st == lz.LZ_OK
    worst_b, worst_z = 0.0, 0.0
    for j, (i, s) in enumerate(zip(idx, systems)):
        n = 40 if i in SMALLEST else 6
        ref = lanczos.run(Liouvillian(s), n)
        h = _horizon(s, n, ref)
        beta, _, z = ctx.coefficients(inst=j)
        assert ctx.state(j)[0] == 40
        eb = float(np.max(np.abs(beta[:h] - ref.beta[:h]) / ref.beta[:h]))
        ez = float(np.abs(z[:h] - ref.z[:h]).max() / np.abs(ref.z).max())
        print(f"[uneven] member {i}: grid {int(s.nr[0])}, {s.nbnd} bands, {s.nks} k, "
              f"determined over {h} of {n} steps: beta {eb:.1e}, z {ez:.1e}", flush=True)
        # every member is compared over at least its first 8 steps (9 to 40 here)
        assert h >= min(n, 8)
        worst_b, worst_z = max(worst_b, eb), max(worst_z, ez)
    ctx.free()
    assert worst_b < 1e-10
    assert worst_z < 1e-10
