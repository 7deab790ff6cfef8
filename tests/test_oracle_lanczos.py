"""Pins of the pseudo-Hermitian Lanczos recursion and of chi (Sec. 2.5):
exhaustive Krylov spaces against the direct resolvent, the Casida form and
the closed forms; the matrix-free recursion against the explicit-matrix one;
invariances of beta, z and chi."""
import numpy as np
import pytest

from oracle import closed_forms, lanczos, spectrum
from oracle.brute import Brute
from oracle.liouvillian import Liouvillian
from synth import config_system

OMEGA = np.linspace(0.0, 3.0, 241)


@pytest.mark.parametrize("approx", ["tddft", "rpa", "ipa"])
def test_exhaustive_lanczos_equals_direct_resolvent(micro, approx):
    L = Liouvillian(micro, approx)
    b = Brute(micro, approx).matrices()
    nt = len(b.dE)
    r = lanczos.run(L, 2 * nt + 5, reorth=True)
    assert r.status == "breakdown" and r.steps == 2 * nt
    eta = 0.05
    ref = b.chi_direct(OMEGA, eta)
    chi = spectrum.chi_from_coefficients(r.beta, r.z, OMEGA, eta, L.cell.omega)
    assert np.abs(chi - ref).max() < 1e-10 * np.abs(ref).max()
    cas = b.chi_casida(OMEGA, eta)
    assert np.abs(cas - ref).max() < 1e-10 * np.abs(ref).max()


def test_independent_particle_closed_form(micro):
    L = Liouvillian(micro, "ipa")
    nt = len(Brute(micro, "ipa").transition_basis().dE)
    r = lanczos.run(L, 2 * nt + 5, reorth=True)
    chi = spectrum.chi_from_coefficients(r.beta, r.z, OMEGA, 0.05, L.cell.omega)
    ref = closed_forms.ipa_chi(micro, OMEGA, 0.05)
    assert np.abs(chi - ref).max() < 1e-10 * np.abs(ref).max()


def test_matrix_free_recursion_matches_explicit_matrix_recursion(micro):
    """First 50 steps, no reorthogonalisation: beta and z to 1e-10."""
    L = Liouvillian(micro, "tddft")
    b = Brute(micro, "tddft")
    D, K, _ = b.explicit_operators()
    w = np.concatenate([[micro.wk[k]] * (micro.nbnd * int(micro.npw_kq[k])) for k in range(micro.nks)])
    pcs = []
    for k in range(micro.nks):
        u = L.u_kq[k]
        pcs.append(np.eye(u.shape[1]) - u.T @ u.conj())
    def project(v):
        out, o = [], 0
        for k in range(micro.nks):
            npw = int(micro.npw_kq[k])
            for _ in range(micro.nbnd):
                out.append(pcs[k] @ v[o:o + npw])
                o += npw
        return np.concatenate(out)
    yflat = b.flatten(L.rhs())
    r_mat = lanczos.pseudo_hermitian_lanczos(
        lambda v: D @ v, lambda v: (D + K) @ v, lambda a, c: complex(np.sum(w * np.conj(a) * c)),
        yflat, 50, project=project, y_scale=float(micro.nbnd))
    r_mf = lanczos.run(L, 50)
    assert r_mat.steps == r_mf.steps == 50
    assert np.abs(r_mat.beta - r_mf.beta).max() < 1e-10 * np.abs(r_mf.beta).max()
    assert np.abs(r_mat.z - r_mf.z).max() < 1e-10 * np.abs(r_mf.z).max()


@pytest.mark.parametrize("approx", ["ipa", "rpa", "tddft"])
def test_free_electron_dyson_closed_form_and_lucky_breakdown(free, approx):
    L = Liouvillian(free, approx)
    r = lanczos.run(L, 60)
    d = closed_forms.free_electron_transitions(free.at, free.ecut, free.q, free.g0)
    assert r.status == "breakdown"
    assert r.steps == 2 * len(np.unique(np.round(d, 9)))
    chi = spectrum.chi_from_coefficients(r.beta, r.z, OMEGA, 0.02, L.cell.omega)
    fxc = float(free.fxc_r[0])
    assert np.allclose(free.fxc_r, fxc, rtol=1e-12)
    ref = closed_forms.free_electron_chi(free.at, free.ecut, free.q, free.g0, OMEGA, 0.02, approx, fxc)
    assert np.abs(chi - ref).max() < 1e-12 * np.abs(ref).max()


def test_free_electron_pauli_blocked_rhs_vanishes():
    """G0 = 0, small q: every transition G -> G is blocked, chi = 0."""
    s = config_system("free", g0=(0, 0, 0))
    r = lanczos.run(Liouvillian(s), 20)
    assert r.status == "breakdown" and r.steps == 0
    chi = spectrum.chi_from_coefficients(r.beta, r.z, OMEGA, 0.02, 1.0)
    assert np.all(chi == 0)


def test_invariance_under_phases_and_degenerate_rotations(free):
    """beta, z, chi do not change when the valence orbitals are multiplied by
    phases and rotated inside a degenerate shell."""
    rng = np.random.default_rng(9)
    r0 = lanczos.run(Liouvillian(free, "tddft"), 4)
    s2 = config_system("free")
    e = s2.et_k[0]
    shell = np.where(np.abs(e - e.max()) < 1e-9)[0]
    a = rng.standard_normal((len(shell), len(shell))) + 1j * rng.standard_normal((len(shell), len(shell)))
    uq, _ = np.linalg.qr(a)
    s2.evc_k = s2.evc_k.copy()
    s2.evc_k[0, shell] = uq @ s2.evc_k[0, shell]
    s2.evc_k[0] *= np.exp(1j * rng.uniform(0, 2 * np.pi, s2.nbnd))[:, None]
    s2.evc_kq = s2.evc_kq.copy()
    s2.evc_kq[0] *= np.exp(1j * rng.uniform(0, 2 * np.pi, s2.nbnd))[:, None]
    r1 = lanczos.run(Liouvillian(s2, "tddft"), 4)
    assert np.allclose(r0.beta, r1.beta, rtol=1e-12)
    assert np.allclose(r0.z, r1.z, rtol=1e-12, atol=1e-14)


def test_phase_invariance_generic_cell(micro):
    rng = np.random.default_rng(11)
    r0 = lanczos.run(Liouvillian(micro), 30)
    s2 = config_system("micro")
    s2.evc_k = s2.evc_k * np.exp(1j * rng.uniform(0, 2 * np.pi, s2.evc_k.shape[:2]))[..., None]
    s2.evc_kq = s2.evc_kq * np.exp(1j * rng.uniform(0, 2 * np.pi, s2.evc_kq.shape[:2]))[..., None]
    r1 = lanczos.run(Liouvillian(s2), 30)
    assert np.abs(r0.beta - r1.beta).max() < 1e-10 * r0.beta.max()
    assert np.abs(r0.z - r1.z).max() < 1e-10 * np.abs(r0.z).max()


def test_scaling_rhs_scales_only_start_norm(micro):
    L = Liouvillian(micro)
    y = L.rhs()
    c = 2.5 * np.exp(0.3j)
    r0 = lanczos.pseudo_hermitian_lanczos(L.apply_D, L.apply_DK, L.inner, y, 20, project=L.project_c)
    r1 = lanczos.pseudo_hermitian_lanczos(L.apply_D, L.apply_DK, L.inner, c * y, 20, project=L.project_c)
    assert abs(r1.beta[0] - abs(c) * r0.beta[0]) < 1e-12 * r1.beta[0]
    assert np.allclose(r1.beta[1:], r0.beta[1:], rtol=1e-11)
    assert np.allclose(r1.z, abs(c) * r0.z, rtol=1e-11, atol=1e-14)


def test_tridiagonal_eigenvalues_come_in_pairs_and_z_is_real(cfg1):
    r = lanczos.run(Liouvillian(cfg1), 60)
    m = len(r.beta)
    t = np.diag(r.beta[1:], 1) + np.diag(r.beta[1:], -1)
    ev = np.sort(np.linalg.eigvalsh(t))
    assert np.allclose(ev, -ev[::-1], atol=1e-12 * np.abs(ev).max())
    assert np.abs(r.z.imag).max() < 1e-12 * np.abs(r.z).max()
    assert np.all(r.z[0::2] == 0)
    assert m == 60


def test_projecting_only_the_new_vector_gives_the_same_recursion(cfg1):
    """Operators whose output keeps its valence part, with P_c applied only to
    each new vector, give the coefficients of the recursion that also projects
    every output: each Lanczos sum pairs an output with a conduction vector,
    and each new vector is projected before an operator acts on it.  (The
    device recursion takes this order; the oracle projects both.)"""
    L = Liouvillian(cfg1)

    def d_raw(x):
        return L.pack([L.ham[k].apply(b) - L.eps[k][:, None] * b
                       for k, b in enumerate(L.blocks(x))])

    def dk_raw(x):
        v = L.hxc_potential(L.density(x))
        return d_raw(x) + L.pack([L.cell.to_coef(v[None, :] * L.u_r[k], L.nl_kq[k])
                                  for k in range(L.nks)])

    # the raw operators really leave a valence part in their outputs
    y = L.rhs()
    assert np.abs(L.project_c(dk_raw(y)) - dk_raw(y)).max() > 1e-3 * np.abs(dk_raw(y)).max()
    ref = lanczos.run(L, 40)
    alt = lanczos.pseudo_hermitian_lanczos(d_raw, dk_raw, L.inner, y, 40, project=L.project_c,
                                           y_scale=float(L.nbnd))
    assert alt.steps == ref.steps == 40
    assert np.max(np.abs(alt.beta - ref.beta) / ref.beta) < 1e-11
    assert np.abs(alt.z - ref.z).max() < 1e-11 * np.abs(ref.z).max()


@pytest.mark.parametrize("approx", ["tddft", "rpa", "ipa"])
def test_nonhermitian_exhaustive_equals_direct_resolvent(micro, approx):
    """The biorthogonal recursion with two-sided re-biorthogonalisation
    exhausts the Krylov space at the same dimension and reproduces the
    direct resolvent of the explicit L."""
    L = Liouvillian(micro, approx)
    b = Brute(micro, approx).matrices()
    nt = len(b.dE)
    r = lanczos.run(L, 2 * nt + 5, reorth=True, variant="nh")
    assert r.status == "breakdown" and r.steps == 2 * nt
    chi = spectrum.chi_from_coefficients(r.beta, r.z, OMEGA, 0.05, L.cell.omega, gamma=r.gamma)
    ref = b.chi_direct(OMEGA, 0.05)
    assert np.abs(chi - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("approx", ["ipa", "rpa", "tddft"])
def test_nonhermitian_free_electron_dyson_and_breakdown(free, approx):
    L = Liouvillian(free, approx)
    r = lanczos.run(L, 60, variant="nh")
    d = closed_forms.free_electron_transitions(free.at, free.ecut, free.q, free.g0)
    assert r.status == "breakdown"
    assert r.steps == 2 * len(np.unique(np.round(d, 9)))
    chi = spectrum.chi_from_coefficients(r.beta, r.z, OMEGA, 0.02, L.cell.omega, gamma=r.gamma)
    fxc = float(free.fxc_r[0])
    ref = closed_forms.free_electron_chi(free.at, free.ecut, free.q, free.g0, OMEGA, 0.02, approx, fxc)
    assert np.abs(chi - ref).max() < 1e-12 * np.abs(ref).max()


def test_nonhermitian_reduces_to_symmetric_chain_without_kernel(micro):
    """IPA (K = 0): L^dagger = L, so u_j = v_j, gamma = beta and the chain is
    the Hermitian Lanczos of L in the plain product."""
    r = lanczos.run(Liouvillian(micro, "ipa"), 40, variant="nh")
    assert np.abs(r.gamma - r.beta).max() < 1e-12 * r.beta.max()


def test_nonhermitian_recursion_amplifies_rounding(cfg1):
    """A relative perturbation of 6e-8 (single-precision rounding) on every
    operator application moves the loss function of 60 steps by far more in
    the non-Hermitian recursion than in the pseudo-Hermitian one (measured
    2e-3 against 4e-6 on this cell): the two biorthogonal chains lose their
    coupling to rounding, the J-metric recursion does not."""
    L = Liouvillian(cfg1, "tddft")
    y = L.rhs()
    om = np.linspace(0.0, 2.0, 2000)

    def loss_change(fn, nh):
        rng = np.random.default_rng(1)

        def noisy(f):
            def g(x):
                v = f(x)
                e = 6e-8 * (rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape))
                return v * (1 + e / np.sqrt(2))
            return g
        kw = dict(project=L.project_c, y_scale=float(L.nbnd))
        r0 = fn(L.apply_D, L.apply_DK, L.inner, y, 60, **kw)
        r1 = fn(noisy(L.apply_D), noisy(L.apply_DK), L.inner, y, 60, **kw)
        out = []
        for r in (r0, r1):
            out.append(spectrum.spectrum(r.beta, r.z, om, 0.01, L.cell.omega, L.Q,
                                         gamma=r.gamma if nh else None)[2])
        floor = 1e-6 * np.abs(out[0]).max()
        return np.max(np.abs(out[1] - out[0]) / np.maximum(np.abs(out[0]), floor))

    ph = loss_change(lanczos.pseudo_hermitian_lanczos, False)
    nh = loss_change(lanczos.nonhermitian_lanczos, True)
    assert nh > 100 * ph


def test_gapless_system_is_not_positive_definite():
    """Without a gap (an empty state at k+q below a filled one at k) some
    transition energies are negative, D is indefinite and so is the metric
    diag(D+K, D) of the pseudo-Hermitian recursion (Sec. 2.5): the recursion
    must stop with not_pd, and the explicit-matrix recursion agrees."""
    s = config_system("gapless")
    b = Brute(s, "tddft")
    assert b.transition_basis().dE.min() < -0.05
    L = Liouvillian(s, "tddft")
    r = lanczos.run(L, 300)
    assert r.status == "not_pd"
    assert 2 < r.steps < 300
    D, K, _ = b.explicit_operators()
    assert np.linalg.eigvalsh(0.5 * (D + D.conj().T)).min() < 0
    w = np.concatenate([[s.wk[k]] * (s.nbnd * int(s.npw_kq[k])) for k in range(s.nks)])
    pcs = []
    for k in range(s.nks):
        u = L.u_kq[k]
        pcs.append(np.eye(u.shape[1]) - u.T @ u.conj())

    def project(v):
        out, o = [], 0
        for k in range(s.nks):
            npw = int(s.npw_kq[k])
            for _ in range(s.nbnd):
                out.append(pcs[k] @ v[o:o + npw])
                o += npw
        return np.concatenate(out)
    r_mat = lanczos.pseudo_hermitian_lanczos(
        lambda v: D @ v, lambda v: (D + K) @ v, lambda a, c: complex(np.sum(w * np.conj(a) * c)),
        b.flatten(L.rhs()), 300, project=project, y_scale=float(s.nbnd))
    assert r_mat.status == "not_pd" and r_mat.steps == r.steps
    assert np.abs(r_mat.beta - r.beta).max() < 1e-9 * np.abs(r.beta).max()
