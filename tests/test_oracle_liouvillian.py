"""Pins of the oracle's D, K and y (Sec. 2.4): the matrix-free operators
against explicit matrices built from explicit Fourier sums, Hermiticity in the
weighted product, and positivity of the RPA kernel."""
import numpy as np
import pytest

from oracle.brute import Brute
from oracle.liouvillian import Liouvillian
from synth import config_system, random_batch


@pytest.mark.parametrize("approx", ["tddft", "rpa", "ipa"])
def test_matrix_free_D_and_K_equal_explicit_matrices(micro, approx):
    L = Liouvillian(micro, approx)
    b = Brute(micro, approx)
    D, K, _ = b.explicit_operators()
    for seed in (1, 2):
        x = random_batch(micro, seed)
        xf = b.flatten(x)
        d_ref, k_ref = D @ xf, K @ xf
        scale = np.abs(d_ref).max()
        assert np.abs(b.flatten(L.apply_D(x)) - d_ref).max() < 1e-13 * scale
        assert np.abs(b.flatten(L.apply_K(x)) - k_ref).max() < 1e-13 * scale


def _conduction_batch(L, s, seed):
    return L.project_c(random_batch(s, seed))


@pytest.mark.parametrize("name", ["micro", "cfg1", "cfg2lo"])
def test_D_and_K_hermitian_on_conduction_manifold(name):
    s = config_system(name)
    L = Liouvillian(s, "tddft")
    a, c = _conduction_batch(L, s, 5), _conduction_batch(L, s, 6)
    for op in (L.apply_D, L.apply_K):
        lhs = L.inner(a, op(c))
        rhs = np.conj(L.inner(c, op(a)))
        scale = abs(L.inner(a, L.apply_D(a))) + abs(L.inner(c, L.apply_D(c)))
        assert abs(lhs - rhs) <= 1e-12 * scale


def test_rhs_lies_in_conduction_manifold(cfg1):
    L = Liouvillian(cfg1)
    y = L.rhs()
    for k, b in enumerate(L.blocks(y)):
        assert np.abs(b @ L.u_kq[k].conj().T).max() < 1e-13


def test_rpa_kernel_is_positive_semidefinite(micro):
    b = Brute(micro, "rpa").matrices()
    ev = np.linalg.eigvalsh(0.5 * (b.Ksym + b.Ksym.conj().T))
    assert ev.min() > -1e-12 * ev.max()


def test_metric_positive_definite_for_workload_cells():
    """D and D+K positive definite (J-metric) on the tiny cells."""
    for name in ("micro",):
        s = config_system(name)
        b = Brute(s, "tddft").matrices()
        assert b.dE.min() > 0
        ev = np.linalg.eigvalsh(np.diag(b.dE) + b.Ksym)
        assert ev.min() > 0


def test_response_density_equals_pair_density_sum(micro):
    """n'[x](r) for x = a single transition vector is 4 w_k rho_t(r)."""
    L = Liouvillian(micro, "rpa")
    b = Brute(micro, "rpa").transition_basis()
    k, n, ci = b.trans[3]
    h, _ = b.hamiltonian(k)
    _, vec = np.linalg.eigh(h)
    x = np.zeros((micro.nks, micro.nbnd, micro.npwx), dtype=np.complex128)
    x[k, n, :int(micro.npw_kq[k])] = vec[:, micro.nbnd + ci]
    ref = 4 * micro.wk[k] * b.rho[3]
    assert np.abs(L.density(x) - ref).max() < 1e-12 * np.abs(ref).max()
