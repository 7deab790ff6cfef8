"""Pins of the oracle's Kohn-Sham Hamiltonian, ground state and projector
(Sec. 2.3).  These check the oracle against explicit Fourier sums and against
the eigen-properties of the synthetic ground state, never against itself."""
import numpy as np
import pytest

from oracle.brute import Brute
from oracle.liouvillian import Liouvillian
from oracle.pw import Cell, Hamiltonian
from synth import config_system, random_batch


def _hmax(h):
    return np.abs(np.linalg.eigvalsh(h)).max()


def test_fft_hamiltonian_equals_explicit_sum(micro):
    """H applied through FFTs equals the explicit matrix built with explicit
    exponentials (kinetic + V~(G-G') + projectors)."""
    L = Liouvillian(micro)
    b = Brute(micro)
    x = random_batch(micro, 3)
    hx = L.apply_h(x)
    for k in range(micro.nks):
        h, _ = b.hamiltonian(k)
        npw = int(micro.npw_kq[k])
        ref = x[k, :, :npw] @ h.T
        err = np.abs(hx[k, :, :npw] - ref).max() / (_hmax(h) * np.abs(x[k]).max())
        assert err < 1e-13


@pytest.mark.parametrize("name", ["micro", "cfg1", "cfg2lo"])
def test_hamiltonian_hermitian(name):
    s = config_system(name)
    L = Liouvillian(s)
    a, c = random_batch(s, 1), random_batch(s, 2)
    ha, hc = L.apply_h(a), L.apply_h(c)
    for k in range(s.nks):
        lhs = np.vdot(a[k], hc[k])
        rhs = np.vdot(ha[k], c[k])
        scale = np.linalg.norm(a[k]) * np.linalg.norm(c[k]) * np.abs(ha[k]).max() / np.abs(a[k]).max()
        assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("name", ["micro", "cfg1", "cfg2lo", "free"])
def test_valence_states_are_eigenstates_at_k_plus_q(name):
    """||H_{k+q} u - eps u|| small for the occupied states that build P_c."""
    s = config_system(name)
    L = Liouvillian(s)
    for k in range(s.nks):
        u = L.u_kq[k]
        hu = L.ham[k].apply(u)
        e = s.et_kq[k, :s.nbnd]
        assert np.abs(hu - e[:, None] * u).max() < 1e-8
        assert np.abs(u @ u.conj().T - np.eye(s.nbnd)).max() < 1e-13


@pytest.mark.parametrize("name", ["cfg1", "free"])
def test_valence_states_are_eigenstates_at_k(name):
    """Local-potential cells: the orbitals at k (which carry eps_nk into D)
    are eigenstates of the oracle's own H_k."""
    s = config_system(name)
    cell = Cell(s.at, s.nr)
    for k in range(s.nks):
        npw = int(s.npw_k[k])
        h = Hamiltonian(cell, s.nl_k[k, :npw], s.xk[k], s.vloc_r)
        u = s.evc_k[k, :, :npw]
        hu = h.apply(u)
        assert np.abs(hu - s.et_k[k][:, None] * u).max() < 1e-8
        assert np.abs(u @ u.conj().T - np.eye(s.nbnd)).max() < 1e-13


@pytest.mark.parametrize("name", ["micro", "cfg1", "free"])
def test_ground_state_density_integrates_to_electron_count(name):
    s = config_system(name)
    omega = abs(np.linalg.det(s.at))
    total = s.n0_r.sum() * omega / s.n0_r.size
    assert abs(total - 2 * s.nbnd) < 1e-10


def test_projector_idempotent_and_kills_valence(micro):
    L = Liouvillian(micro)
    x = random_batch(micro, 4)
    for k, b in enumerate(L.blocks(x)):
        p1 = L.pc(k, b)
        p2 = L.pc(k, p1)
        assert np.abs(p1 - p2).max() < 1e-14 * np.abs(b).max()
        assert np.abs(L.pc(k, L.u_kq[k])).max() < 1e-14


def test_free_electron_orbitals_are_plane_waves(free):
    """V = 0: every occupied orbital lives on the 7 shortest G of the shell and
    the energies are 1/2 |G|^2 (0 and 1/2 b^2, six-fold)."""
    b = 2 * np.pi / free.at[0, 0]
    e = np.sort(free.et_k[0])
    assert abs(e[0]) < 1e-12
    assert np.allclose(e[1:], 0.5 * b * b, atol=1e-12)
