"""Susceptibility, dielectric function and loss function from the Lanczos
coefficients (Sec. 2.5, eqs. resolvent_Liouvillian_Lanczos_q, post_processing,
resolvent_Liouvillian_Lanczos_2_for_chi; Sec. 2.1 eq.
def_inv_microscopic_diel_tensor; Sec. 3.3 for the Lorentzian broadening).

    (omega + i eta - T_M) x = e_1          T_M symmetric tridiagonal, zero
                                           diagonal, off-diagonals beta_2..beta_M
    chi(omega) = (4/Omega) beta_1 sum_j z_j x_j
    eps^-1     = 1 + 4 pi chi / |Q|^2,   loss = -Im eps^-1,   eps = 1/eps^-1

z_j is real in exact arithmetic: it is <y, (D(D+K))^i D y>_w up to the
normalisations, a palindromic product of Hermitian operators.  The sum uses
Re z_j, dropping the rounding-level imaginary part.

The prefactor reading: (z, x) with the normalised start vector must be
multiplied by the start norm beta_1; 4/Omega collects the spin factor 2, the
SBR factor 2 of the response density and the per-volume normalisation of the
orbitals.  It is pinned by the independent-particle sum over states and by the
first-moment (f-sum) closed form.

Each frequency is solved by LU with partial pivoting on the band matrix
(LAPACK gbsv through scipy.linalg.solve_banded).  The non-Hermitian form
(gamma given) has a non-symmetric T with sub-diagonal beta and super-diagonal
gamma, and its z_j are used as they are.

Extrapolation (Sec. 3.3, the itermax0 / itermax / extrapolation inputs of
the spectrum program; the paper defers the scheme to its references): the
computed coefficients are extended to a larger tridiagonal matrix.  Reading
used here: beyond the m0 computed coefficients every beta takes the mean of
the last half of the computed beta_2..beta_m0 ('constant'), or the mean of the
members of that window with the same index parity ('osc', bi-constant), and
z_j = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def chi_from_coefficients(beta, z, omega, eta, volume, m=None, gamma=None):
    """gamma None: the pseudo-Hermitian T (symmetric, real z reading);
    otherwise T has sub-diagonal beta and super-diagonal gamma (the
    non-Hermitian form) and z is kept complex."""
    beta = np.asarray(beta, dtype=np.float64)
    z = np.asarray(z, dtype=np.complex128)
    if gamma is None:
        z = z.real
    m = len(beta) if m is None else int(m)
    if m == 0:
        # no Lanczos vector: the right-hand side vanished, chi = 0
        return np.zeros(len(omega), dtype=np.complex128)
    sub = beta[1:m]
    sup = sub if gamma is None else np.asarray(gamma, dtype=np.complex128)[1:m]
    out = np.empty(len(omega), dtype=np.complex128)
    rhs = np.zeros(m, dtype=np.complex128)
    rhs[0] = 1.0
    ab = np.zeros((3, m), dtype=np.complex128)
    ab[0, 1:] = -sup
    ab[2, :-1] = -sub
    for i, w in enumerate(np.asarray(omega, dtype=np.float64)):
        ab[1, :] = w + 1j * eta
        x = sla.solve_banded((1, 1), ab, rhs)
        out[i] = np.sum(z[:m] * x)
    return (4.0 / volume) * beta[0] * out


def extrapolate(beta, z, m0, m, scheme):
    """The first m0 coefficients extended to m by `scheme` ('no', 'constant'
    or 'osc').  Returns (beta[0..m), z[0..m)); beta[i-1] is beta_i."""
    beta = np.asarray(beta, dtype=np.float64)[:m0]
    z = np.asarray(z, dtype=np.complex128)[:m0]
    if scheme == "no" or m <= m0:
        return beta, z
    if m0 < 4:
        raise ValueError("extrapolation needs at least 4 computed coefficients")
    lo = max(2, m0 // 2 + 1)                       # window beta_lo..beta_m0 (1-based)
    idx = np.arange(lo, m0 + 1)
    win = beta[idx - 1]
    if scheme == "constant":
        tail = {0: win.mean(), 1: win.mean()}
    elif scheme == "osc":
        tail = {par: win[idx % 2 == par].mean() for par in (0, 1)}
    else:
        raise ValueError(scheme)
    ext = np.array([tail[i % 2] for i in range(m0 + 1, m + 1)])
    return np.concatenate([beta, ext]), np.concatenate([z, np.zeros(m - m0, dtype=np.complex128)])


def dielectric(chi, qcart):
    """eps^-1, loss = -Im eps^-1 and eps = 1/eps^-1 (a scalar inverse)."""
    q2 = float(np.dot(qcart, qcart))
    eps_inv = 1.0 + 4.0 * np.pi * np.asarray(chi) / q2
    return eps_inv, -eps_inv.imag, 1.0 / eps_inv


def spectrum(beta, z, omega, eta, volume, qcart, m=None, m_total=None, scheme="no", gamma=None):
    """With m_total > m and scheme 'constant' or 'osc', the coefficients are
    extrapolated from the first m to m_total before the solve (pseudo-Hermitian
    form only); gamma selects the non-Hermitian form."""
    if m_total is not None and scheme != "no":
        if gamma is not None:
            raise ValueError("extrapolation of the non-Hermitian coefficients is not defined here")
        m0 = len(beta) if m is None else int(m)
        beta, z = extrapolate(beta, z, m0, int(m_total), scheme)
        m = len(beta)
    chi = chi_from_coefficients(beta, z, omega, eta, volume, m, gamma=gamma)
    eps_inv, loss, eps = dielectric(chi, qcart)
    return chi, eps_inv, loss, eps
