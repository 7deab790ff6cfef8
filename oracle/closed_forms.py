"""Closed forms that pin the oracle.

  ipa_chi            independent-particle sum over states (K = 0, the IPA
                     level of Sec. 3.2):
                     chi_0 = (2/Omega) sum_k w_k sum_{n,c} |<c,k+q|e^{iG0.r}|n,k>|^2
                             [1/(w~ - d) - 1/(w~ + d)],  d = eps_{c,k+q} - eps_{n,k}
  free_electron_chi  V = 0, one closed shell at Gamma: every pair density is
                     the single plane wave e^{iG0.r}/Omega, so K is rank one
                     and chi = chi_0 / (1 - (4 pi/|Q|^2 + f_xc) chi_0)
                     (the Dyson-like screening form recalled in Sec. 1)
  first_moment       <y, D y>_w, the coefficient of the 1/omega^2 tail of chi
                     (chi -> (4/Omega) <y,Dy>_w / omega^2), written out for
                     local potentials through
                     e^{-iG0.r} H_{k+q} e^{iG0.r} = H_k + Q.(-i grad + k) + Q^2/2
                     (the Thomas-Reiche-Kuhn rule of Sec. 2.1; exact for local
                     potentials, Sec. 3.3), valid when the k+q basis contains
                     the G0-shifted k sphere.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .brute import Brute
from .pw import miller_from_index, reciprocal


def ipa_chi(s, omega, eta):
    b = Brute(s, approx="ipa").transition_basis()
    w = np.asarray(omega)[:, None] + 1j * eta
    a = (b.wt * np.abs(b.yt) ** 2)[None, :]
    d = b.dE[None, :]
    return (2.0 / b.omega) * np.sum(a * (1.0 / (w - d) - 1.0 / (w + d)), axis=1)


def free_electron_transitions(at, ecut, q, g0, nocc=7):
    """Allowed transitions G_n -> G_n + G0 of a free-electron closed shell at
    Gamma: returns the excitation energies d (one per allowed transition)."""
    bg = reciprocal(at)
    lim = int(math.ceil(math.sqrt(2 * ecut) * np.max(np.linalg.norm(at, axis=1)) / (2 * np.pi))) + 2
    mill = np.array(list(itertools.product(range(-lim, lim + 1), repeat=3)))
    g = mill @ bg
    e0 = 0.5 * np.einsum("ij,ij->i", g, g)
    occ0 = mill[np.argsort(e0, kind="stable")[:nocc]]
    gq = np.asarray(q)[None, :] + g
    eq = 0.5 * np.einsum("ij,ij->i", gq, gq)
    in_sphere = {tuple(m) for m in mill[eq <= ecut]}
    occq = {tuple(m) for m in mill[np.argsort(eq, kind="stable")[:nocc]]}
    d = []
    for m in occ0:
        t = tuple(np.asarray(m) + np.asarray(g0))
        if t in in_sphere and t not in occq:
            gt = np.asarray(q) + np.asarray(t) @ bg
            gn = np.asarray(m) @ bg
            d.append(0.5 * gt @ gt - 0.5 * gn @ gn)
    return np.array(d)


def free_electron_chi(at, ecut, q, g0, omega, eta, approx="tddft", fxc=0.0, nocc=7):
    omega_cell = abs(np.linalg.det(at))
    d = free_electron_transitions(at, ecut, q, g0, nocc)
    w = np.asarray(omega)[:, None] + 1j * eta
    chi0 = (2.0 / omega_cell) * np.sum(1.0 / (w - d[None, :]) - 1.0 / (w + d[None, :]), axis=1)
    if approx == "ipa":
        return chi0
    Q = np.asarray(q) + np.asarray(g0) @ reciprocal(at)
    f = 4.0 * np.pi / float(Q @ Q) + (fxc if approx == "tddft" else 0.0)
    return chi0 / (1.0 - f * chi0)


def first_moment(s):
    """<y, D y>_w for a local potential (no projectors)."""
    if len(s.dkb):
        raise ValueError("the closed form holds for local potentials only")
    b = Brute(s, approx="ipa")
    bg = reciprocal(s.at)
    g0 = np.asarray(s.g0)
    Q = np.asarray(s.q) + g0 @ bg
    total = 0.0
    for k in range(b.nks):
        npk = int(s.npw_k[k])
        mk = miller_from_index(s.nl_k[k, :npk], s.nr)
        uk = np.asarray(s.evc_k[k, :, :npk])
        kg = np.asarray(s.xk[k])[None, :] + mk @ bg
        vel = np.einsum("ng,gi->ni", np.abs(uk) ** 2, kg) @ Q       # Q.<u|(-i grad + k)|u>
        part = s.nbnd * 0.5 * float(Q @ Q) + np.sum(vel)
        # valence-valence (Pauli) term with energies from the explicit H_{k+q}
        h, mkq = b.hamiltonian(k, "kq")
        npq = len(mkq)
        ukq = np.asarray(s.evc_kq[k, :, :npq])
        ekq = np.real(np.einsum("mg,gh,mh->m", ukq.conj(), h, ukq))
        pos = {tuple(v): i for i, v in enumerate(mk.tolist())}
        shifted = np.zeros((s.nbnd, npq), dtype=np.complex128)
        for i, v in enumerate((mkq - g0[None, :]).tolist()):
            if tuple(v) in pos:
                shifted[:, i] = uk[:, pos[tuple(v)]]
        mel = shifted @ ukq.conj().T                                   # [n, m] = <m|e^{iG0r}|n>
        part -= np.sum(np.abs(mel) ** 2 * (ekq[None, :] - np.asarray(s.et_k[k])[:, None]))
        total += s.wk[k] * part
    return float(total)
