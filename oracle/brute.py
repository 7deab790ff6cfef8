"""Explicit-matrix forms of the Liouvillian for tiny cells.

Nothing here goes through an FFT or through the matrix-free operators of
``liouvillian``: every Fourier transform is an explicit sum of exponentials
over grid points, so these matrices are an independent check of the
matrix-free oracle.

  * ``hamiltonian``: H_{GG'} = 1/2|k+q+G|^2 delta_GG' + V~(G-G')
    + sum_p beta_p(G) D_p beta_p*(G'), with V~(dG) = N^-1 sum_j V(r_j)
    e^{-i dG.r_j} (Sec. 2.3; exactly the grid operator, aliasing included).
  * ``transition_basis``: all eigenpairs of H_{k+q}; conduction states
    c >= nbnd give transitions t = (k, n, c).  D is diagonal there with
    entries eps_{c,k+q} - eps_{n,k} (eq. D_super-operator_2).
  * K in that basis (eqs. K_super-operator_2, SBR_charge-density_2,
    V_HXC_resp_1/2):  K_tt' = 4 w_t' <rho_t | v'[rho_t']>, with the pair
    density rho_t(r) = conj(u_nk(r)) u_{c,k+q}(r).
  * ``chi_direct``: solve (omega~ - L)(q,p) = (0,y) for the explicit L of
    eq. Liouvillian_SBR and return chi = (4/Omega) <y, q>_w
    (eqs. Liouvillian_eq_SBR_2, susceptibility_Q).
  * ``chi_casida``: the same resolvent through the Hermitian matrix
    D^1/2 (D + K~) D^1/2 (eliminating p from the SBR equations), with
    K~ = W^1/2 K W^-1/2.
  * ``explicit_operators``: D and K as dense matrices in the plane-wave basis
    of the batch, for driving the Lanczos recursion with matrices.
"""
from __future__ import annotations

import math

import numpy as np

from .pw import miller_from_index, reciprocal


class Brute:
    def __init__(self, s, approx="tddft"):
        self.s = s
        self.approx = approx
        self.at = np.asarray(s.at, dtype=np.float64)
        self.nr = tuple(int(v) for v in s.nr)
        self.ntot = int(np.prod(self.nr))
        self.omega = float(abs(np.linalg.det(self.at)))
        self.bg = reciprocal(self.at)
        self.nks = int(np.asarray(s.xk).shape[0])
        self.nbnd = int(np.asarray(s.et_k).shape[1])
        n1, n2, n3 = self.nr
        j = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
        self.jfrac = j / np.array(self.nr)[None, :]          # fractional grid coordinates
        self.q = np.asarray(s.q, dtype=np.float64)
        self.g0 = np.asarray(s.g0, dtype=np.int64)
        self.Q = self.q + self.g0 @ self.bg
        self.wk = np.asarray(s.wk, dtype=np.float64)

    # ------------------------------------------------------------ Fourier sums
    def _phase(self, mill):
        """e^{i G.r_j} = exp(2 pi i sum_a m_a j_a / N_a): [ntot, len(mill)]."""
        return np.exp(2j * np.pi * (self.jfrac @ np.asarray(mill, dtype=np.float64).T))

    def miller(self, nl):
        return miller_from_index(nl, self.nr)

    def orbital_r(self, coef, mill):
        """u(r_j) = Omega^-1/2 sum_G u(G) e^{iG.r_j}; coef [..., npw]."""
        return (coef @ self._phase(mill).T) / math.sqrt(self.omega)

    # ------------------------------------------------------------ Hamiltonian
    def hamiltonian(self, k, which="kq"):
        s = self.s
        if which == "kq":
            npw = int(s.npw_kq[k]); nl = s.nl_kq[k, :npw]; kvec = np.asarray(s.xk[k]) + self.q
        else:
            npw = int(s.npw_k[k]); nl = s.nl_k[k, :npw]; kvec = np.asarray(s.xk[k])
        m = self.miller(nl)
        g = kvec[None, :] + m @ self.bg
        dm = m[:, None, :] - m[None, :, :]
        flat = dm.reshape(-1, 3)
        uniq, inv = np.unique(flat, axis=0, return_inverse=True)
        vtil = (np.asarray(s.vloc_r) @ np.conj(self._phase(uniq))) / self.ntot
        h = vtil[inv.ravel()].reshape(npw, npw).astype(np.complex128)
        h[np.diag_indices(npw)] += 0.5 * np.einsum("ij,ij->i", g, g)
        if which == "kq" and len(s.dkb):
            b = np.asarray(s.vkb_kq[k, :, :npw])
            h += b.T @ (np.asarray(s.dkb)[:, None] * b.conj())
        elif which == "k" and len(s.dkb):
            raise ValueError("projectors at k are not part of the inputs")
        return h, m

    # ----------------------------------------------------------- transitions
    def transition_basis(self):
        """Transitions t = (k, n, c) with their energies, pair densities on the
        grid and right-hand-side components y_t = <c, k+q | y_nk>."""
        s = self.s
        self.trans = []
        rho, dE, yt, wt = [], [], [], []
        for k in range(self.nks):
            h, mkq = self.hamiltonian(k, "kq")
            e, c = np.linalg.eigh(h)
            cond = c[:, self.nbnd:]
            ec = e[self.nbnd:]
            npk = int(s.npw_k[k])
            mk = self.miller(s.nl_k[k, :npk])
            uk = np.asarray(s.evc_k[k, :, :npk])
            ur = self.orbital_r(uk, mk)                          # [nbnd, N]
            cr = self.orbital_r(cond.T, mkq)                     # [ncond, N]
            # e^{iG0.r} u_nk expressed on the k+q sphere: coefficient at G' is u(G'-G0)
            pos = {tuple(v): i for i, v in enumerate(mk.tolist())}
            shifted = np.zeros((self.nbnd, len(mkq)), dtype=np.complex128)
            for i, v in enumerate((mkq - self.g0[None, :]).tolist()):
                if tuple(v) in pos:
                    shifted[:, i] = uk[:, pos[tuple(v)]]
            yc = shifted @ np.conj(cond)                          # [nbnd, ncond]: <c|e^{iG0r}u_n>
            for n in range(self.nbnd):
                for ci in range(cond.shape[1]):
                    self.trans.append((k, n, ci))
                    dE.append(ec[ci] - s.et_k[k, n])
                    yt.append(yc[n, ci])
                    wt.append(self.wk[k])
                rho.append(np.conj(ur[n])[None, :] * cr)          # [ncond, N]
        self.rho = np.concatenate(rho, axis=0)
        self.dE = np.array(dE)
        self.yt = np.array(yt)
        self.wt = np.array(wt)
        return self

    def _kernel_matrix(self):
        """<rho_t | v'[rho_t']> = Omega sum_G 4pi/|q+G|^2 conj(rho_t(G)) rho_t'(G)
        + (Omega/N) sum_j f_xc(r_j) conj(rho_t(r_j)) rho_t'(r_j)."""
        nt = len(self.dE)
        if self.approx == "ipa":
            return np.zeros((nt, nt), dtype=np.complex128)
        c = np.stack(np.meshgrid(*[np.where(np.arange(n) >= (n + 1) // 2, np.arange(n) - n, np.arange(n))
                                   for n in self.nr], indexing="ij"), -1).reshape(-1, 3)
        qg = self.q[None, :] + c @ self.bg
        vh = 4.0 * np.pi / np.einsum("ij,ij->i", qg, qg)
        rho_g = (self.rho @ np.conj(self._phase(c))) / self.ntot       # explicit DFT
        kmat = self.omega * (np.conj(rho_g) * vh[None, :]) @ rho_g.T
        if self.approx == "tddft":
            f = np.asarray(self.s.fxc_r)
            kmat += (self.omega / self.ntot) * (np.conj(self.rho) * f[None, :]) @ self.rho.T
        return kmat

    def matrices(self):
        if not hasattr(self, "rho"):
            self.transition_basis()
        self.Kc = self._kernel_matrix()                 # <rho_t|v'[rho_t']>
        self.Kmat = 4.0 * self.Kc * self.wt[None, :]    # K_tt' = 4 w_t' <rho_t|v'rho_t'>
        sw = np.sqrt(self.wt)
        self.Ksym = 4.0 * sw[:, None] * self.Kc * sw[None, :]
        return self

    # ------------------------------------------------------------------- chi
    def chi_direct(self, omega, eta):
        if not hasattr(self, "Kmat"):
            self.matrices()
        nt = len(self.dE)
        D = np.diag(self.dE)
        L = np.zeros((2 * nt, 2 * nt), dtype=np.complex128)
        L[:nt, nt:] = D
        L[nt:, :nt] = D + self.Kmat
        rhs = np.concatenate([np.zeros(nt), self.yt])
        out = []
        for w in omega:
            sol = np.linalg.solve((w + 1j * eta) * np.eye(2 * nt) - L, rhs)
            out.append(np.sum(self.wt * np.conj(self.yt) * sol[:nt]))
        return (4.0 / self.omega) * np.array(out)

    def casida(self):
        if not hasattr(self, "Ksym"):
            self.matrices()
        sd = np.sqrt(self.dE)
        m = sd[:, None] * (np.diag(self.dE) + self.Ksym) * sd[None, :]
        lam, vec = np.linalg.eigh(0.5 * (m + m.conj().T))
        amp = vec.conj().T @ (sd * np.sqrt(self.wt) * self.yt)
        return lam, amp

    def chi_casida(self, omega, eta):
        lam, amp = self.casida()
        w = np.asarray(omega)[:, None] + 1j * eta
        return (4.0 / self.omega) * np.sum(np.abs(amp)[None, :] ** 2 / (w * w - lam[None, :]), axis=1)

    # -------------------------------------------- plane-wave-basis operators
    def explicit_operators(self):
        """Dense D and K acting on the flattened batch (k, n, G in k+q sphere),
        built from explicit Fourier sums.  Returns (D, K, sizes)."""
        s = self.s
        blocks, offs, sizes = [], [0], []
        phases, pcs, urs, mills = [], [], [], []
        for k in range(self.nks):
            h, mkq = self.hamiltonian(k, "kq")
            npw = h.shape[0]
            ukq = np.asarray(s.evc_kq[k, :, :npw])
            pc = np.eye(npw) - ukq.T @ ukq.conj()
            for n in range(self.nbnd):
                blocks.append(pc @ (h - s.et_k[k, n] * np.eye(npw)))
                offs.append(offs[-1] + npw)
                sizes.append(npw)
            npk = int(s.npw_k[k])
            mk = self.miller(s.nl_k[k, :npk])
            urs.append(self.orbital_r(np.asarray(s.evc_k[k, :, :npk]), mk))
            phases.append(self._phase(mkq))
            pcs.append(pc)
            mills.append(mkq)
        ntot = offs[-1]
        D = np.zeros((ntot, ntot), dtype=np.complex128)
        for i, b in enumerate(blocks):
            D[offs[i]:offs[i + 1], offs[i]:offs[i + 1]] = b
        K = np.zeros((ntot, ntot), dtype=np.complex128)
        if self.approx != "ipa":
            # x -> n'(r_j): A [N, ntot]
            A = np.zeros((self.ntot, ntot), dtype=np.complex128)
            i = 0
            for k in range(self.nks):
                for n in range(self.nbnd):
                    A[:, offs[i]:offs[i + 1]] = (4.0 * self.wk[k] / math.sqrt(self.omega)) * \
                        np.conj(urs[k][n])[:, None] * phases[k]
                    i += 1
            c = np.stack(np.meshgrid(*[np.where(np.arange(n) >= (n + 1) // 2, np.arange(n) - n, np.arange(n))
                                       for n in self.nr], indexing="ij"), -1).reshape(-1, 3)
            E = self._phase(c)                                   # [N, N] e^{iG.r_j}
            qg = self.q[None, :] + c @ self.bg
            vh = 4.0 * np.pi / np.einsum("ij,ij->i", qg, qg)
            B = E @ (vh[:, None] * np.conj(E).T) / self.ntot      # Hartree, n(r) -> v_H(r)
            if self.approx == "tddft":
                B = B + np.diag(np.asarray(s.fxc_r))
            V = B @ A                                             # x -> v'(r_j)
            i = 0
            for k in range(self.nks):
                for n in range(self.nbnd):
                    # coefficient on the k+q sphere of v' u_nk, then P_c
                    C = (math.sqrt(self.omega) / self.ntot) * np.conj(phases[k]).T * urs[k][n][None, :]
                    K[offs[i]:offs[i + 1], :] = pcs[k] @ (C @ V)
                    i += 1
        return D, K, offs

    def flatten(self, x):
        s = self.s
        parts = []
        for k in range(self.nks):
            for n in range(self.nbnd):
                parts.append(x[k, n, :int(s.npw_kq[k])])
        return np.concatenate(parts)

    def unflatten(self, v):
        s = self.s
        npwx = np.asarray(s.nl_kq).shape[1]
        out = np.zeros((self.nks, self.nbnd, npwx), dtype=np.complex128)
        o = 0
        for k in range(self.nks):
            npw = int(s.npw_kq[k])
            for n in range(self.nbnd):
                out[k, n, :npw] = v[o:o + npw]
                o += npw
        return out
