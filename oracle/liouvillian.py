"""The Liouvillian in the standard batch representation (Sec. 2.4).

    L_q = [[0, D], [D + K, 0]]                         (eq. Liouvillian_SBR)
    (D x)_nk = P_c^{k+q} (H_{k+q} - eps_nk) x_nk       (eq. D_super-operator_2)
    (K x)_nk = P_c^{k+q} v'_HXC[n'[x]] u_nk            (eq. K_super-operator_2)
    n'(r)    = 4 sum_k w_k sum_n u*_nk(r) x_nk(r)      (eq. SBR_charge-density_2)
    v'_H(G)  = 4 pi n'(G) / |q+G|^2                    (eq. V_HXC_resp_2)
    v'_xc(r) = f_xc(r) n'(r)       (adiabatic kernel, eq. V_HXC_resp_1)
    P_c^k    = 1 - sum_n |u_nk><u_nk|                  (Sec. 2.3)
    y_nk     = P_c^{k+q} e^{iG0.r} u_nk                (eq. RHS_of_Liouville_eq)

Readings of points the paper leaves open (each is listed in the design notes):
  * P_c is applied to the total output of D; on the conduction subspace this
    equals P_c (H - eps) P_c because H_{k+q} commutes with P_c^{k+q}.
  * Sums over k carry the weights w_k (sum w_k = 1); every inner product is
    <a,b>_w = sum_k w_k sum_n sum_G conj(a_nkG) b_nkG, which keeps K Hermitian.
  * The Hartree sum runs over every G of the FFT box (centred Miller range).
  * approximation: "tddft" (Hartree + f_xc), "rpa" (Hartree only),
    "ipa" (K = 0), as the three levels of Sec. 3.2.

Batches are arrays [nks, nbnd, npwx] (complex128) on the k+q spheres, with
zeros beyond npw_kq -- the layout the library takes.
"""
from __future__ import annotations

import numpy as np

from .pw import Cell, Hamiltonian


class Liouvillian:
    def __init__(self, s, approx: str = "tddft"):
        if approx not in ("tddft", "rpa", "ipa"):
            raise ValueError(approx)
        self.approx = approx
        self.cell = c = Cell(s.at, s.nr)
        self.nks = int(np.asarray(s.xk).shape[0])
        self.nbnd = int(np.asarray(s.et_k).shape[1])
        self.npwx = int(np.asarray(s.nl_kq).shape[1])
        self.wk = np.asarray(s.wk, dtype=np.float64)
        self.q = np.asarray(s.q, dtype=np.float64)
        self.g0 = np.asarray(s.g0, dtype=np.int64)
        self.Q = self.q + self.g0.astype(np.float64) @ c.bg
        self.eps = np.asarray(s.et_k, dtype=np.float64)
        self.npw_k = np.asarray(s.npw_k)
        self.npw_kq = np.asarray(s.npw_kq)
        self.nl_k = [np.asarray(s.nl_k[k, :self.npw_k[k]], dtype=np.int64) for k in range(self.nks)]
        self.nl_kq = [np.asarray(s.nl_kq[k, :self.npw_kq[k]], dtype=np.int64) for k in range(self.nks)]
        self.u_k = [np.asarray(s.evc_k[k, :, :self.npw_k[k]]) for k in range(self.nks)]
        self.u_kq = [np.asarray(s.evc_kq[k, :, :self.npw_kq[k]]) for k in range(self.nks)]
        dkb = np.asarray(s.dkb, dtype=np.float64)
        self.ham = []
        for k in range(self.nks):
            vkb = np.asarray(s.vkb_kq[k, :, :self.npw_kq[k]]) if len(dkb) else None
            self.ham.append(Hamiltonian(c, self.nl_kq[k], np.asarray(s.xk[k]) + self.q,
                                        s.vloc_r, vkb, dkb))
        self.fxc = np.asarray(s.fxc_r, dtype=np.float64)
        # valence orbitals at k in real space, u_nk(r_j)
        self.u_r = [c.to_real(self.u_k[k], self.nl_k[k]) for k in range(self.nks)]
        # Hartree kernel 4 pi / |q+G|^2 over the whole FFT box
        qg = c.box_gvec() + self.q[None, :]
        q2 = np.einsum("ij,ij->i", qg, qg)
        if np.any(q2 == 0.0):
            raise ValueError("q + G = 0 is on the grid: the Hartree kernel is singular")
        self.vh_kernel = 4.0 * np.pi / q2

    # ---------------------------------------------------------------- helpers
    def blocks(self, x):
        return [x[k, :, :self.npw_kq[k]] for k in range(self.nks)]

    def pack(self, blocks):
        out = np.zeros((self.nks, self.nbnd, self.npwx), dtype=np.complex128)
        for k, b in enumerate(blocks):
            out[k, :, :self.npw_kq[k]] = b
        return out

    def inner(self, a, b):
        """<a,b>_w = sum_k w_k sum_n sum_G conj(a) b."""
        return complex(sum(self.wk[k] * np.vdot(a[k], b[k]) for k in range(self.nks)))

    def pc(self, k, x):
        """P_c^{k+q} x for x [nbnd, npw_kq]: x - sum_m u_m <u_m, x>."""
        u = self.u_kq[k]
        return x - (x @ u.conj().T) @ u

    def project_c(self, x):
        """P_c^{k+q} on every block of a batch."""
        return self.pack([self.pc(k, b) for k, b in enumerate(self.blocks(x))])

    # ------------------------------------------------------------- operators
    def apply_h(self, x):
        """H_{k+q} on every band of a batch (no projector, no eps)."""
        return self.pack([self.ham[k].apply(b) for k, b in enumerate(self.blocks(x))])

    def apply_D(self, x):
        out = []
        for k, b in enumerate(self.blocks(x)):
            hb = self.ham[k].apply(b) - self.eps[k][:, None] * b
            out.append(self.pc(k, hb))
        return self.pack(out)

    def density(self, x):
        """n'(r) = 4 sum_k w_k sum_n conj(u_nk(r)) x_nk(r)."""
        n = np.zeros(self.cell.ntot, dtype=np.complex128)
        for k, b in enumerate(self.blocks(x)):
            xr = self.cell.to_real(b, self.nl_kq[k])
            n += 4.0 * self.wk[k] * np.sum(np.conj(self.u_r[k]) * xr, axis=0)
        return n

    def hxc_potential(self, n):
        """v'(r_j) = sum_G 4 pi n(G)/|q+G|^2 e^{iG.r_j} + f_xc(r_j) n(r_j),
        with n(G) = N^-1 sum_j n(r_j) e^{-iG.r_j}."""
        c = self.cell
        if self.approx == "ipa":
            return np.zeros_like(n)
        ng = np.fft.fftn(n.reshape(c.nr)).ravel() / c.ntot
        v = np.fft.ifftn((self.vh_kernel * ng).reshape(c.nr)).ravel() * c.ntot
        if self.approx == "tddft":
            v = v + self.fxc * n
        return v

    def apply_K(self, x):
        if self.approx == "ipa":
            return np.zeros_like(x)
        v = self.hxc_potential(self.density(x))
        out = []
        for k in range(self.nks):
            f = self.cell.to_coef(v[None, :] * self.u_r[k], self.nl_kq[k])
            out.append(self.pc(k, f))
        return self.pack(out)

    def apply_DK(self, x):
        return self.apply_D(x) + self.apply_K(x)

    def apply_L(self, upper, lower):
        """L (upper, lower) = (D lower, (D+K) upper)."""
        return self.apply_D(lower), self.apply_DK(upper)

    def rhs(self):
        """y_nk = P_c^{k+q} [e^{iG0.r} u_nk(r)] on the k+q sphere; the
        components of the shifted orbital outside that sphere are dropped."""
        c = self.cell
        n1, n2, n3 = c.nr
        j1, j2, j3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
        ph = np.exp(2j * np.pi * (self.g0[0] * j1 / n1 + self.g0[1] * j2 / n2 + self.g0[2] * j3 / n3)).ravel()
        out = []
        for k in range(self.nks):
            f = c.to_coef(ph[None, :] * self.u_r[k], self.nl_kq[k])
            out.append(self.pc(k, f))
        return self.pack(out)
