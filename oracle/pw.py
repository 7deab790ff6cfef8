"""Plane-wave primitives of the oracle and the Kohn-Sham Hamiltonian H_{k+q}.

The operators act on lattice-periodic parts of Bloch functions (Sec. 2.3, the
definition of operators with a wave-vector subscript).  The Hamiltonian at
k+q is the kinetic term 1/2 |k+q+G|^2 (diagonal in G), the local potential
(multiplication in real space, reached by FFT) and the separable non-local
projectors sum_p |beta_p> D_p <beta_p| (the pseudopotential setting of the
program summary; the paper does not write the projector form out).

Conventions: u(r) = Omega^-1/2 sum_G u(G) e^{iG.r}; grid point j at
r_j = sum_i (j_i/N_i) a_i, linear index (j1*N2+j2)*N3+j3; a plane wave of
Miller index m sits at the linear index of m mod N.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

FFT_WORKERS = 1  # the CPU baseline raises this to use all host cores


def reciprocal(at):
    return 2.0 * np.pi * np.linalg.inv(np.asarray(at, dtype=np.float64)).T


def miller_from_index(nl, nr):
    """Centred Miller indices (in [-N/2, N/2)) of linear grid indices."""
    n1, n2, n3 = (int(v) for v in nr)
    nl = np.asarray(nl, dtype=np.int64)
    i3 = nl % n3
    i2 = (nl // n3) % n2
    i1 = nl // (n2 * n3)
    m = np.stack([i1, i2, i3], axis=-1)
    n = np.array([n1, n2, n3])
    return np.where(m >= (n + 1) // 2, m - n, m)


class Cell:
    """Geometry, grid and G-vector tables of one instance."""

    def __init__(self, at, nr):
        self.at = np.asarray(at, dtype=np.float64)
        self.nr = tuple(int(v) for v in nr)
        self.ntot = int(np.prod(self.nr))
        self.omega = float(abs(np.linalg.det(self.at)))
        self.bg = reciprocal(self.at)

    # real space <-> coefficients -------------------------------------------
    def to_real(self, coef, nl):
        """Coefficients on a sphere (..., npw) -> real-space values (..., N)."""
        lead = coef.shape[:-1]
        g = np.zeros(lead + (self.ntot,), dtype=np.complex128)
        g[..., nl] = coef
        g = g.reshape(lead + self.nr)
        axes = tuple(range(len(lead), len(lead) + 3))
        f = sfft.ifftn(g, axes=axes, workers=FFT_WORKERS) * (self.ntot / math.sqrt(self.omega))
        return f.reshape(lead + (self.ntot,))

    def to_coef(self, f, nl):
        """Real-space values (..., N) -> coefficients on a sphere (..., npw):
        c(G) = Omega^1/2 N^-1 sum_j f(r_j) e^{-iG.r_j}."""
        lead = f.shape[:-1]
        axes = tuple(range(len(lead), len(lead) + 3))
        g = sfft.fftn(f.reshape(lead + self.nr), axes=axes, workers=FFT_WORKERS)
        g = g.reshape(lead + (self.ntot,)) * (math.sqrt(self.omega) / self.ntot)
        return g[..., nl]

    def gvec(self, nl, kvec):
        """Cartesian k + G of each linear index."""
        m = miller_from_index(nl, self.nr).astype(np.float64)
        return np.asarray(kvec)[None, :] + m @ self.bg

    def box_gvec(self):
        """Cartesian G of every grid index (centred Miller representative)."""
        return self.gvec(np.arange(self.ntot), np.zeros(3))

    def r_points(self):
        n1, n2, n3 = self.nr
        j1, j2, j3 = np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3, indexing="ij")
        f = np.stack([j1.ravel(), j2.ravel(), j3.ravel()], axis=1)
        return f @ self.at


class Hamiltonian:
    """H_{k+q} on one sphere: kinetic + local + separable projectors."""

    def __init__(self, cell: Cell, nl, kvec, vloc_r, vkb=None, dkb=None):
        self.cell = cell
        self.nl = np.asarray(nl, dtype=np.int64)
        g = cell.gvec(self.nl, kvec)
        self.kin = 0.5 * np.einsum("ij,ij->i", g, g)
        self.vloc = np.asarray(vloc_r, dtype=np.float64)
        self.vkb = None if vkb is None or len(dkb) == 0 else np.asarray(vkb)
        self.dkb = None if self.vkb is None else np.asarray(dkb, dtype=np.float64)

    def apply(self, x):
        """x: [..., npw] -> H x."""
        y = self.kin * x
        y = y + self.cell.to_coef(self.vloc * self.cell.to_real(x, self.nl), self.nl)
        if self.vkb is not None:
            b = x @ self.vkb.conj().T            # <beta_p | x>
            y = y + (b * self.dkb) @ self.vkb    # sum_p beta_p D_p <beta_p|x>
        return y
