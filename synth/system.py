"""Synthetic crystal, plane-wave spheres and a seeded ground state.

Everything here is input preparation (the ground-state step that precedes the
linear-response calculation in paper Sec. 3.1).  The model is deliberately
simple: a local potential made of Gaussian wells, optional separable
Kleinman-Bylander projectors with Gaussian radial parts (s and p channels),
and the lowest ``nbnd`` eigenpairs of the resulting Hamiltonian at every k and
k+q.  The adiabatic LDA kernel is evaluated at the resulting density.
"""
from __future__ import annotations

import dataclasses
import logging
import math
import multiprocessing as mp
import os
from typing import Optional

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

_WORKERS = -1
_log = logging.getLogger(__name__)


# --------------------------------------------------------------------------
# geometry and plane-wave spheres
# --------------------------------------------------------------------------

def reciprocal(at: np.ndarray) -> np.ndarray:
    """Rows b_j with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(at, dtype=np.float64)).T


def centred(n: int) -> np.ndarray:
    """Integers 0..n-1 mapped to their centred representative in [-n/2, n/2)."""
    i = np.arange(n)
    return np.where(i < (n + 1) // 2, i, i - n) if n % 2 else np.where(i < n // 2, i, i - n)


def linear_index(mill: np.ndarray, nr) -> np.ndarray:
    n1, n2, n3 = (int(v) for v in nr)
    m = np.asarray(mill, dtype=np.int64)
    return (((m[:, 0] % n1) * n2 + (m[:, 1] % n2)) * n3 + (m[:, 2] % n3)).astype(np.int64)


def sphere_miller(at, nr, kvec, ecut) -> np.ndarray:
    """Miller indices m with 0.5 |k + m.bg|^2 <= ecut, sorted by kinetic energy
    (ties broken by linear grid index).  Raises if the sphere does not fit in
    the centred FFT box."""
    bg = reciprocal(at)
    kvec = np.asarray(kvec, dtype=np.float64)
    gmax = math.sqrt(2.0 * ecut) + np.linalg.norm(kvec)
    # a box that surely contains the sphere
    lim = [int(math.ceil(gmax * np.linalg.norm(np.asarray(at)[i]) / (2 * np.pi))) + 1 for i in range(3)]
    r = [np.arange(-l, l + 1) for l in lim]
    m1, m2, m3 = np.meshgrid(*r, indexing="ij")
    mill = np.stack([m1.ravel(), m2.ravel(), m3.ravel()], axis=1)
    g = kvec[None, :] + mill @ bg
    kin = 0.5 * np.einsum("ij,ij->i", g, g)
    sel = kin <= ecut
    mill, kin = mill[sel], kin[sel]
    nr = np.asarray(nr)
    lo = -(nr // 2)
    hi = (nr - 1) // 2
    if np.any(mill < lo[None, :]) or np.any(mill > hi[None, :]):
        raise ValueError("plane-wave sphere does not fit in the FFT box")
    idx = linear_index(mill, nr)
    order = np.lexsort((idx, np.round(kin, 12)))
    return mill[order]


def mp_kpoints(at, nk, shift) -> np.ndarray:
    """Monkhorst-Pack style mesh nk[0] x nk[1] x nk[2] with fractional shift
    (each component in [0,1) of one mesh step), folded to [-1/2, 1/2)."""
    bg = reciprocal(at)
    ks = []
    for i in range(nk[0]):
        for j in range(nk[1]):
            for l in range(nk[2]):
                f = np.array([(i + shift[0]) / nk[0], (j + shift[1]) / nk[1], (l + shift[2]) / nk[2]])
                f = f - np.floor(f + 0.5)
                ks.append(f @ bg)
    return np.array(ks, dtype=np.float64)


# --------------------------------------------------------------------------
# potentials and projectors
# --------------------------------------------------------------------------

def _gvec_box(at, nr):
    bg = reciprocal(at)
    c = [centred(int(n)) for n in nr]
    m1, m2, m3 = np.meshgrid(*c, indexing="ij")
    mill = np.stack([m1, m2, m3], axis=-1).astype(np.float64)
    return mill @ bg  # [N1,N2,N3,3]


def gaussian_wells_r(at, nr, tau_cart, depth, width) -> np.ndarray:
    """V(r_j) = -depth * sum_a sum_R exp(-|r_j - tau_a - R|^2 / (2 width^2)),
    evaluated through its Fourier series on the FFT box (the Gaussian decays
    below 1e-16 well inside the box for the grids used).  Returns the real
    grid in linear-index order."""
    at = np.asarray(at, dtype=np.float64)
    omega = abs(np.linalg.det(at))
    g = _gvec_box(at, nr)
    g2 = np.einsum("...i,...i->...", g, g)
    pref = -depth * (2.0 * np.pi * width * width) ** 1.5 / omega
    vg = np.zeros(g2.shape, dtype=np.complex128)
    for t in np.asarray(tau_cart, dtype=np.float64):
        vg += pref * np.exp(-0.5 * g2 * width * width) * np.exp(-1j * (g @ t))
    # drop the unpaired Nyquist planes so the real-space field is real
    for ax, n in enumerate(nr):
        if int(n) % 2 == 0:
            sl = [slice(None)] * 3
            sl[ax] = int(n) // 2
            vg[tuple(sl)] = 0.0
    n3 = int(np.prod(nr))
    vr = np.fft.ifftn(vg) * n3
    return np.ascontiguousarray(vr.real).ravel()


def kb_projectors(at, mill, kvec, tau_cart, radii, coefs=None) -> np.ndarray:
    """Separable projectors on the sphere of kvec: for each atom one s and
    three p channels,
        beta_s(g)   = Omega^-1/2 c_s exp(-g^2 r_s^2/2) exp(-i g.tau)
        beta_p_a(g) = -i Omega^-1/2 c_p g_a exp(-g^2 r_p^2/2) exp(-i g.tau)
    with g = kvec + G and c chosen so that each has unit continuum norm.
    ``radii`` is [nat, 2] (r_s, r_p).  Returns [4*nat, npw] complex."""
    at = np.asarray(at, dtype=np.float64)
    omega = abs(np.linalg.det(at))
    g = np.asarray(kvec)[None, :] + np.asarray(mill, dtype=np.float64) @ reciprocal(at)
    g2 = np.einsum("ij,ij->i", g, g)
    out = []
    for a, t in enumerate(np.asarray(tau_cart, dtype=np.float64)):
        rs, rp = radii[a]
        cs = math.sqrt(8.0 * math.pi ** 1.5 * rs ** 3)
        cp = math.sqrt(16.0 * math.pi ** 1.5 * rp ** 5)
        ph = np.exp(-1j * (g @ t)) / math.sqrt(omega)
        out.append(cs * np.exp(-0.5 * g2 * rs * rs) * ph)
        for ax in range(3):
            out.append(-1j * cp * g[:, ax] * np.exp(-0.5 * g2 * rp * rp) * ph)
    return np.array(out, dtype=np.complex128)


# --------------------------------------------------------------------------
# adiabatic LDA kernels
# --------------------------------------------------------------------------

_RHO_MIN = 1e-10


def x_lda_fxc(n: np.ndarray) -> np.ndarray:
    """Exchange-only LDA kernel d^2(n eps_x)/dn^2 = -(1/3)(3/pi)^(1/3) n^(-2/3);
    zero where n < 1e-10 bohr^-3."""
    n = np.asarray(n, dtype=np.float64)
    out = np.zeros_like(n)
    m = n >= _RHO_MIN
    out[m] = -(1.0 / 3.0) * (3.0 / math.pi) ** (1.0 / 3.0) * n[m] ** (-2.0 / 3.0)
    return out


def pz_lda_fxc(n: np.ndarray) -> np.ndarray:
    """Perdew-Zunger 1981 LDA (unpolarised) kernel d^2(n eps_xc)/dn^2 in Ha bohr^3.

    With r_s = (3/(4 pi n))^(1/3) one has d/dn = -(r_s/(3n)) d/dr_s, giving
    f_c = (r_s^2 eps_c'' - 2 r_s eps_c') / (9 n).  Correlation parameters from
    Perdew & Zunger, Phys. Rev. B 23, 5048 (1981), Hartree units."""
    n = np.asarray(n, dtype=np.float64)
    out = x_lda_fxc(n)
    m = n >= _RHO_MIN
    nn = n[m]
    rs = (3.0 / (4.0 * math.pi * nn)) ** (1.0 / 3.0)
    gam, b1, b2 = -0.1423, 1.0529, 0.3334
    A, B, C, D = 0.0311, -0.048, 0.0020, -0.0116
    hi = rs >= 1.0
    e1 = np.empty_like(rs)
    e2 = np.empty_like(rs)
    r = rs[hi]
    den = 1.0 + b1 * np.sqrt(r) + b2 * r
    d1 = b1 / (2.0 * np.sqrt(r)) + b2
    d2 = -b1 / (4.0 * r ** 1.5)
    e1[hi] = -gam * d1 / den ** 2
    e2[hi] = -gam * d2 / den ** 2 + 2.0 * gam * d1 ** 2 / den ** 3
    r = rs[~hi]
    e1[~hi] = A / r + C * (np.log(r) + 1.0) + D
    e2[~hi] = -A / r ** 2 + C / r
    _ = B
    out[m] += (rs * rs * e2 - 2.0 * rs * e1) / (9.0 * nn)
    return out


# --------------------------------------------------------------------------
# ground-state Hamiltonian (input preparation only)
# --------------------------------------------------------------------------

class _Ham:
    """Kohn-Sham Hamiltonian of the synthetic model on one sphere."""

    def __init__(self, at, nr, vloc_r, mill, kvec, vkb=None, dkb=None):
        self.nr = tuple(int(v) for v in nr)
        self.mill = np.asarray(mill)
        self.idx = linear_index(self.mill, self.nr)
        g = np.asarray(kvec)[None, :] + self.mill.astype(np.float64) @ reciprocal(at)
        self.kin = 0.5 * np.einsum("ij,ij->i", g, g)
        self.v = np.asarray(vloc_r, dtype=np.float64).reshape(self.nr)
        self.vkb = vkb
        self.dkb = dkb

    def dense(self) -> np.ndarray:
        n1, n2, n3 = self.nr
        vg = np.fft.fftn(self.v) / (n1 * n2 * n3)
        dm = self.mill[:, None, :] - self.mill[None, :, :]
        h = vg[dm[..., 0] % n1, dm[..., 1] % n2, dm[..., 2] % n3].astype(np.complex128)
        h[np.diag_indices_from(h)] += self.kin
        if self.vkb is not None and len(self.dkb):
            # sum_p |beta_p> D_p <beta_p|: H_GG' += sum_p beta_p(G) D_p conj(beta_p(G'))
            h += (self.vkb.T * self.dkb[None, :]) @ self.vkb.conj()
        return 0.5 * (h + h.conj().T)

    def apply(self, x: np.ndarray) -> np.ndarray:
        """x: [npw, nb] -> H x."""
        n1, n2, n3 = self.nr
        nb = x.shape[1]
        grid = np.zeros((nb, n1 * n2 * n3), dtype=np.complex128)
        grid[:, self.idx] = x.T
        grid = grid.reshape(nb, n1, n2, n3)
        f = sfft.ifftn(grid, axes=(1, 2, 3), workers=_WORKERS, overwrite_x=True)
        f *= self.v[None]
        f = sfft.fftn(f, axes=(1, 2, 3), workers=_WORKERS, overwrite_x=True).reshape(nb, -1)
        y = f[:, self.idx].T + self.kin[:, None] * x
        if self.vkb is not None and len(self.dkb):
            y += self.vkb.T @ (self.dkb[:, None] * (self.vkb.conj() @ x))
        return y


def _lowest_eigenpairs(ham: _Ham, nev: int, x0: Optional[np.ndarray] = None,
                       tol: float = 1e-10, maxit: int = 2000):
    """Lowest nev eigenpairs of a Hermitian plane-wave Hamiltonian; raises if
    the block Davidson iteration leaves a wanted residual norm above 10 tol
    (an unconverged valence set would make every reference built on it
    differ from a converged one)."""
    npw = len(ham.kin)
    if npw <= 2600 or x0 is None:
        h = ham.dense()
        w, v = sla.eigh(h, subset_by_index=[0, nev - 1], driver="evr")
        return w, v
    # block Davidson with a kinetic preconditioner, started from x0; large
    # blocks (the 128 bands of the 96^3 cell, whose top bands lie within
    # 0.3 mHa of each other) restart thick: the Ritz block and the last
    # corrections
    nb = x0.shape[1]
    thick = nev > 64
    x, _ = np.linalg.qr(x0)
    hx = ham.apply(x)
    basis, hbasis = x, hx
    last_t = None
    for _it in range(maxit):
        hs = basis.conj().T @ hbasis
        hs = 0.5 * (hs + hs.conj().T)
        w, c = np.linalg.eigh(hs)
        w, c = w[:nb], c[:, :nb]
        x = basis @ c
        hx = hbasis @ c
        res = hx - x * w[None, :]
        rn = np.linalg.norm(res, axis=0)
        if _it % 20 == 0:
            _log.debug("davidson it %d basis %d residual %.2e", _it, basis.shape[1], np.max(rn[:nev]))
        if np.max(rn[:nev]) < tol:
            break
        act = rn > tol * 0.1
        t = res[:, act] / (ham.kin[:, None] - w[None, act] + 1.0)
        # orthogonalise the corrections against the current Ritz block
        if basis.shape[1] + t.shape[1] > 4 * nb:
            if thick and last_t is not None:
                q, _ = np.linalg.qr(np.concatenate([x, last_t], axis=1))
                basis, hbasis = q, ham.apply(q)
            else:
                basis, hbasis = x, hx
        t -= basis @ (basis.conj().T @ t)
        t -= basis @ (basis.conj().T @ t)
        t, r = np.linalg.qr(t)
        keep = np.abs(np.diag(r)) > 1e-12
        t = t[:, keep]
        if t.shape[1] == 0:
            break
        ht = ham.apply(t)
        if thick:
            last_t = t
        basis = np.concatenate([basis, t], axis=1)
        hbasis = np.concatenate([hbasis, ht], axis=1)
    # final Rayleigh-Ritz on an exactly orthonormal block
    q, _ = np.linalg.qr(x)
    hq = ham.apply(q)
    hs = q.conj().T @ hq
    w, c = np.linalg.eigh(0.5 * (hs + hs.conj().T))
    v = (q @ c)[:, :nev]
    rn = np.linalg.norm(ham.apply(v) - v * w[None, :nev], axis=0)
    if np.max(rn) > 10 * tol:
        raise RuntimeError(f"block Davidson: residual {np.max(rn):.1e} after {maxit} iterations")
    return w[:nev], v


def _solve_sphere(args):
    """Lowest eigenpairs on one sphere (one k or k+q point)."""
    at, nr, vloc, kv, kbase, ecut, tau, radii, dkb, nev, tol, union_g0 = args
    kb_on = radii is not None
    bg = reciprocal(at)
    mill = sphere_miller(at, nr, kv, ecut)
    if union_g0 is not None:
        shifted = sphere_miller(at, nr, kbase, ecut) + np.asarray(union_g0)[None, :]
        allm = np.concatenate([mill, shifted])
        _, first = np.unique(linear_index(allm, nr), return_index=True)
        allm = allm[np.sort(first)]
        gg = kv[None, :] + allm @ bg
        kin = 0.5 * np.einsum("ij,ij->i", gg, gg)
        order = np.lexsort((linear_index(allm, nr), np.round(kin, 12)))
        mill = allm[order]
    vkb = kb_projectors(at, mill, kv, tau, radii) if kb_on else None
    ham = _Ham(at, nr, vloc, mill, kv, vkb, dkb)
    x0 = None
    if len(mill) > 2600:
        # start from the eigenvectors of a low-cutoff Hamiltonian
        lo = ecut
        while True:
            lo *= 0.7
            mlo = sphere_miller(at, nr, kv, lo)
            if len(mlo) <= 2200:
                break
        vlo = kb_projectors(at, mlo, kv, tau, radii) if kb_on else None
        hlo = _Ham(at, nr, vloc, mlo, kv, vlo, dkb)
        nbuf = 24 if nev > 64 else 8   # buffer vectors of the block
        _, vl = sla.eigh(hlo.dense(), subset_by_index=[0, nev + nbuf - 1], driver="evr")
        pos = {int(i): j for j, i in enumerate(linear_index(mill, nr))}
        x0 = np.zeros((len(mill), nev + nbuf), dtype=np.complex128)
        rows = np.array([pos[int(i)] for i in linear_index(mlo, nr)])
        x0[rows] = vl
    w, v = _lowest_eigenpairs(ham, nev, x0, tol=tol)
    # fix the gauge: largest coefficient of each band real positive
    for b in range(v.shape[1]):
        j = np.argmax(np.abs(v[:, b]))
        v[:, b] *= np.conj(v[j, b]) / abs(v[j, b])
    return mill, v, w, vkb


def _random_sphere(args):
    """Sphere and projectors of one k or k+q point with random orthonormal
    orbitals instead of eigenstates (operator-level tests of large cells,
    where diagonalisation is out of reach).  The orbital energies are placed
    below a lower bound of the Hamiltonian on the sphere, so that D stays
    positive definite on the conduction manifold."""
    at, nr, vloc, kv, kbase, ecut, tau, radii, dkb, nev, tol, union_g0, seed = args
    mill = sphere_miller(at, nr, kv, ecut)
    vkb = kb_projectors(at, mill, kv, tau, radii) if radii is not None else None
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((len(mill), nev)) + 1j * rng.standard_normal((len(mill), nev))
    v, _ = np.linalg.qr(x)
    lower = float(vloc.min())
    if vkb is not None:
        lower += float(np.sum(np.minimum(dkb, 0.0) * np.sum(np.abs(vkb) ** 2, axis=1)))
    w = lower - 0.5 - 0.05 * np.arange(nev)[::-1]
    return mill, v, w, vkb


def _pool_init():
    global _WORKERS, _LIMITER
    _WORKERS = 1
    from threadpoolctl import threadpool_limits
    _LIMITER = threadpool_limits(1)


def _run_jobs(jobs):
    """Solve the spheres, in worker processes when there are several large ones."""
    if len(jobs[0]) == 13:
        return [_random_sphere(j) for j in jobs]
    big = sum(1 for j in jobs if sphere_miller(j[0], j[1], j[3], j[5]).shape[0] > 2600)
    ncpu = min(len(os.sched_getaffinity(0)), 16)
    if big < 2 or ncpu < 2:
        return [_solve_sphere(j) for j in jobs]
    # spawned workers: the caller may already hold a GPU context, which a
    # forked child must not inherit
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(ncpu, len(jobs)), initializer=_pool_init) as pool:
        return pool.map(_solve_sphere, jobs, chunksize=1)


# --------------------------------------------------------------------------
# the assembled system
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SystemArrays:
    """Inputs of one (system, q) instance in the layout the library takes.
    Complex arrays are complex128; padding beyond npw is zero."""
    nr: np.ndarray            # int32[3]
    at: np.ndarray            # [3,3] bohr, rows a1 a2 a3
    q: np.ndarray             # [3] bohr^-1 cartesian
    g0: np.ndarray            # int32[3] Miller index of G0 (Q = q + G0)
    xk: np.ndarray            # [nks,3]
    wk: np.ndarray            # [nks]
    npw_k: np.ndarray         # int32[nks]
    npw_kq: np.ndarray        # int32[nks]
    nl_k: np.ndarray          # int32[nks,npwx]
    nl_kq: np.ndarray         # int32[nks,npwx]
    evc_k: np.ndarray         # complex[nks,nbnd,npwx]
    evc_kq: np.ndarray        # complex[nks,nbnd,npwx]
    et_k: np.ndarray          # [nks,nbnd]
    vloc_r: np.ndarray        # [N]
    fxc_r: np.ndarray         # [N]
    vkb_kq: np.ndarray        # complex[nks,nproj,npwx]
    dkb: np.ndarray           # [nproj]
    # metadata (not library inputs)
    et_kq: np.ndarray = None  # [nks, nbnd+extra] energies at k+q
    n0_r: np.ndarray = None
    ecut: float = 0.0
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def nks(self):
        return int(self.xk.shape[0])

    @property
    def nbnd(self):
        return int(self.et_k.shape[1])

    @property
    def nproj(self):
        return int(self.dkb.shape[0])

    @property
    def npwx(self):
        return int(self.nl_k.shape[1])

    @property
    def omega(self):
        return float(abs(np.linalg.det(self.at)))

    @property
    def qcart(self):
        return self.q + self.g0.astype(np.float64) @ reciprocal(self.at)

    def gap(self) -> float:
        """min over k, n of eps_{nbnd+1,k+q} - eps_{n,k}."""
        return float(np.min(self.et_kq[:, self.nbnd]) - np.max(self.et_k))


def build_system(*, at, nr, ecut, tau_frac, depth, width, nbnd, kpts, q, g0=(0, 0, 0),
                 kb=None, xc="pz", wk=None, kq_basis="sphere", extra_bands=2,
                 tol=1e-10, orbitals="eigen", seed=0) -> SystemArrays:
    """Assemble one synthetic instance.

    kb: None or dict(radii=[nat,2], dkb=[nat,2]) for s/p projectors.
    kq_basis: "sphere" (the k+q sphere) or "union" (the k+q sphere together
    with the k sphere shifted by G0, used where an exact f-sum is required).
    orbitals: "eigen" (lowest eigenpairs) or "random" (seeded orthonormal
    orbitals, for operator tests of cells too large to diagonalise)."""
    at = np.asarray(at, dtype=np.float64)
    nr = np.asarray(nr, dtype=np.int32)
    tau_frac = np.asarray(tau_frac, dtype=np.float64)
    tau = tau_frac @ at
    kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    nks = kpts.shape[0]
    wk = np.full(nks, 1.0 / nks) if wk is None else np.asarray(wk, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    g0 = np.asarray(g0, dtype=np.int32)
    vloc = gaussian_wells_r(at, nr, tau, depth, width)
    if kb is not None:
        radii = np.asarray(kb["radii"], dtype=np.float64)
        dat = np.asarray(kb["dkb"], dtype=np.float64)
        dkb = np.concatenate([[d[0], d[1], d[1], d[1]] for d in dat]).astype(np.float64)
    else:
        radii = None
        dkb = np.zeros(0)
    nev = nbnd + extra_bands
    jobs = []
    for i, k in enumerate(kpts):
        jobs.append((at, nr, vloc, k, k, ecut, tau, radii, dkb, nev, tol, None))
        jobs.append((at, nr, vloc, k + q, k, ecut, tau, radii, dkb, nev, tol,
                     g0 if kq_basis == "union" else None))
    if orbitals == "random":
        jobs = [j + (seed * 1000 + t,) for t, j in enumerate(jobs)]
    elif orbitals != "eigen":
        raise ValueError(orbitals)
    res = _run_jobs(jobs)
    mk, mkq, uk, ukq, ek, ekq, bkq = [], [], [], [], [], [], []
    for i in range(nks):
        (m1, v1, w1, _), (m2, v2, w2, b2) = res[2 * i], res[2 * i + 1]
        mk.append(m1); uk.append(v1[:, :nbnd]); ek.append(w1[:nbnd])
        mkq.append(m2); ukq.append(v2[:, :nbnd]); ekq.append(w2); bkq.append(b2)
    npwx = max(max(len(m) for m in mk), max(len(m) for m in mkq))
    nproj = len(dkb)
    nl_k = np.zeros((nks, npwx), dtype=np.int32)
    nl_kq = np.zeros((nks, npwx), dtype=np.int32)
    evc_k = np.zeros((nks, nbnd, npwx), dtype=np.complex128)
    evc_kq = np.zeros((nks, nbnd, npwx), dtype=np.complex128)
    vkb_kq = np.zeros((nks, nproj, npwx), dtype=np.complex128)
    for i in range(nks):
        nl_k[i, :len(mk[i])] = linear_index(mk[i], nr)
        nl_kq[i, :len(mkq[i])] = linear_index(mkq[i], nr)
        evc_k[i, :, :len(mk[i])] = uk[i].T
        evc_kq[i, :, :len(mkq[i])] = ukq[i].T
        if nproj:
            vkb_kq[i, :, :len(mkq[i])] = bkq[i]
    # ground-state density n0(r) = 2 sum_k w_k sum_n |u_nk(r)|^2
    omega = abs(np.linalg.det(at))
    ntot = int(np.prod(nr))
    n0 = np.zeros(ntot)
    for i in range(nks):
        g = np.zeros((nbnd, ntot), dtype=np.complex128)
        g[:, nl_k[i, :len(mk[i])]] = evc_k[i, :, :len(mk[i])]
        ur = sfft.ifftn(g.reshape(nbnd, *nr), axes=(1, 2, 3), workers=_WORKERS).reshape(nbnd, -1) * (ntot / math.sqrt(omega))
        n0 += 2.0 * wk[i] * np.sum(np.abs(ur) ** 2, axis=0)
    if xc == "pz":
        fxc = pz_lda_fxc(n0)
    elif xc == "x":
        fxc = x_lda_fxc(n0)
    elif xc == "none":
        fxc = np.zeros(ntot)
    else:
        raise ValueError(xc)
    return SystemArrays(
        nr=nr, at=at, q=q, g0=g0, xk=kpts, wk=wk,
        npw_k=np.array([len(m) for m in mk], dtype=np.int32),
        npw_kq=np.array([len(m) for m in mkq], dtype=np.int32),
        nl_k=nl_k, nl_kq=nl_kq, evc_k=evc_k, evc_kq=evc_kq,
        et_k=np.array(ek), vloc_r=vloc, fxc_r=fxc, vkb_kq=vkb_kq, dkb=dkb,
        et_kq=np.array(ekq), n0_r=n0, ecut=float(ecut),
        info=dict(depth=depth, width=width, tau_frac=tau_frac.tolist()),
    )
