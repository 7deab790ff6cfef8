"""Pseudo-Hermitian Lanczos recursion for the SBR Liouvillian (Sec. 2.5).

The paper names the method (a generalised Hermitian Lanczos under a metric
that redefines the scalar product, needing half the Liouvillian applications
of the biorthogonal variant) without writing it out.  The reading used here:

  * Metric J = diag(D + K, D).  With D and K Hermitian, J L = L^dagger J, so L
    is self-adjoint in <a,b>_J = <a, J b>; J is positive definite when D and
    D + K are (a gapped, stable ground state).
  * L maps an upper-only vector (q,0) to a lower-only one (0,(D+K)q) and back,
    so Krylov vectors alternate between the two components, every diagonal
    coefficient alpha_j vanishes, and J w equals L w with its components
    swapped: the metric costs no extra operator application.
  * Start vector r = (0, y) (the starting vector the paper gives for both
    Lanczos flavours); beta_1 = ||r||_J = sqrt(<y, D y>).
  * Step j (one application of L per step):
        w          = L v_j - beta_j v_{j-1}
        Lw         = L w           (D+K on an upper w, D on a lower w)
        beta_{j+1} = sqrt(Re <w, Lw>_w)   (the J-norm of w)
        v_{j+1} = w / beta_{j+1};  L v_{j+1} = Lw / beta_{j+1}
        gamma_{j+1} = beta_{j+1}
        z_{j+1} = <y, upper part of v_{j+1}>_w   (0 for a lower v_{j+1})
    which realises eq. zeta_coef_q with the probe {y, 0} (the SBR of n_Q).
  * Every new vector w is restricted to the conduction manifold (w <- P_c w
    block by block) before L is applied.  The SBR vectors live there in
    exact arithmetic (y, D and K all end in P_c), so this changes nothing
    but rounding; without it the valence components that rounding leaves
    behind lie in the null space of J, are invisible to every J-inner
    product, and grow like prod(beta_j / beta_{j+1}) along the recursion.
  * No reorthogonalisation (the paper mentions none); an optional full
    J-reorthogonalisation exists for the exhaustive-Krylov tests only.
  * A zero right-hand side (every transition Pauli-blocked, ||y||_w^2 <=
    tol^2 nbnd) ends the recursion before its first step: chi = 0.
  * Termination, with b the largest of beta_2..beta_j and tol = 1e-7:
    beta_{j+1}^2 < -(tol b)^2 (or beta_2^2 <= 0) means J is not positive
    definite; |beta_{j+1}^2| <= (tol b)^2 is a lucky breakdown -- the Krylov
    space is exhausted (to rounding) and the coefficients so far are exact.

M steps apply L M times and give beta_1..beta_M, gamma = beta, z_1..z_M.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BREAKDOWN_TOL = 1e-7


@dataclass
class LanczosResult:
    beta: np.ndarray
    gamma: np.ndarray
    z: np.ndarray
    status: str = "ok"          # "ok", "breakdown", "not_pd"
    steps: int = 0
    history: list = field(default_factory=list)


def pseudo_hermitian_lanczos(apply_D, apply_DK, inner, y, nsteps: int, project=None,
                             reorth: bool = False, tol: float = BREAKDOWN_TOL,
                             y_scale: float = 1.0) -> LanczosResult:
    """Run nsteps steps.  apply_D / apply_DK act on a batch; inner is the
    weighted inner product <a,b>_w; y is the right-hand side batch; project
    is P_c on a batch (None when the operators already live on the
    conduction manifold, as explicit transition-basis matrices do);
    y_scale is the squared norm y would have without P_c (the number of
    bands for normalised orbitals): ||y||^2 <= tol^2 y_scale means y = 0."""
    beta = np.zeros(nsteps)
    z = np.zeros(nsteps, dtype=np.complex128)
    # start: r = (0, y) is lower; L r = (D y, 0) is upper
    if inner(y, y).real <= (tol ** 2) * y_scale:
        # every transition is blocked (y = 0 to rounding): chi vanishes
        return LanczosResult(beta[:0], beta[:0], z[:0], "breakdown", 0)
    Lr = apply_D(y)
    b2 = inner(y, Lr).real
    if b2 <= 0.0:
        return LanczosResult(beta[:0], beta[:0], z[:0], "not_pd", 0)
    beta[0] = math.sqrt(b2)
    v_prev = np.zeros_like(y)
    v = y / beta[0]
    Lv = Lr / beta[0]
    v_is_upper = False
    basis = [(v, Lv, v_is_upper)] if reorth else None
    status, done = "ok", 1
    bmax = 0.0
    for j in range(1, nsteps):
        w = Lv - beta[j - 1] * v_prev if j > 1 else Lv.copy()
        if project is not None:
            w = project(w)
        w_is_upper = not v_is_upper
        Lw = apply_DK(w) if w_is_upper else apply_D(w)
        if reorth:
            for _ in range(2):
                for (bv, bLv, bup) in basis:
                    if bup == w_is_upper:
                        # <v_i, w>_J = <J v_i, w> with J v_i = L v_i swapped
                        c = inner(bLv, w)
                        w = w - c * bv
                        Lw = Lw - c * bLv
        b2 = inner(w, Lw).real
        if b2 < -(tol * bmax) ** 2 or (b2 <= 0.0 and bmax == 0.0):
            status = "not_pd"
            break
        if b2 <= (tol * bmax) ** 2:
            status = "breakdown"
            break
        bj = math.sqrt(b2)
        beta[j] = bj
        bmax = max(bmax, bj)
        v_prev, v, Lv = v, w / bj, Lw / bj
        v_is_upper = w_is_upper
        z[j] = inner(y, v) if v_is_upper else 0.0
        done = j + 1
        if reorth:
            basis.append((v, Lv, v_is_upper))
    return LanczosResult(beta[:done].copy(), beta[:done].copy(), z[:done].copy(), status, done)


def nonhermitian_lanczos(apply_D, apply_DK, inner, y, nsteps: int, project=None,
                         reorth: bool = False, tol: float = BREAKDOWN_TOL,
                         y_scale: float = 1.0) -> LanczosResult:
    """The non-Hermitian Lanczos biorthogonalisation of Sec. 2.5: two chains,
    v_j driven by L and u_j by L^dagger = [[0, D+K], [D, 0]], both started
    from u_1 = v_1 = (0, y) / ||y||, with (u_i, v_j) = delta_ij and
    T_ij = (u_i, L v_j).  Reading of the coefficients (the paper names the
    algorithm and its beta, gamma): with s = (u^_{j+1}, v^_{j+1}),
        v^_{j+1} = L v_j - gamma_j v_{j-1},   u^_{j+1} = L^dagger u_j - beta_j u_{j-1},
        beta_{j+1} = sqrt|s|,  gamma_{j+1} = s / beta_{j+1}  (complex in general),
        v_{j+1} = v^_{j+1} / beta_{j+1},  u_{j+1} = u^_{j+1} / conj(gamma_{j+1}),
    so T has sub-diagonal beta and super-diagonal gamma (zero diagonal: the
    chains alternate between the components as in the pseudo-Hermitian
    form).  z_j = ((y, 0), v_j).  Each step applies L once and L^dagger once:
    one D and one D+K application, twice the pseudo-Hermitian cost.  beta_1 =
    ||y||; a step with |s| <= (tol b)^2 (b the largest beta_2..beta_j) is a
    breakdown; P_c is applied to both new vectors as in the other form."""
    beta = np.zeros(nsteps)
    gamma = np.zeros(nsteps, dtype=np.complex128)
    z = np.zeros(nsteps, dtype=np.complex128)
    ny2 = inner(y, y).real
    if ny2 <= (tol ** 2) * y_scale:
        return LanczosResult(beta[:0], gamma[:0], z[:0], "breakdown", 0)
    beta[0] = math.sqrt(ny2)
    gamma[0] = beta[0]
    v = y / beta[0]
    u = v.copy()
    v_prev = np.zeros_like(y)
    u_prev = np.zeros_like(y)
    upper = False
    basis = [(v, u, upper)] if reorth else None
    status, done, bmax = "ok", 1, 0.0
    for j in range(1, nsteps):
        if upper:        # v = (q, 0): L v = (0, (D+K) q);  L^dagger u = (0, D q_u)
            Lv, Lu = apply_DK(v), apply_D(u)
        else:            # v = (0, p): L v = (D p, 0);      L^dagger u = ((D+K) p_u, 0)
            Lv, Lu = apply_D(v), apply_DK(u)
        vh = Lv - gamma[j - 1] * v_prev
        uh = Lu - beta[j - 1] * u_prev
        if project is not None:
            vh, uh = project(vh), project(uh)
        new_upper = not upper
        if reorth:
            for _ in range(2):
                for (bv, bu, bup) in basis:
                    if bup == new_upper:
                        vh = vh - inner(bu, vh) * bv
                        uh = uh - inner(bv, uh) * bu
        sv = inner(uh, vh)
        if abs(sv) <= (tol * bmax) ** 2:
            status = "breakdown"
            break
        bj = math.sqrt(abs(sv))
        gj = sv / bj
        beta[j], gamma[j] = bj, gj
        bmax = max(bmax, bj)
        v_prev, v = v, vh / bj
        u_prev, u = u, uh / np.conj(gj)
        upper = new_upper
        z[j] = inner(y, v) if upper else 0.0
        done = j + 1
        if reorth:
            basis.append((v, u, upper))
    return LanczosResult(beta[:done].copy(), gamma[:done].copy(), z[:done].copy(), status, done)


def run(liouvillian, nsteps: int, reorth: bool = False, variant: str = "ph") -> LanczosResult:
    """Lanczos on an oracle Liouvillian from its own right-hand side y:
    variant "ph" (pseudo-Hermitian) or "nh" (non-Hermitian biorthogonal)."""
    y = liouvillian.rhs()
    fn = pseudo_hermitian_lanczos if variant == "ph" else nonhermitian_lanczos
    return fn(liouvillian.apply_D, liouvillian.apply_DK, liouvillian.inner, y, nsteps,
              project=liouvillian.project_c, reorth=reorth, y_scale=float(liouvillian.nbnd))
