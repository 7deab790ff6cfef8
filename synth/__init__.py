"""Seeded synthetic ground states that feed both the oracle and the GPU library.

This package is input preparation only.  It plays the role of the ground-state
calculation that precedes the linear-response run (paper Sec. 3.1): it produces
Kohn-Sham orbitals u_nk and u_n,k+q, their energies, the local potential, the
Kleinman-Bylander projectors and the adiabatic LDA kernel f_xc.  None of the
Liouvillian, Lanczos or spectrum arithmetic lives here; the oracle and the HIP
path each implement that on their own and only read the arrays built here.

Conventions (shared by every consumer of these arrays, stated once here):
  * ``at`` rows are the lattice vectors a1, a2, a3 in bohr; ``bg`` rows are the
    reciprocal vectors with a_i . b_j = 2 pi delta_ij.
  * The FFT grid is nr = (N1, N2, N3); grid point (j1, j2, j3) sits at
    r = sum_i (j_i / N_i) a_i and is stored at linear index (j1*N2 + j2)*N3 + j3.
  * A plane wave with Miller index m = (m1, m2, m3) is stored at the linear
    index of (m1 mod N1, m2 mod N2, m3 mod N3).  Miller indices of orbitals lie
    in [-N/2, N/2) so the centred representative recovers them.
  * Orbitals are lattice-periodic parts normalised over the cell:
    u(r) = Omega^{-1/2} sum_G u(G) e^{iG.r}, sum_G |u(G)|^2 = 1.
  * Energies in Hartree, lengths in bohr.
"""
from .system import (  # noqa: F401
    SystemArrays, build_system, reciprocal, sphere_miller, linear_index,
    mp_kpoints, gaussian_wells_r, kb_projectors, pz_lda_fxc, x_lda_fxc,
)
from .configs import config_system, CONFIGS, QSWEEP_FRACS, q_sweep, k_sphere_system  # noqa: F401
from .vectors import random_batch  # noqa: F401
