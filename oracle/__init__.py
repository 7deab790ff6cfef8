"""Reference oracle: a plain, slow, double-precision CPU implementation of the
Liouville-Lanczos hot path (Timrov, Vast, Gebauer, Baroni, "turboEELS").

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls it and shares no code with it: the two only read the same synthetic
input arrays.

Modules
  pw           plane-wave <-> real-space transforms and the KS Hamiltonian
               H_{k+q} (kinetic in G-space, local potential in real space,
               separable projectors)                      [Sec. 2.3]
  liouvillian  D, K, P_c, the response density, the Hartree + ALDA response
               potential and the right-hand side y     [Sec. 2.3-2.4]
  lanczos      the pseudo-Hermitian Lanczos recursion giving beta, gamma, z
                                                          [Sec. 2.5]
  spectrum     chi, eps^-1, eps and the loss function from the tridiagonal
               matrix                                     [Sec. 2.1, 2.5, 3.3]
  brute        explicit matrices built with explicit Fourier sums, for tiny
               cells (direct resolvent, Casida form)      [Sec. 2.2, 2.4]
  closed_forms independent-particle sum over states, free-electron Dyson
               form, first-moment (f-sum) closed form     [Sec. 2.1, 3.2-3.3]

Parity status: every function above is pinned by a CPU test against a closed
form, a brute-force diagonalisation or an invariant, except the parts listed
as "parity unpinned" in their own docstrings.
"""
