/*
 * lz.h -- C ABI of the Liouville-Lanczos hot path on AMD Instinct MI355X (gfx950).
 *
 * The library computes the charge-density susceptibility chi(Q,Q;omega) of a
 * periodic insulator within linearised TDDFT (Timrov, Vast, Gebauer, Baroni,
 * "turboEELS").  It applies the Liouvillian superoperator in the standard
 * batch representation (Sec. 2.4, eqs. Liouvillian_SBR, D_super-operator_2,
 * K_super-operator_2) to a batch of response orbitals over bands and
 * k-points at fixed q, runs the pseudo-Hermitian Lanczos recursion (Sec. 2.5)
 * -- or, for comparison, the non-Hermitian biorthogonal one the paper
 * contrasts it with -- and evaluates chi, eps^-1 and the loss function from
 * the tridiagonal matrix
 * (eqs. post_processing, resolvent_Liouvillian_Lanczos_2_for_chi,
 * def_inv_microscopic_diel_tensor).
 *
 * Units: Hartree atomic units (energies in Ha, lengths in bohr).
 * Complex numbers are stored interleaved (re, im).
 * Every call returns an lz_status and never throws or aborts across the ABI;
 * lz_last_error() gives a message for the last non-OK status of the calling
 * thread.
 */
#ifndef LZ_H
#define LZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lz_ctx lz_ctx; /* opaque; owns every device buffer of a run */

typedef enum {
  LZ_OK = 0,
  LZ_ERR_ARG = 1,    /* a null pointer, an inconsistent size or index, an unsupported grid */
  LZ_ERR_HIP = 2,    /* a HIP runtime failure; the context is unusable afterwards */
  LZ_ERR_OOM = 3,    /* device allocation failed */
  LZ_ERR_NOT_PD = 4, /* beta^2 <= 0: the metric diag(D+K, D) is not positive definite */
  LZ_ERR_STATE = 5,  /* call order violated (e.g. a spectrum longer than the recursion) */
  LZ_BREAKDOWN = 6   /* informational: Krylov space exhausted, coefficients so far exact */
} lz_status;

typedef enum {
  LZ_FP64 = 0,            /* every array and every FFT in double precision */
  LZ_FP32 = 1,            /* vectors, FFTs, pointwise work and projector products in
                             single precision; Lanczos scalars and the spectrum in double */
  LZ_FP32_SPLITBF16 = 2   /* as LZ_FP32, with the projector products on the matrix cores as
                             three bf16 products of (hi, lo) splits of every FP32 operand
                             (x ~ bf16(x) + bf16(x - bf16(x)); the lo*lo term is dropped,
                             about 2^-16 relative per product), FP32 accumulation */
} lz_precision;

typedef enum {   /* levels of theory of Sec. 3.2 */
  LZ_TDDFT = 0,  /* Hartree + adiabatic xc kernel f_xc */
  LZ_RPA = 1,    /* Hartree only ("RPA with crystal local-field effects") */
  LZ_IPA = 2     /* K = 0 (independent particles) */
} lz_approx;

/*
 * One (system, q) instance: the ground-state data of Sec. 3.1 plus q.
 * Host arrays in double precision, owned by the caller and deep-copied by
 * lz_init (the caller may free them when lz_init returns).
 *
 *  nr        FFT grid N1 = N2 = N3 (cubic grids only; the transforms of
 *            other shapes are not validated and are refused).  N must factor
 *            into 2, 3, 5 with 2 <= N <= 96.  Grid point (j1,j2,j3) is at
 *            r = sum_i (j_i/N_i) a_i, stored at (j1*N2 + j2)*N3 + j3.
 *  at        lattice vectors, rows a1, a2, a3 (bohr).
 *  q         q in Cartesian bohr^-1;  g0: Miller index of G0 (Q = q + G0).
 *  nks       number of k-points; nbnd: occupied bands per k (the valence
 *            manifold of P_c); nproj: separable projectors (0 = local only);
 *            npwx: padded stride of every plane-wave array (>= max npw).
 *  xk        [nks][3] k-points (Cartesian bohr^-1);  wk: [nks] weights, sum 1.
 *  npw_k, npw_kq   [nks] plane-wave counts of the spheres at k and k+q.
 *  nl_k, nl_kq     [nks][npwx] linear grid index of each plane wave
 *            (Miller index m stored at the index of m mod N; Miller indices
 *            must lie in [-N/2, N/2) so the centred representative recovers
 *            them).  Entries beyond npw are ignored.
 *  evc_k     [nks][nbnd][npwx] complex: u_nk on the k sphere (orthonormal).
 *  evc_kq    [nks][nbnd][npwx] complex: u_n,k+q on the k+q sphere (orthonormal);
 *            they define P_c^{k+q} = 1 - sum_n |u_n,k+q><u_n,k+q| (Sec. 2.3).
 *  et_k      [nks][nbnd] eps_nk (Ha).
 *  vloc_r    [N] total local Kohn-Sham potential on the grid (Ha).
 *  fxc_r     [N] adiabatic xc kernel f_xc(r) (Ha bohr^3); ignored for RPA/IPA.
 *  vkb_kq    [nks][nproj][npwx] complex projectors beta_p(k+q+G);
 *  dkb       [nproj] their energies: V_NL = sum_p |beta_p> D_p <beta_p|.
 *            (both may be NULL when nproj == 0)
 *  Orbitals are normalised over the cell: u(r) = Omega^-1/2 sum_G u(G) e^{iG.r}.
 */
typedef struct {
  int32_t nr[3];
  double at[9];
  double q[3];
  int32_t g0[3];
  int32_t nks, nbnd, nproj, npwx;
  const double *xk, *wk;
  const int32_t *npw_k, *npw_kq;
  const int32_t *nl_k, *nl_kq;
  const double *evc_k, *evc_kq;
  const double *et_k;
  const double *vloc_r, *fxc_r;
  const double *vkb_kq, *dkb;
} lz_system;

typedef enum {             /* Lanczos recursions of Sec. 2.5 */
  LZ_PSEUDO_HERMITIAN = 0, /* one Liouvillian half-application per step (the production method) */
  LZ_NON_HERMITIAN = 1     /* biorthogonal chains v (driven by L) and u (by L^dagger, with
                              L^dagger = [[0, D+K], [D, 0]]): one D and one D+K application per
                              step; complex gamma and z */
} lz_algorithm;

typedef enum {        /* where the projector products (P_c and separable projectors) run */
  LZ_GEMM_AUTO = 0,   /* matrix cores when nbnd >= 32 and nbnd + nproj >= 64, else vector ALU */
  LZ_GEMM_VALU = 1,   /* vector ALU kernels (tuned for few bands) */
  LZ_GEMM_MFMA = 2    /* matrix cores (MFMA), any size */
} lz_projector_gemm;

typedef struct {
  lz_precision prec;
  lz_approx approx;
  int32_t max_steps;  /* capacity of the coefficient arrays (>= 1) */
  int32_t use_graph;  /* nonzero: lz_step replays every pair of steps after the first as one
                         captured hipGraph (built on first use; not while the stage timer is
                         on; with batched, one graph holds the pair of every group); results
                         are bitwise identical to the eager launches */
  int32_t autotune;   /* 0: the built-in launch heuristics.  1: lz_init times, per instance,
                         candidate launch configurations (projector products on the vector
                         ALU or the matrix cores, unless projector_gemm asks for one; two
                         sizes of the density band groups; three plane-wave chunk lengths of
                         the vector-ALU projector dot; the register-line or lane-pair plane
                         transforms against LDS Stockham passes, see fft_planes) on a few
                         operator applications
                         and keeps the fastest (lz_get_tuning reports it).  Candidates agree
                         to rounding, so with 1 the bits of a run may depend on the timing. */
  lz_algorithm algorithm;
  int32_t streams;    /* instances of one context that lz_step advances side by side, each
                         on its own HIP stream (instance i on stream i mod streams):
                         0 = min(n_inst, 4), 1 = one instance after another; at most 64.
                         Results do not depend on it (bitwise). */
  lz_projector_gemm projector_gemm;  /* results agree to rounding across the choices */
  int32_t density_group_bands;  /* bands per group of the response-density pass (the groups'
                                   partial densities are summed in a fixed order):
                                   0 = the built-in heuristic (or the autotuner's pick),
                                   n >= 1 = n (clamped to nks * nbnd); fixed, it is not tuned */
  int32_t projector_chunk;      /* plane waves per partial of the vector-ALU projector dot:
                                   0 = the heuristic (64; or the autotuner's pick among 64, 128,
                                   256), or one of 64, 128, 256; fixed, it is not tuned */
  int32_t fft_planes;  /* schedule of the 2-D plane transforms: 0 = register-line (one thread
                          per line: 24^2-48^2 planes in FP32) or lane-pair (64^2-96^2 in FP32,
                          the v'u pass on 48^2 in FP64) kernels where they exist, else LDS
                          Stockham passes, and with autotune the autotuner also times the
                          other; 1 = the former, 2 = the LDS passes everywhere; fixed (1, 2)
                          it is not tuned.  Results agree to rounding across the choices. */
  int32_t batched;  /* 1: lz_step advances the pseudo-Hermitian recursions of all instances
                       with one launch per kernel of a step over all of them (a work list of
                       (instance, block) items; instances whose steps issue different kernels
                       -- other grids, precisions or projector paths -- form groups, each
                       group launched as one, groups side by side on the `streams` streams).
                       Applies while every running instance is at the same step, no stage
                       timer is on and the algorithm is pseudo-Hermitian; otherwise, and with
                       0, every instance issues its own launches.  Results do not depend on
                       it (bitwise). */
} lz_options;

/*
 * Create a context on HIP device `device` for n_inst instances (sys[0..n_inst-1]).
 * Work is ordered on `hip_stream` (a hipStream_t; NULL = the device's null
 * stream).  Builds the stick tables, the valence orbitals in real space and the
 * right-hand side y = P_c^{k+q} e^{iG0.r} u_nk (eq. RHS_of_Liouville_eq).
 * Errors: LZ_ERR_ARG (see the field rules above; also q + G = 0 on the grid for
 * TDDFT/RPA, weights not summing to 1, duplicate plane waves), LZ_ERR_OOM,
 * LZ_ERR_HIP.  *out is NULL on error.
 */
lz_status lz_init(const lz_system *sys, int32_t n_inst, const lz_options *opt,
                  int32_t device, void *hip_stream, lz_ctx **out);

/*
 * One application of the SBR Liouvillian (eqs. Liouvillian_SBR,
 * D_super-operator_2, K_super-operator_2) to every instance:
 *     q_out = D p_in,     p_out = (D + K) q_in,
 * (D x)_nk = P_c^{k+q}(H_{k+q} - eps_nk) x_nk and
 * (K x)_nk = P_c^{k+q} v'_HXC[n'[x]] u_nk with n' = 4 sum_k w_k sum_n u*_nk x_nk.
 * Arguments are device pointers on the context's device holding complex
 * arrays [inst][nks][nbnd][npwx] in the caller's plane-wave order (that of
 * nl_kq), complex128 for LZ_FP64 and complex64 otherwise; padding beyond npw_kq
 * is ignored on input and written as zero.  Either half may be skipped by
 * passing NULL for both its input and output.  Inputs and outputs must not
 * alias.  Stream-ordered; returns without synchronising.
 */
lz_status lz_apply_liouvillian(lz_ctx *ctx, const void *q_in, const void *p_in,
                               void *q_out, void *p_out);

/*
 * Advance the Lanczos recursion of every instance by n_steps steps; the first
 * call starts from the vector (0, y).  Step j gives beta_{j+1}, gamma_{j+1}
 * and z_{j+1}.
 * Pseudo-Hermitian: one Liouvillian half-application per step, gamma = beta.
 * Non-Hermitian: u_1 = v_1 = (0, y)/||y||; step 0 takes only the norm
 * (beta_1 = gamma_1 = ||y||), every later step applies L to v_j and L^dagger
 * to u_j (one D and one D+K application) and sets, with
 * s = (L^dagger u_j - beta_j u_{j-1}, L v_j - gamma_j v_{j-1}),
 * beta_{j+1} = sqrt|s|, gamma_{j+1} = s / beta_{j+1} (complex) and
 * z_{j+1} = ((y, 0), v_{j+1}); breakdown when |s| <= (1e-7 max beta)^2.
 * Coefficients stay on the device.  On return *steps_done is the
 * total number of completed steps of instance 0.  Synchronises the stream once
 * at the end to read the status flags.
 * Returns LZ_BREAKDOWN when an instance exhausted its Krylov space (its
 * coefficients so far are exact and its later steps are no-ops),
 * LZ_ERR_NOT_PD when the metric is indefinite, LZ_ERR_STATE when the
 * coefficient capacity (max_steps) would be exceeded.
 */
lz_status lz_step(lz_ctx *ctx, int32_t n_steps, int32_t *steps_done);

/* Restart the recursion of every instance from (0, y), keeping the context
 * (tables, orbitals, y).  Later lz_step calls overwrite the coefficients from
 * index 0.  Stream-ordered. */
lz_status lz_reset(lz_ctx *ctx);

/* Copy coefficients first..first+count-1 (0-based: index j holds beta_{j+1})
 * of instance inst to host arrays beta[count], gamma[count], z[count][2].
 * Any of the three may be NULL.  LZ_ERR_STATE if they are not computed yet;
 * LZ_ERR_ARG for a non-NULL gamma of a non-Hermitian instance (complex: see
 * lz_get_gamma). */
lz_status lz_get_coefficients(lz_ctx *ctx, int32_t inst, int32_t first, int32_t count,
                              double *beta, double *gamma, double *z);

/* gamma_{first+1}..gamma_{first+count} of instance inst as complex numbers,
 * host array gamma[count][2] (the super-diagonal of T; equal to beta with a
 * zero imaginary part for the pseudo-Hermitian recursion).  LZ_ERR_STATE if
 * not computed yet. */
lz_status lz_get_gamma(lz_ctx *ctx, int32_t inst, int32_t first, int32_t count, double *gamma);

/* Number of completed steps and recursion status (0 running, LZ_BREAKDOWN,
 * LZ_ERR_NOT_PD) of one instance.  Synchronises the stream. */
lz_status lz_get_state(lz_ctx *ctx, int32_t inst, int32_t *steps_done, int32_t *status);

/*
 * Spectrum of instance inst from its first m coefficients (Sec. 2.5, Sec. 3.3),
 * computed on the device in double precision:
 *   (omega + i eta - T_m) x = e_1,   chi = (4/Omega) beta_1 sum_j Re(z_j) x_j,
 * (z_j is real in exact arithmetic; its rounding-level imaginary part is dropped),
 * T_m with sub-diagonal beta and super-diagonal gamma.  For a non-Hermitian
 * instance gamma and z are complex and sum_j z_j x_j is used as it is.
 *   eps^-1 = 1 + 4 pi chi / |Q|^2,   loss = -Im eps^-1.
 * omega: host [n_omega] (Ha); eta > 0 (Ha).  Outputs are host arrays:
 * chi[n_omega][2], eps_inv[n_omega][2], loss[n_omega]; any may be NULL.
 * m = 0 with a vanished right-hand side gives chi = 0.
 */
lz_status lz_spectrum(lz_ctx *ctx, int32_t inst, int32_t m, const double *omega,
                      int32_t n_omega, double eta, double *chi, double *eps_inv,
                      double *loss);

/* Extrapolation of the Lanczos coefficients for the spectrum (Sec. 3.3, the
 * itermax0 / itermax / extrapolation inputs of the spectrum program). */
typedef enum {
  LZ_EXTRAP_NONE = 0,      /* the m0 computed coefficients only */
  LZ_EXTRAP_CONSTANT = 1,  /* beta_i for i > m0: mean of the last half of beta_2..beta_m0 */
  LZ_EXTRAP_OSC = 2        /* bi-constant: the mean over the same window of the beta_i
                              with the parity of i */
} lz_extrapolation;

/*
 * As lz_spectrum from the first m0 computed coefficients, the tridiagonal
 * matrix extended to dimension m >= m0 by `extrapolation` (z_j = 0 beyond
 * m0).  The extension costs O(m) per frequency, so m may be taken far larger
 * than the number of steps run.  m is ignored with LZ_EXTRAP_NONE.  Errors:
 * LZ_ERR_ARG for an unknown scheme, m < m0, m > m0 with m0 < 4, or m > m0 for
 * a non-Hermitian instance;
 * LZ_ERR_STATE when m0 exceeds the completed steps.
 */
lz_status lz_spectrum_ext(lz_ctx *ctx, int32_t inst, int32_t m0, int32_t m,
                          int32_t extrapolation, const double *omega, int32_t n_omega,
                          double eta, double *chi, double *eps_inv, double *loss);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as lz_spectrum_ext, bit for bit, with the same arguments and
 * errors, but no device allocation.  The frequency grid, the outputs and the
 * extrapolation tail are staged through a fixed device area of 3.1 MB per
 * device that the library holds from the first lz_init on that device until
 * the process ends.  Limit: n_omega <= 65536 (LZ_ERR_ARG beyond).  Every
 * call on one device shares that area: calls that overlap on one device
 * (from several threads, or on contexts whose streams run concurrently)
 * race and must be serialised by the caller.  Synchronises the context's
 * stream.
 */
lz_status lz_spectrum_ext_noalloc(lz_ctx *ctx, int32_t inst, int32_t m0, int32_t m,
                                  int32_t extrapolation, const double *omega, int32_t n_omega,
                                  double eta, double *chi, double *eps_inv, double *loss);

/* Launch configuration of instance inst (after autotuning, if asked for):
 * where its projector products run (LZ_GEMM_VALU or LZ_GEMM_MFMA; the
 * split-bf16 precision reports LZ_GEMM_MFMA), the bands per group of its
 * density pass and the plane-wave chunks of its projector dots.  Any output
 * may be NULL. */
lz_status lz_get_tuning(lz_ctx *ctx, int32_t inst, int32_t *projector_gemm,
                        int32_t *density_group_bands, int32_t *projector_chunks,
                        int32_t *fft_planes);

/* Host-side launch plan, without a system or a device: the launch
 * parameters lz_init derives with its heuristic (before any autotuning) for
 * a cubic grid of n points per side (n a product of 2, 3 and 5 in [2, 128],
 * n^2 <= 9216), nbnd bands at each of nks k-points, npwx plane waves per
 * padded row, nproj separable projectors and precision prec; for tests and
 * tools that check the host helpers over every supported grid.  `slots` is
 * a number of density-pass blocks resident at once (the round rule of the
 * LDS density pass; 0 skips it).  out (host, LZ_PLAN_LEN int32, caller-owned):
 *   [0] compile-time FFT length (0: runtime radix plans)
 *   [1] plane length of the register-line / lane-pair kernels (0: LDS passes)
 *   [2] density band-group size of the default schedule: the register-form
 *       heuristic where [1] > 0, else [3]
 *   [3] density band-group size of the LDS passes: the round rule for
 *       `slots` when slots > 0, else the heuristic lz_init falls back to
 *   [4] the round rule's size for `slots` (0 if slots = 0)
 *   [5..8]  vector-ALU projector path: dot chunk (plane waves), chunks,
 *           blocks of the output update, the same over the projector rows
 *   [9..12] the same for the matrix-core path (split-bf16 products for
 *           LZ_FP32_SPLITBF16)
 *   [13] band-group size after clamping to 1..nks*nbnd, [14] groups.
 * LZ_ERR_ARG for sizes lz_init would refuse or a NULL out; no device call. */
#define LZ_PLAN_LEN 15
lz_status lz_launch_plan(int32_t n, int32_t prec, int32_t nbnd, int32_t nks, int32_t npwx,
                         int32_t nproj, int32_t slots, int32_t *out);

/* Copy the right-hand side y of instance inst to a device array in the
 * caller's layout and precision (as lz_apply_liouvillian). */
lz_status lz_get_rhs(lz_ctx *ctx, int32_t inst, void *y_out);

/* Stage timing for measurement: `mask` selects stages by bit (bit s = stage
 * s; -1 = all, 0 = off).  Every later launch of a selected stage in lz_step
 * and lz_apply_liouvillian is bracketed by HIP events on the context's
 * stream, and lz_stage_times returns, per stage, the summed event-measured
 * duration (ms) and the number of timed launches since the last
 * lz_stage_timer call.  Stages (8 entries): 0 z pass sphere->sticks,
 * 1 plane pass of a D step, 2 plane pass with the response density,
 * 3 Hartree+xc potential, 4 plane pass v'u, 5 z pass sticks->sphere,
 * 6 projector products (P_c and separable projectors), 7 Lanczos vector
 * update and reductions.  Stages 0, 1, 2, 4 and 5 are one kernel launch
 * each.  Arrays total_ms[8], count[8]; either may be NULL. */
lz_status lz_stage_timer(lz_ctx *ctx, int32_t mask);
lz_status lz_stage_times(lz_ctx *ctx, int32_t inst, double *total_ms, int32_t *count);

/*
 * Checkpoint and restart of the recursion of one instance (Sec. 3.2 and the
 * restart / restart_step inputs of App. A: more steps added to an existing
 * run): the step count and scalar state, the coefficients
 * computed so far and the Lanczos vectors, in a host buffer the caller
 * owns (lz_checkpoint_size bytes; about 3 vectors of the instance, 4 for the
 * non-Hermitian recursion).  The header carries the level of theory and a
 * 64-bit fingerprint of the operator the recursion ran with (lattice, q, G0,
 * spheres, orbitals, energies, potentials, the f_xc kernel where TDDFT
 * reads it, projectors).  Loading into a context of the same operator,
 * precision and algorithm, with max_steps at least the saved step count,
 * continues the recursion bit for bit.  Errors: LZ_ERR_ARG for a small
 * buffer, another system (a different fingerprint, e.g. the same crystal
 * at another q), another level of theory, precision or algorithm, or a
 * corrupt header.  All three synchronise the context's stream.
 */
lz_status lz_checkpoint_size(lz_ctx *ctx, int32_t inst, uint64_t *bytes);
lz_status lz_checkpoint_save(lz_ctx *ctx, int32_t inst, void *buf, uint64_t bytes);
lz_status lz_checkpoint_load(lz_ctx *ctx, int32_t inst, const void *buf, uint64_t bytes);

/*
 * Ground-state preparation on the device (the step before the response run,
 * Sec. 3.1): the lowest sys->nbnd eigenpairs of the Kohn-Sham Hamiltonian
 * H_{k+q} = -1/2 nabla^2 + V_loc + sum_p |beta_p> D_p <beta_p| on every k+q
 * sphere of sys (for the orbitals at k, pass a system with q = 0 and the k
 * spheres as k+q spheres), on a block of m = nbnd + n_extra vectors in
 * double precision on device `device`, ordered after `hip_stream`:
 *   3 m <= 256: LOBPCG (Knyazev 2001) with the Teter-Payne-Allan kinetic
 *     preconditioner and Rayleigh-Ritz in the span of the block, its
 *     orthonormalised preconditioned residuals and the previous search
 *     directions;
 *   256 < 3 m <= 512: Chebyshev-filtered subspace iteration (Zhou and Saad
 *     2007): per iteration a Chebyshev polynomial of H (degree up to 40,
 *     bounded so that the filter keeps the highest wanted direction within
 *     1e8 of the lowest) small on [largest Ritz value, an upper bound of the
 *     spectrum from the kinetic energies, max V_loc and a Gershgorin bound of
 *     the projectors], orthonormalisation and Rayleigh-Ritz of order m.
 * It stops when every wanted residual norm ||H u - eps u|| is below tol, or
 * after max_iter iterations.
 * The orbital and energy fields of sys (evc_k, evc_kq, et_k, fxc_r) are not
 * read.  Outputs (host): evc_out [nks][nbnd][npwx] complex (caller order of
 * nl_kq, orthonormal, phases arbitrary), et_out [nks][nbnd] ascending,
 * *iterations and *max_residual (either may be NULL).  Synchronous.  Errors:
 * LZ_ERR_ARG for 3 (nbnd + n_extra) > 512 (the dense problems run in one
 * 1024-thread block per sphere), a sphere smaller than 3 (nbnd + n_extra),
 * or the lz_init rules on the remaining fields.
 */
lz_status lz_ground_state(const lz_system *sys, int32_t n_extra, double tol, int32_t max_iter,
                          int32_t device, void *hip_stream, double *evc_out, double *et_out,
                          int32_t *iterations, double *max_residual);

typedef enum {    /* adiabatic LDA kernels */
  LZ_XC_X = 0,    /* Slater exchange only */
  LZ_XC_PZ = 1    /* Slater exchange + Perdew-Zunger (1981) correlation, the paper's functional */
} lz_xc;

/*
 * Ground-state density and adiabatic xc kernel on the device (Sec. 3.1: the
 * ground state the response starts from; f_xc of the xc response potential,
 * eq. V_HXC_resp_1):
 *   n0(r) = 2 sum_k w_k sum_n |u_nk(r)|^2   (spin-unpolarised; orbitals
 *            normalised over the cell, u(r) = Omega^-1/2 sum_G u(G) e^{iG.r}),
 *   f_xc(r) = d^2 (n eps_xc(n)) / dn^2 at n0(r), 0 where n0 < 1e-10 bohr^-3.
 * Reads nr, at, nks, nbnd, npwx, xk, wk, npw_k, nl_k and evc_k of sys (the
 * orbitals at k, e.g. from lz_ground_state on a system with q = 0) and the
 * lz_init rules on them; q, the k+q fields, the energies, fxc_r and the
 * projectors are not read.  Outputs (host, either may be NULL): n0_out[N]
 * (bohr^-3) and fxc_out[N] (Ha bohr^3) in the grid order of vloc_r.
 * Synchronous; ordered after `hip_stream` on device `device`.
 */
lz_status lz_ground_density(const lz_system *sys, int32_t xc, int32_t device, void *hip_stream,
                            double *n0_out, double *fxc_out);

/* Release every resource of the context (NULL is accepted). */
lz_status lz_free(lz_ctx *ctx);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char *lz_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LZ_H */
