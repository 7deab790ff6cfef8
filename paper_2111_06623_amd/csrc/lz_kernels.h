// Host-visible launchers of the device kernels (all stream-ordered, no syncs).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lz_batch.h"
#include "lz_device.h"

namespace lz {

// Row tables of the register-line plane kernels (lz_plane_reg.h).
struct RegPlaneArgs {
  int S, nact;
  const int* soff;        // [S] LDS offset of each stick in a plane (row pitch n + 1)
  const int* soffc;       // [S] the same in a compact plane (active rows only, in act order)
  const int* act;         // [nact] grid row i1 of each stored row
  signed char slot[128];  // index of grid row i1 in act, -1 when it holds no stick
};

// Geometry of the FFT work shared by the kernels of one instance.
struct Grid3 {
  int n1, n2, n3;
  int S;        // sticks (i1, i2 columns) touching any sphere
  int nact;     // rows i1 holding at least one stick
  int pitch2;   // LDS row pitch of a plane (n2 + 1)
  const int* si1;   // [S] stick row i1
  const int* si2;   // [S] stick column i2
  const int* act;   // [nact] active rows
  FftPlan p1, p2, p3;
  const void* tw1;  // twiddles of each plan (cplx<T>)
  const void* tw2;
  const void* tw3;
  // register-line plane kernels (cubic grids, see reg_plane_size)
  const int* soff_f;       // [S] LDS offset si1 (n+1) + si2 of each stick
  const int* soff_c;       // [S] LDS offset slot[si1] (n+1) + si2 in a compact plane
  signed char slot[128];   // index of each grid row i1 in act, or -1
  int lds_planes;          // 1: the LDS Stockham plane kernels even where register-line or
                           // lane-pair kernels exist (a launch schedule the autotuner times)
};

template <typename T> struct LaunchFft {
  // sphere (stick-major order of nb bands, band stride xs) -> sticks [b][z][S]
  static void zfft_inv(const Grid3& g, const void* x, int64_t xs, void* sticks, const int* map,
                       int nb, int nbnd, const LzDevState* st, hipStream_t s);
  // sticks -> plane inverse -> *V -> forward -> sticks
  static void plane_local(const Grid3& g, const void* sin, void* sout, const void* vloc, int nb,
                          const LzDevState* st, hipStream_t s);
  // as plane_local, also accumulating the response density of band groups
  static void plane_local_density(const Grid3& g, const void* sin, void* sout, const void* vloc,
                                  const void* ur, const double* bandw, void* dpart, int nb,
                                  int gsize, const LzDevState* st, hipStream_t s);
  // sticks -> real-space planes [b][z][n1][n2]
  static void plane_to_real(const Grid3& g, const void* sin, void* rout, int nb, hipStream_t s);
  // real-space u_b(r) * v'(r) -> forward -> sticks (accumulated into sout)
  static void plane_vu(const Grid3& g, const void* ur, const void* vp, void* sout, int nb,
                       const LzDevState* st, hipStream_t s);
  // sticks -> forward z -> sphere, plus (kin - eps) x
  static void zfft_fwd(const Grid3& g, const void* sticks, const void* x, int64_t xs, void* y,
                       const int* map, const void* kin, const double* eps, int nb, int nbnd,
                       int npwx, const LzDevState* st, hipStream_t s);
  // density partials -> n'(r) and v'(r) (Hartree + optional f_xc)
  static void hxc(const Grid3& g, const void* dpart, int ngroups, void* nr, void* work,
                  const void* khart, const void* fxc, bool with_fxc, void* vp,
                  const LzDevState* st, hipStream_t s);
  // blocks of the LDS density pass that one compute unit holds at once
  // (occupancy calculator), 0 where the density pass takes another form
  static int density_blocks_per_cu(const Grid3& g);
};

template <typename T> struct LaunchLin {
  // chunk partials of R[k][p][n] = sum_G conj(A[k][p][G]) X[k][n][G], rows p < P
  // of A (a_rows per k), laid out [k][chunk][n][p]; with LW != null the dot
  // first forms X <- a*LW + b*X (state coefficients)
  // (gemm: kGemmValu vector ALU, kGemmMfma matrix cores, kGemmBf16x3 matrix
  // cores with split-bf16 products (FP32 only), lz_gemm_mfma.h; with the
  // matrix cores LW must be null)
  static void proj_dot(const void* A, int P, int a_rows, void* X, const void* LW, int nbnd,
                       int npwx, int nks, int chunk, int nchunk, void* partial,
                       const LzDevState* st, hipStream_t s, int gemm = 0);
  static bool dot_single_tile(int P, int nbnd, int gemm = 0);
  // G per chunk of the matrix-core dot for P rows (about 1024 blocks in all)
  static int mfma_chunk(int P, int nbnd, int npwx, int nks);
  // R[k][p][n] from the partials
  static void reduce(const void* partial, int nchunk, int P, int nbnd, int nks, void* R,
                     hipStream_t s);
  // reduction of the partials and the update coefficients (see lz_linalg.hip)
  static void reduce_coef_in(const void* partial, int nchunk, const void* M, const double* dkb,
                             int nbnd, int nproj, int nks, bool skip_pc, void* C,
                             const LzDevState* st, hipStream_t s);
  static void reduce_coef_out(const void* partial, int nchunk, const void* Cin, const void* M,
                              int nbnd, int nproj, int nks, void* C, const LzDevState* st,
                              hipStream_t s);
  // Y[k][n][G] += sum_{p<P} A[k][p][G] C[k][p][n]; with lzpart the Lanczos
  // sums of (X, Y, y) per block (update_blocks of them)
  static void proj_update(void* Y, const void* A, int P, int a_rows, const void* C, int c_rows,
                          int nbnd, int npwx, int nks, const void* X, const void* y,
                          const double* wk, double* lzpart, const LzDevState* st, hipStream_t s,
                          int gemm = 0);
  static int update_blocks(int P, int nbnd, int npwx, int nks, int gemm = 0);
  // non-Hermitian formation on the output side (P = a_rows = c_rows): as
  // proj_update, then H <- c1 LY' + c2 H with the state coefficients of the
  // u chain (v_chain false) or of the v chain, which also sums (U2, H) and
  // (y, H) into lzpart (4 per block, update_blocks of them)
  static void nh_form(bool v_chain, void* LY, const void* A, int P, const void* C, int nbnd,
                      int npwx, int nks, void* H, const void* y, const void* U2, const double* wk,
                      double* lzpart, const LzDevState* st, hipStream_t s, int gemm = 0);
  // Lanczos: w <- a*LW + b*w
  static void lz_update(void* w, const void* lw, int64_t n, const LzDevState* st, hipStream_t s);
  // user order <-> internal order
  static void perm_in(const void* xu, void* xi, const int* perm, const int* npw, int nks, int nbnd,
                      int npwx, hipStream_t s);
  static void perm_out(const void* xi, void* xu, const int* perm, const int* npw, int nks,
                       int nbnd, int npwx, hipStream_t s);
  static void copy(void* dst, const void* src, int64_t n, hipStream_t s);
};

template <typename T> hipError_t enable_large_lds_fft();
// grid size N served by the register-line plane kernels (0: the LDS-pass kernels)
template <typename T> int reg_plane_size(const Grid3& g);
template <typename T> int reg_plane_len(int n);

void launch_lz_finalize(const double* partial, int nblk, LzDevState* st, double* beta, double* z,
                        int max_steps, double tol, double yscale, hipStream_t s);
// m coefficients, the first m0 computed, beta_i = tail_even / tail_odd beyond;
// gam (complex) non-null for the non-Hermitian recursion
void launch_spectrum(const double* beta, const double* gam, const double* z, int m0, int m,
                     double tail_even, double tail_odd, const double* omega, int nw, double eta,
                     double pref, double fq, double* chi, double* einv, double* loss,
                     hipStream_t s);
// the same with the tail means (beta beyond m0) computed on the device into
// tail[2] from the first m0 coefficients ('osc': per index parity); no host
// round trip
void launch_spectrum_dev_tail(const double* beta, const double* gam, const double* z, int m0,
                              int m, int osc, double* tail, const double* omega, int nw,
                              double eta, double pref, double fq, double* chi, double* einv,
                              double* loss, hipStream_t s);
// non-Hermitian recursion: ||y||^2 partials (kNhNormBlocks x 4) and the
// scalar decisions of one step
constexpr int kNhNormBlocks = 256;
template <typename T>
void launch_nh_norm(const void* y, const double* wk, int64_t per_k, int nks, double* partial,
                    hipStream_t s);
void launch_nh_finalize(const double* partial, int nblk, LzDevState* st, double* beta, double* gam,
                        double* z, int max_steps, double tol, double yscale, hipStream_t s);
void launch_set_state(LzDevState* st, hipStream_t s);

// small dense kernels of the ground-state eigensolver (double precision,
// one block per k; lz_small.h)
constexpr int kSmallOrderMax = 512;
void launch_heev(void* A, int n, int ld, double* w, void* V, int nks, hipStream_t s);
void launch_small_take(void* dst, const void* src, int rows, int cols, int lds, int col0,
                       int src_stride, double alpha, int nks, hipStream_t s);
void launch_orth_coef(const void* Q, const double* lam, int m, double tol, void* C, int* keep,
                      int nks, hipStream_t s);
void launch_mask_dropped(void* T, int n2, int off, int cnt, const int* keep, int nks,
                         hipStream_t s);
// out = c0 HY + c1 Y + c2 Xold with (c0, c1, c2) = coef[k][3] per sphere (the
// Chebyshev filter of the eigensolver; out may alias Xold)
void launch_cheb_step(void* out, const void* HY, const void* Y, const void* Xold,
                      const double* coef, int m, int npwx, int nks, hipStream_t s);
// unit-diagonal form of Gram matrices G[k] (m x m) with the column scales
// d[k] = 1/sqrt(diag), and the rows of coefficients C[k] scaled by d[k]
void launch_gram_unit(void* G, int m, double* dscale, int nks, hipStream_t s);
void launch_row_scale(void* C, int m, const double* dscale, int nks, hipStream_t s);
// ground-state density n0 = sum_b w[b] |ur[b]|^2 and the LDA kernel f_xc(n0)
// (xc = 1 Perdew-Zunger, 0 exchange only) on np grid points (lz_small.h)
void launch_ground_density(const void* ur, const double* w, int nb, int64_t np, int xc,
                           double* n0, double* fxc, hipStream_t s);
void launch_gs_residual(const void* X, const void* HX, const double* theta, const void* kin, int m,
                        int npwx, int nks, double e0, void* R, void* W, hipStream_t s);

constexpr int kStickTile = 16;    // sticks per block in the z passes
constexpr int kStickMaxPt = 8;
constexpr int kColTile = 16;      // grid columns per block in the Hartree z pass
int plane_mp(int n1, int n2);
constexpr int kProjChunk = 64;  // plane waves per block of a projector product
constexpr int kGemmValu = 0, kGemmMfma = 1, kGemmBf16x3 = 2;

}  // namespace lz
