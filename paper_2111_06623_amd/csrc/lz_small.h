// Small dense kernels of the ground-state eigensolver (Sec. 3.1: the valence
// Kohn-Sham orbitals that precede the linear-response run): one block per
// k-point on matrices of a few hundred rows at most, double precision,
// row-major [k][n][ld].
#pragma once
#include "lz_kernels.h"

namespace lz {

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

constexpr int kSmallMax = 512;  // largest matrix order of the small kernels
constexpr int kHeevThreads = 1024;  // threads of the one block per matrix of k_heev_jacobi

// Eigen-decomposition of the Hermitian part of A[k] (n x n, leading dimension
// ld) by two-sided cyclic Jacobi with the round-robin parallel ordering: in
// each of the ne - 1 rounds of a sweep (ne = n rounded up to even; an odd n
// gets an idle partner) the ne / 2 disjoint pairs (p, q) are rotated at once.
// A pair with a_pq = |a_pq| e^{i phi} is rotated by J = P R, P = diag(1,
// e^{-i phi}), R the real Jacobi rotation of [[a_pp, |a_pq|], [|a_pq|, a_qq]]
// (t = sign(tau) / (|tau| + sqrt(1 + tau^2)), tau = (a_qq - a_pp) / 2|a_pq|):
// columns [a_ip, a_iq] J, then rows J^H [a_pj; a_qj], and V <- V J.  Sweeps
// stop when the off-diagonal norm is below 1e-15 of the matrix norm (or
// after max_sweeps).  Eigenvalues ascending into w[k][0..n), eigenvectors
// into the columns of V[k]; A[k] is destroyed.
__global__ __launch_bounds__(kHeevThreads) void k_heev_jacobi(double2* __restrict__ A, int n, int ld,
                                                     double* __restrict__ w,
                                                     double2* __restrict__ V, int max_sweeps) {
  __shared__ double rc[kSmallMax / 2], rs[kSmallMax / 2];
  __shared__ double2 ru[kSmallMax / 2];
  __shared__ int rp[kSmallMax / 2], rq[kSmallMax / 2];
  __shared__ double red[kHeevThreads];
  __shared__ int idx[kSmallMax];
  __shared__ double dsort[kSmallMax];
  __shared__ int stop;
  const int k = blockIdx.x, tid = threadIdx.x;
  double2* a = A + (int64_t)k * n * ld;
  double2* v = V + (int64_t)k * n * ld;
  const int ne = n + (n & 1);
  const int npair = ne / 2;
  // Hermitian part, V = I
  for (int t = tid; t < n * n; t += kHeevThreads) {
    const int i = t / n, j = t - i * n;
    if (i <= j) {
      const double2 x = a[i * ld + j], y = a[j * ld + i];
      const double2 h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
      a[i * ld + j] = i == j ? make_double2(h.x, 0.0) : h;
      if (i != j) a[j * ld + i] = zconj(h);
    }
    v[i * ld + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal against total Frobenius norm
    double off = 0.0, tot = 0.0;
    for (int t = tid; t < n * n; t += kHeevThreads) {
      const int i = t / n, j = t - i * n;
      const double2 x = a[i * ld + j];
      const double m2 = x.x * x.x + x.y * x.y;
      tot += m2;
      if (i != j) off += m2;
    }
    red[tid] = off;
    __syncthreads();
    for (int h = kHeevThreads / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int h = kHeevThreads / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) stop = (offs <= 1e-30 * red[0]) ? 1 : 0;
    __syncthreads();
    if (stop) break;
    for (int r = 0; r < ne - 1; ++r) {
      if (tid < npair) {
        int p, q;
        if (tid == 0) {
          p = r % (ne - 1);
          q = ne - 1;
        } else {
          p = (r + tid) % (ne - 1);
          q = (r - tid + ne - 1) % (ne - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        double2 u = make_double2(1.0, 0.0);
        if (q < n) {
          const double2 b = a[p * ld + q];
          const double g = sqrt(b.x * b.x + b.y * b.y);
          const double app = a[p * ld + p].x, aqq = a[q * ld + q].x;
          if (g > 1e-300 && g > 1e-18 * (fabs(app) + fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * g);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            u = make_double2(b.x / g, b.y / g);
          }
        }
        rc[tid] = c;
        rs[tid] = s;
        ru[tid] = u;
        rp[tid] = p;
        rq[tid] = q < n ? q : -1;
      }
      __syncthreads();
      // columns of A and V: [x_p, x_q] <- [x_p c - x_q u* s, x_p s + x_q u* c]
      for (int t = tid; t < npair * n; t += kHeevThreads) {
        const int pr = t / n, i = t - pr * n;
        const int p = rp[pr], q = rq[pr];
        if (q < 0 || rs[pr] == 0.0) continue;
        const double c = rc[pr], s = rs[pr];
        const double2 us = zconj(ru[pr]);
        const double2 x = a[i * ld + p], y = a[i * ld + q];
        const double2 yu = zmul(y, us);
        a[i * ld + p] = make_double2(c * x.x - s * yu.x, c * x.y - s * yu.y);
        a[i * ld + q] = make_double2(s * x.x + c * yu.x, s * x.y + c * yu.y);
        const double2 xv = v[i * ld + p], yv = v[i * ld + q];
        const double2 yvu = zmul(yv, us);
        v[i * ld + p] = make_double2(c * xv.x - s * yvu.x, c * xv.y - s * yvu.y);
        v[i * ld + q] = make_double2(s * xv.x + c * yvu.x, s * xv.y + c * yvu.y);
      }
      __syncthreads();
      // rows of A: [x_p; x_q] <- [c x_p - u s x_q; s x_p + u c x_q]
      for (int t = tid; t < npair * n; t += kHeevThreads) {
        const int pr = t / n, j = t - pr * n;
        const int p = rp[pr], q = rq[pr];
        if (q < 0 || rs[pr] == 0.0) continue;
        const double c = rc[pr], s = rs[pr];
        const double2 u = ru[pr];
        const double2 x = a[p * ld + j], y = a[q * ld + j];
        const double2 uy = zmul(u, y);
        a[p * ld + j] = make_double2(c * x.x - s * uy.x, c * x.y - s * uy.y);
        a[q * ld + j] = make_double2(s * x.x + c * uy.x, s * x.y + c * uy.y);
      }
      __syncthreads();
      // the rotated pair is now diagonal
      if (tid < npair) {
        const int p = rp[tid], q = rq[tid];
        if (q >= 0 && rs[tid] != 0.0) {
          a[p * ld + q] = make_double2(0.0, 0.0);
          a[q * ld + p] = make_double2(0.0, 0.0);
          a[p * ld + p].y = 0.0;
          a[q * ld + q].y = 0.0;
        }
      }
      __syncthreads();
    }
  }
  // ascending order (selection of indices by one thread), columns of V permuted
  if (tid == 0) {
    for (int i = 0; i < n; ++i) {
      idx[i] = i;
      dsort[i] = a[i * ld + i].x;
    }
    for (int i = 0; i < n; ++i) {
      int best = i;
      for (int j = i + 1; j < n; ++j)
        if (dsort[j] < dsort[best]) best = j;
      const double td = dsort[i]; dsort[i] = dsort[best]; dsort[best] = td;
      const int ti = idx[i]; idx[i] = idx[best]; idx[best] = ti;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kHeevThreads) w[(int64_t)k * n + i] = dsort[i];
  for (int t = tid; t < n * n; t += kHeevThreads) {
    const int i = t / n, j = t - i * n;
    a[i * ld + j] = v[i * ld + idx[j]];
  }
  __syncthreads();
  for (int t = tid; t < n * n; t += kHeevThreads) {
    const int i = t / n, j = t - i * n;
    v[i * ld + j] = a[i * ld + j];
  }
}

// dst[k][i][j] = alpha src[k][i][col0 + j], i < rows, j < cols (src leading
// dimension lds, dst leading dimension cols)
__global__ __launch_bounds__(256) void k_small_take(double2* __restrict__ dst,
                                                    const double2* __restrict__ src, int rows,
                                                    int cols, int lds, int col0, int src_stride,
                                                    double alpha) {
  const int k = blockIdx.x;
  for (int t = threadIdx.x; t < rows * cols; t += 256) {
    const int i = t / cols, j = t - i * cols;
    const double2 x = src[(int64_t)k * src_stride + i * lds + col0 + j];
    dst[(int64_t)k * rows * cols + t] = make_double2(alpha * x.x, alpha * x.y);
  }
}

// Orthonormalising coefficients from the eigen-decomposition S = Q diag(lam) Q^H
// of a Gram matrix (m x m, ascending lam): C[:, j] = Q[:, j] / sqrt(lam_j) for
// lam_j > tol max(lam), else 0 (a direction the block does not span); keep[k][j]
// is 1 for the kept columns.
__global__ __launch_bounds__(256) void k_orth_coef(const double2* __restrict__ Q,
                                                   const double* __restrict__ lam, int m,
                                                   double tol, double2* __restrict__ C,
                                                   int* __restrict__ keep) {
  const int k = blockIdx.x;
  const double lmax = lam[(int64_t)k * m + m - 1];
  for (int t = threadIdx.x; t < m * m; t += 256) {
    const int i = t / m, j = t - i * m;
    const double l = lam[(int64_t)k * m + j];
    const bool ok = lmax > 0.0 && l > tol * lmax;
    const double f = ok ? 1.0 / sqrt(l) : 0.0;
    const double2 q = Q[(int64_t)k * m * m + t];
    C[(int64_t)k * m * m + t] = make_double2(f * q.x, f * q.y);
    if (i == 0) keep[(int64_t)k * m + j] = ok ? 1 : 0;
  }
}

// T[k] (n2 x n2): on the basis vectors off + j that were dropped (keep[k][j]
// == 0, j < cnt: zero rows and columns) a diagonal above every eigenvalue of the rest,
// 2 (g + 1) with g the largest Gershgorin row sum, so that they sort last
// (a scale comparable with T keeps the relative stopping test of the
// Jacobi sweeps meaningful)
__global__ __launch_bounds__(256) void k_mask_dropped(double2* __restrict__ T, int n2, int off,
                                                      int cnt, const int* __restrict__ keep) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double2* t = T + (int64_t)k * n2 * n2;
  double g = 0.0;
  for (int i = threadIdx.x; i < n2; i += 256) {
    double r = 0.0;
    for (int j = 0; j < n2; ++j) {
      const double2 x = t[(int64_t)i * n2 + j];
      r += sqrt(x.x * x.x + x.y * x.y);
    }
    g = fmax(g, r);
  }
  red[threadIdx.x] = g;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double pen = 2.0 * (red[0] + 1.0);
  for (int j = threadIdx.x; j < cnt; j += 256)
    if (!keep[(int64_t)k * cnt + j]) {
      const int d = off + j;
      t[(int64_t)d * n2 + d] = make_double2(pen, 0.0);
    }
}

// Residuals and preconditioned corrections of a block of Ritz pairs:
// R = H x_n - theta_n x_n;  W = R * p(kin_G / e0), p(x) the rational kinetic
// preconditioner (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4)
// of Teter, Payne and Allan (1989).  R is left in Rout for its norms.
__global__ __launch_bounds__(256) void k_gs_residual(const double2* __restrict__ X,
                                                     const double2* __restrict__ HX,
                                                     const double* __restrict__ theta,
                                                     const double* __restrict__ kin, int m,
                                                     int npwx, int nks, double e0,
                                                     double2* __restrict__ Rout,
                                                     double2* __restrict__ W) {
  const int64_t total = (int64_t)nks * m * npwx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kb = i / npwx;  // k * m + n
    const int g = (int)(i - kb * npwx);
    const int k = (int)(kb / m);
    const double th = theta[kb];
    const double2 x = X[i], h = HX[i];
    const double2 r = make_double2(h.x - th * x.x, h.y - th * x.y);
    Rout[i] = r;
    const double y = kin[(int64_t)k * npwx + g] / e0;
    const double num = 27.0 + y * (18.0 + y * (12.0 + 8.0 * y));
    const double p = num / (num + 16.0 * y * y * y * y);
    W[i] = make_double2(p * r.x, p * r.y);
  }
}

// One step of the Chebyshev filter of the eigensolver (the three-term
// recurrence of scaled Chebyshev polynomials of H):
//   out = c0 HY + c1 Y + c2 Xold,   (c0, c1, c2) = coef[k][0..3) per sphere k
// on nks blocks of m vectors of npwx plane waves; out may alias Xold.
__global__ __launch_bounds__(256) void k_cheb_step(double2* out, const double2* __restrict__ HY,
                                                   const double2* __restrict__ Y,
                                                   const double2* Xold,
                                                   const double* __restrict__ coef, int m,
                                                   int npwx, int nks) {
  const int64_t total = (int64_t)nks * m * npwx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / ((int64_t)m * npwx));
    const double c0 = coef[3 * k], c1 = coef[3 * k + 1], c2 = coef[3 * k + 2];
    const double2 h = HY[i], y = Y[i];
    double2 r = make_double2(c0 * h.x + c1 * y.x, c0 * h.y + c1 * y.y);
    if (c2 != 0.0) {
      const double2 x = Xold[i];
      r.x += c2 * x.x;
      r.y += c2 * x.y;
    }
    out[i] = r;
  }
}

// Unit-diagonal form of a Gram matrix (the Gram matrix of the block with its
// columns scaled to unit norm): d_j = 1/sqrt(G_jj), G_ij <- d_i G_ij d_j, and
// d into dscale[k][m].  A filtered block whose columns differ in norm by many
// orders (the filter damps the upper columns of the block) keeps their
// distinct directions through this scaling.
__global__ __launch_bounds__(256) void k_gram_unit(double2* __restrict__ G, int m,
                                                   double* __restrict__ dscale) {
  const int k = blockIdx.x;
  double2* g = G + (int64_t)k * m * m;
  double* d = dscale + (int64_t)k * m;
  for (int j = threadIdx.x; j < m; j += 256) {
    const double x = g[(int64_t)j * m + j].x;
    d[j] = x > 0.0 ? 1.0 / sqrt(x) : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m * m; t += 256) {
    const int i = t / m, j = t - i * m;
    const double f = d[i] * d[j];
    g[t] = make_double2(f * g[t].x, f * g[t].y);
  }
}

// C[k][i][j] *= d[k][i] (rows of coefficients, after k_gram_unit)
__global__ __launch_bounds__(256) void k_row_scale(double2* __restrict__ C, int m,
                                                   const double* __restrict__ dscale) {
  const int k = blockIdx.x;
  for (int t = threadIdx.x; t < m * m; t += 256) {
    const int i = t / m;
    const double f = dscale[(int64_t)k * m + i];
    double2& c = C[(int64_t)k * m * m + t];
    c = make_double2(f * c.x, f * c.y);
  }
}

// Ground-state density and adiabatic LDA kernel (Sec. 3.1; the kernel of
// the xc response potential, Sec. 2.2): from the valence orbitals on the
// grid, raw sums ur[b][p] = sum_G u_b(G) e^{iG.r_p} (the Omega^-1/2 of the
// cell normalisation is in w), n0[p] = sum_b w[b] |ur[b][p]|^2 with
// w[b] = 2 w_k / Omega (spin-unpolarised), bands added in index order; then
// f_xc(n0) = d^2(n eps_xc)/dn^2, zero where n0 < 1e-10 bohr^-3.
//   exchange (Slater): n eps_x = -(3/4)(3/pi)^(1/3) n^(4/3),
//                      f_x = -(1/3)(3/pi)^(1/3) n^(-2/3);
//   correlation (Perdew-Zunger 1981, unpolarised, Hartree units), with
//   r_s = (3/(4 pi n))^(1/3) and dr_s/dn = -r_s/(3n):
//     r_s >= 1: eps_c = gamma / (1 + beta1 sqrt(r_s) + beta2 r_s)
//     r_s <  1: eps_c = A ln r_s + B + C r_s ln r_s + D r_s
//     f_c = (r_s^2 eps_c'' - 2 r_s eps_c') / (9 n)   (derivatives in r_s).
// xc = 1: exchange and correlation; xc = 0: exchange only.
__device__ __forceinline__ double lda_fxc(double n, int xc) {
  if (!(n >= 1e-10)) return 0.0;
  const double third = 1.0 / 3.0;
  double f = -third * cbrt(3.0 / M_PI) * pow(n, -2.0 * third);
  if (xc) {
    const double rs = cbrt(3.0 / (4.0 * M_PI * n));
    double e1, e2;
    if (rs >= 1.0) {
      const double gam = -0.1423, b1 = 1.0529, b2 = 0.3334;
      const double sr = sqrt(rs);
      const double den = 1.0 + b1 * sr + b2 * rs;
      const double d1 = 0.5 * b1 / sr + b2;
      const double d2 = -0.25 * b1 / (rs * sr);
      e1 = -gam * d1 / (den * den);
      e2 = -gam * d2 / (den * den) + 2.0 * gam * d1 * d1 / (den * den * den);
    } else {
      const double A = 0.0311, C = 0.0020, D = -0.0116;
      e1 = A / rs + C * (log(rs) + 1.0) + D;
      e2 = -A / (rs * rs) + C / rs;
    }
    f += (rs * rs * e2 - 2.0 * rs * e1) / (9.0 * n);
  }
  return f;
}

__global__ __launch_bounds__(256) void k_ground_density(const double2* __restrict__ ur,
                                                        const double* __restrict__ w, int nb,
                                                        int64_t np, int xc,
                                                        double* __restrict__ n0,
                                                        double* __restrict__ fxc) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double2 u = ur[(int64_t)b * np + p];
      acc += w[b] * (u.x * u.x + u.y * u.y);
    }
    n0[p] = acc;
    fxc[p] = lda_fxc(acc, xc);
  }
}

}  // namespace lz