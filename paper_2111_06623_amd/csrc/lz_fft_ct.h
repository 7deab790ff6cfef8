// Compile-time FFTs for the grid lengths of the production workloads.
//
// For a length N listed in ct_radix the radix sequence, the strides and the
// twiddle offsets are compile-time constants, so every index computation of
// a pass folds to shifts and multiplies and every butterfly loop unrolls.
// Radix-8 and radix-16 butterflies run in registers as 4x2 and 4x4
// Cooley-Tukey splits, which halves the number of LDS round trips (and block
// barriers) against a radix-4 plan.  The host builds twiddle tables with the
// same radix lists (make_plan), so table offsets agree with ct_twoff.
#pragma once
#include <type_traits>

#include "lz_device.h"

namespace lz {

__host__ __device__ constexpr int ct_radix(int n, int p) {
  return n == 24   ? (p == 0 ? 8 : p == 1 ? 3 : 0)
         : n == 32 ? (p == 0 ? 8 : p == 1 ? 4 : 0)
         : n == 40 ? (p == 0 ? 8 : p == 1 ? 5 : 0)
         : n == 48 ? (p == 0 ? 16 : p == 1 ? 3 : 0)
         : n == 64 ? (p == 0 ? 16 : p == 1 ? 4 : 0)
         : n == 72 ? (p == 0 ? 8 : p == 1 ? 3 : p == 2 ? 3 : 0)
         : n == 96 ? (p == 0 ? 8 : p == 1 ? 4 : p == 2 ? 3 : 0)
                   : 0;
}

// every length with a compile-time plan, for the kernel dispatch switches
#define LZ_CT_SIZES(X) X(24) X(32) X(40) X(48) X(64) X(72) X(96)
__host__ __device__ constexpr int ct_npass(int n) {
  int c = 0;
  while (c < 8 && ct_radix(n, c) != 0) ++c;
  return c;
}
__host__ __device__ constexpr bool ct_supported(int n) { return ct_npass(n) > 0; }
__host__ __device__ constexpr int ct_ns(int n, int p) {
  int s = 1;
  for (int i = 0; i < p; ++i) s *= ct_radix(n, i);
  return s;
}
__host__ __device__ constexpr int ct_twoff(int n, int p) {
  int o = 0;
  for (int i = 0; i < p; ++i) o += ct_ns(n, i) * (ct_radix(n, i) - 1);
  return o;
}
__host__ __device__ constexpr int ct_twsize(int n) { return ct_twoff(n, ct_npass(n)); }

// exp(2 pi i m / 16)
constexpr double kCos16[16] = {1.0,
                               0.92387953251128675613,
                               0.70710678118654752440,
                               0.38268343236508977173,
                               0.0,
                               -0.38268343236508977173,
                               -0.70710678118654752440,
                               -0.92387953251128675613,
                               -1.0,
                               -0.92387953251128675613,
                               -0.70710678118654752440,
                               -0.38268343236508977173,
                               0.0,
                               0.38268343236508977173,
                               0.70710678118654752440,
                               0.92387953251128675613};
constexpr double kSin16[16] = {0.0,
                               0.38268343236508977173,
                               0.70710678118654752440,
                               0.92387953251128675613,
                               1.0,
                               0.92387953251128675613,
                               0.70710678118654752440,
                               0.38268343236508977173,
                               0.0,
                               -0.38268343236508977173,
                               -0.70710678118654752440,
                               -0.92387953251128675613,
                               -1.0,
                               -0.92387953251128675613,
                               -0.70710678118654752440,
                               -0.38268343236508977173};

// a * exp(DIR 2 pi i M / 16), exact for the quarter turns
template <typename T, int M, int DIR>
__device__ __forceinline__ cplx<T> w16(cplx<T> a) {
  constexpr int m = ((M % 16) + 16) % 16;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return mul_i<T>(a, DIR);
  } else if constexpr (m == 8) {
    return mk<T>(-a.x, -a.y);
  } else if constexpr (m == 12) {
    return mul_i<T>(a, -DIR);
  } else {
    const T c = T(kCos16[m]);
    const T s = T(DIR * kSin16[m]);
    return mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// radix-16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <typename T, int DIR, int N2>
__device__ __forceinline__ void dft16_stage1(const cplx<T>* v, cplx<T> (&y)[4][4]) {
  cplx<T> a[4] = {v[N2], v[4 + N2], v[8 + N2], v[12 + N2]};
  Dft<T, 4, DIR>::run(a);
  y[N2][0] = a[0];
  y[N2][1] = w16<T, N2 * 1, DIR>(a[1]);
  y[N2][2] = w16<T, N2 * 2, DIR>(a[2]);
  y[N2][3] = w16<T, N2 * 3, DIR>(a[3]);
}

template <typename T, int DIR> struct Dft<T, 16, DIR> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> y[4][4];
    dft16_stage1<T, DIR, 0>(v, y);
    dft16_stage1<T, DIR, 1>(v, y);
    dft16_stage1<T, DIR, 2>(v, y);
    dft16_stage1<T, DIR, 3>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cplx<T> b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<T, 4, DIR>::run(b);
      v[k1] = b[0];
      v[k1 + 4] = b[1];
      v[k1 + 8] = b[2];
      v[k1 + 12] = b[3];
    }
  }
};

// radix-8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2
template <typename T, int DIR, int N2>
__device__ __forceinline__ void dft8_stage1(const cplx<T>* v, cplx<T> (&y)[2][4]) {
  cplx<T> a[4] = {v[N2], v[2 + N2], v[4 + N2], v[6 + N2]};
  Dft<T, 4, DIR>::run(a);
  y[N2][0] = a[0];
  y[N2][1] = w16<T, 2 * N2 * 1, DIR>(a[1]);
  y[N2][2] = w16<T, 2 * N2 * 2, DIR>(a[2]);
  y[N2][3] = w16<T, 2 * N2 * 3, DIR>(a[3]);
}

template <typename T, int DIR> struct Dft<T, 8, DIR> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> y[2][4];
    dft8_stage1<T, DIR, 0>(v, y);
    dft8_stage1<T, DIR, 1>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      v[k1] = cadd<T>(y[0][k1], y[1][k1]);
      v[k1 + 4] = csub<T>(y[0][k1], y[1][k1]);
    }
  }
};

// Layouts of a batch of transforms in LDS with compile-time pitch.
template <int PITCH> struct LayRows {      // rows listed in an LDS array, unit stride
  const int* rows;
  static constexpr int stride = 1;
  __device__ __forceinline__ int base(int b) const { return rows[b] * PITCH; }
};
template <int PITCH> struct LayRowsAll {   // every row, unit stride
  static constexpr int stride = 1;
  __device__ __forceinline__ int base(int b) const { return b * PITCH; }
};
template <int PITCH> struct LayCols {      // every column, stride PITCH
  static constexpr int stride = PITCH;
  __device__ __forceinline__ int base(int b) const { return b; }
};

// One pass of a compile-time plan over nbatch <= NBMAX transforms, in place,
// NT threads: loads into registers, barrier, stores, barrier.  In the last
// pass (NS R = N, so M = NS and k = j) a butterfly stores to exactly the
// elements j + s M it loaded from, which no other butterfly touches: its
// stores cannot overwrite what another thread has still to load, and the
// barrier between loads and stores is left out.
// Pointwise work folded into the stores of a plan's last pass: no factor.
struct NoEpilogue {
  template <typename T>
  __device__ __forceinline__ T load(int, int) const { return T(1); }
};

template <typename T, int N, int P, int DIR, int NBMAX, typename L, int NT = 256,
          typename E = NoEpilogue>
__device__ __forceinline__ void ct_pass(cplx<T>* lds, const L& lay, int nbatch,
                                        const cplx<T>* tw, int tid, const E& epi = E{}) {
  constexpr int R = ct_radix(N, P);
  constexpr int NS = ct_ns(N, P);
  constexpr int M = N / R;
  constexpr bool LAST = P + 1 == ct_npass(N);
  static_assert(!LAST || NS == M, "the last pass of a plan maps each butterfly onto itself");
  constexpr int MAXB = (NBMAX * M + NT - 1) / NT;
  const cplx<T>* twp = tw + ct_twoff(N, P);
  const int total = nbatch * M;
  // with an epilogue, the last pass scales output s of butterfly j of line b
  // (element j + s M of the line) by epi.load(b, j + s M), loaded before the
  // butterfly's LDS reads so that its latency overlaps them
  constexpr bool EPI = LAST && !std::is_same<E, NoEpilogue>::value;
  cplx<T> v[MAXB][R];
  T f[EPI ? MAXB : 1][EPI ? R : 1];
  int bbase[MAXB], bo[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int t = tid + i * NT;
    if (t < total) {
      // butterfly j of line b, lines fastest: the lanes of a wave take the
      // same butterfly of consecutive lines, whose elements lie a line
      // pitch apart (odd in complex elements), so their loads and stores
      // fall in distinct LDS banks; with the butterflies of one line on
      // neighbouring lanes, the first pass's stores (outputs j*R + s) put
      // the lanes of a line 16 elements apart, on the same banks
      const int j = t / nbatch;
      const int b = t - j * nbatch;
      const int k = j % NS;
      const int base = lay.base(b);
      bbase[i] = base;
      bo[i] = (j / NS) * NS * R + k;
      if constexpr (EPI) {
#pragma unroll
        for (int s = 0; s < R; ++s) f[i][s] = epi.template load<T>(b, j + s * M);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[base + (j + r * M) * L::stride];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = twp[k * (R - 1) + (r - 1)];
          if (DIR > 0) w.y = -w.y;
          v[i][r] = cmul<T>(v[i][r], w);
        }
      }
      Dft<T, R, DIR>::run(v[i]);
    }
  }
  if constexpr (!LAST) __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int t = tid + i * NT;
    if (t < total) {
      if constexpr (EPI) {
#pragma unroll
        for (int s = 0; s < R; ++s) v[i][s] = cscale<T>(v[i][s], f[i][s]);
      }
#pragma unroll
      for (int s = 0; s < R; ++s) lds[bbase[i] + (bo[i] + s * NS) * L::stride] = v[i][s];
    }
  }
  __syncthreads();
}

template <typename T, int N, int DIR, int NBMAX, typename L, int NT = 256,
          typename E = NoEpilogue>
__device__ __forceinline__ void ct_fft(cplx<T>* lds, const L& lay, int nbatch, const cplx<T>* tw,
                                       int tid, const E& epi = E{}) {
  static_assert(ct_supported(N), "no compile-time plan for this length");
  ct_pass<T, N, 0, DIR, NBMAX, L, NT, E>(lds, lay, nbatch, tw, tid, epi);
  if constexpr (ct_npass(N) > 1) ct_pass<T, N, 1, DIR, NBMAX, L, NT, E>(lds, lay, nbatch, tw, tid, epi);
  if constexpr (ct_npass(N) > 2) ct_pass<T, N, 2, DIR, NBMAX, L, NT, E>(lds, lay, nbatch, tw, tid, epi);
}

}  // namespace lz
