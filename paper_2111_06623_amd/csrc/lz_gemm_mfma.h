// Projector products on the matrix cores (MFMA) for instances with many
// bands and projectors (Sec. 2.3 P_c and the separable projectors; the
// products are complex GEMMs over plane waves).  Same contracts as the
// vector-ALU kernels k_proj_dot / k_proj_update in lz_linalg.hip:
//
//   dot     partial[k][chunk][n][p] = sum_{G in chunk} conj(A[k][p][G]) X[k][n][G]
//   update  Y[k][n][G] += sum_p A[k][p][G] C[k][p][n], then the epilogue of
//           the recursion (plain, Lanczos sums, non-Hermitian formation)
//
// A complex product is four real MFMA products into separate real and
// imaginary accumulators.  A wave owns a 32 x 32 complex output tile:
//   float   one v_mfma_f32_32x32x2f32 per real product, k step 2; lane l
//           supplies left[l % 32][l / 32] and right[l / 32][l % 32], and
//           holds outputs (8 (v / 4) + 4 (l / 32) + v % 4, l % 32), v < 16;
//   double  2 x 2 tiles of v_mfma_f64_16x16x4f64, k step 4; lane l supplies
//           left[l % 16][l / 16] and right[l / 16][l % 16] per tile and
//           holds outputs (l / 16 + 4 w, l % 16), w < 4, per tile.
// (Lane layouts checked on the device against a host product.)  A block is
// 2 x 2 waves over a 64 x 64 output tile; both operands of a k chunk are
// staged in LDS, and the next chunk is fetched into registers while the
// matrix cores work on the current one.  Every sum has a fixed order: results do not depend on
// scheduling.
#pragma once
#include "lz_kernels.h"

namespace lz {

typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct WaveTile;

template <> struct WaveTile<float> {
  static constexpr int KS = 2;   // k per step
  static constexpr int NV = 16;  // outputs per lane
  mfma_f32x16 re, im;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int v = 0; v < 16; ++v) { re[v] = 0.f; im[v] = 0.f; }
  }
  // one k step; left(row, kq) and right(kq, col) return the operands.
  // CONJ: accumulate conj(left) * right, else left * right.
  template <bool CONJ, typename FL, typename FR>
  __device__ __forceinline__ void step(int l, FL left, FR right) {
    const float2 a = left(l % 32, l / 32);
    const float2 b = right(l / 32, l % 32);
    const float ai = CONJ ? a.y : -a.y;  // re += ar br + (conj ? +ai bi : -ai bi)
    re = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, b.x, im, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int v, int l) { return 8 * (v / 4) + 4 * (l / 32) + (v % 4); }
  __device__ __forceinline__ static int col(int v, int l) { return l % 32; }
  __device__ __forceinline__ float2 at(int v) const { return make_float2(re[v], im[v]); }
};

template <> struct WaveTile<double> {
  static constexpr int KS = 4;
  static constexpr int NV = 16;
  mfma_f64x4 re[2][2], im[2][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int w = 0; w < 4; ++w) { re[r][c][w] = 0.0; im[r][c][w] = 0.0; }
  }
  template <bool CONJ, typename FL, typename FR>
  __device__ __forceinline__ void step(int l, FL left, FR right) {
    double2 a[2], b[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) a[r] = left(16 * r + l % 16, l / 16);
#pragma unroll
    for (int c = 0; c < 2; ++c) b[c] = right(l / 16, 16 * c + l % 16);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const double ai = CONJ ? a[r].y : -a[r].y;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        re[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r].x, b[c].x, re[r][c], 0, 0, 0);
        re[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b[c].y, re[r][c], 0, 0, 0);
        im[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r].x, b[c].y, im[r][c], 0, 0, 0);
        im[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, b[c].x, im[r][c], 0, 0, 0);
      }
    }
  }
  // v = 8 r + 4 c + w
  __device__ __forceinline__ static int row(int v, int l) { return 16 * (v / 8) + l / 16 + 4 * (v % 4); }
  __device__ __forceinline__ static int col(int v, int l) { return 16 * ((v / 4) % 2) + l % 16; }
  __device__ __forceinline__ double2 at(int v) const {
    return make_double2(re[v / 8][(v / 4) % 2][v % 4], im[v / 8][(v / 4) % 2][v % 4]);
  }
};

// k chunk staged per LDS round (multiple of the MFMA k step)
template <typename T> constexpr int mfma_kc() { return sizeof(T) == 4 ? 32 : 16; }
constexpr int kMfmaTile = 64;  // block output tile (both dimensions)

// ---------------------------------------------------------------------------
// dot: block = (p tile, n tile) x G chunk x k
// ---------------------------------------------------------------------------
template <typename T>
struct ProjDotMfmaArgs {
  const cplx<T>* A;
  int P;
  int a_rows;
  const cplx<T>* X;
  int nbnd;
  int npwx;
  int chunk;
  int nchunk;
  cplx<T>* partial;
  const LzDevState* st;
};

template <typename T>
__device__ __forceinline__ void proj_dot_mfma_block(const cplx<T>* __restrict__ A, int P,
                                                    int a_rows, const cplx<T>* __restrict__ X,
                                                    int nbnd, int npwx, int chunk, int nchunk,
                                                    cplx<T>* __restrict__ partial,
                                                    const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  constexpr int BT = kMfmaTile, KC = mfma_kc<T>(), PITCH = KC + 1;
  __shared__ cplx<T> As[BT * PITCH], Xs[BT * PITCH];
  const int tilesN = (nbnd + BT - 1) / BT;
  const int p0 = (vb.x / tilesN) * BT, n0 = (vb.x % tilesN) * BT;
  const int ci = vb.y, k = vb.z;
  const int tid = threadIdx.x, l = tid % 64, wave = tid / 64;
  const int wp = (wave / 2) * 32, wn = (wave % 2) * 32;
  const cplx<T>* Ak = A + (int64_t)k * a_rows * npwx;
  const cplx<T>* Xk = X + (int64_t)k * nbnd * npwx;
  const int g_begin = ci * chunk, g_end = min(npwx, g_begin + chunk);
  const cplx<T> zero = mk<T>(T(0), T(0));
  WaveTile<T> acc;
  acc.zero();
  // the next chunk is fetched into registers while the current one computes
  constexpr int NPT = BT * KC / 256;
  T rar[NPT], rai[NPT], rxr[NPT], rxi[NPT];  // split parts: kept in registers
  {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int r = t / KC, c = t - r * KC;
      const int g = (g_begin) + c;
      const int p = p0 + r, n = n0 + r;
      const cplx<T> av = (p < P && g < g_end) ? Ak[(int64_t)p * npwx + g] : zero;
      const cplx<T> xv = (n < nbnd && g < g_end) ? Xk[(int64_t)n * npwx + g] : zero;
      rar[i] = av.x; rai[i] = av.y; rxr[i] = xv.x; rxi[i] = xv.y;
    }
  }
  for (int g0 = g_begin; g0 < g_end; g0 += KC) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int r = t / KC, c = t - r * KC;
      As[r * PITCH + c] = mk<T>(rar[i], rai[i]);
      Xs[r * PITCH + c] = mk<T>(rxr[i], rxi[i]);
    }
    __syncthreads();
    if (g0 + KC < g_end) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int r = t / KC, c = t - r * KC;
      const int g = (g0 + KC) + c;
      const int p = p0 + r, n = n0 + r;
      const cplx<T> av = (p < P && g < g_end) ? Ak[(int64_t)p * npwx + g] : zero;
      const cplx<T> xv = (n < nbnd && g < g_end) ? Xk[(int64_t)n * npwx + g] : zero;
      rar[i] = av.x; rai[i] = av.y; rxr[i] = xv.x; rxi[i] = xv.y;
    }
  }
#pragma unroll
    for (int kk = 0; kk < KC; kk += WaveTile<T>::KS) {
      acc.template step<true>(
          l, [&](int row, int kq) { return As[(wp + row) * PITCH + kk + kq]; },
          [&](int kq, int col) { return Xs[(wn + col) * PITCH + kk + kq]; });
    }
    __syncthreads();
  }
  cplx<T>* out = partial + ((int64_t)k * nchunk + ci) * P * nbnd;
#pragma unroll
  for (int v = 0; v < WaveTile<T>::NV; ++v) {
    const int p = p0 + wp + WaveTile<T>::row(v, l), n = n0 + wn + WaveTile<T>::col(v, l);
    if (p < P && n < nbnd) out[(int64_t)n * P + p] = acc.at(v);
  }
}

template <typename T, bool BAT = false>
__global__ __launch_bounds__(256) void k_proj_dot_mfma(ProjDotMfmaArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (proj_dot_mfma_block<T>(a_.A, a_.P, a_.a_rows, a_.X, a_.nbnd, a_.npwx, a_.chunk,
                                     a_.nchunk, a_.partial, a_.st, vb)));
}

// Epilogue of an update tile (MODE as k_proj_update): the wave's outputs
// at band bw + row, plane wave gw + col; block sums into lzpart.
template <typename T, int MODE, typename TILE>
__device__ __forceinline__ void update_epilogue(const TILE& acc, cplx<T>* __restrict__ Y,
                                                int nbnd, int npwx,
                                                cplx<T>* __restrict__ X,
                                                const cplx<T>* __restrict__ yv,
                                                const cplx<T>* __restrict__ U2,
                                                const double* __restrict__ wk,
                                                double* __restrict__ lzpart, const LzDevState* st,
                                                int bw, int gw, int k, int l,
                                                double (*red)[256], const VBlock& vb) {
  constexpr bool DOTS = MODE == kUpdDots || MODE == kUpdNhV;
  constexpr int NR = MODE == kUpdNhV ? 4 : 3;
  const int tid = threadIdx.x;
  const cplx<T> zero = mk<T>(T(0), T(0));
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int64_t kb = (int64_t)k * nbnd * npwx;
  const double w = DOTS ? wk[k] : 0.0;
  cplx<T> c1 = zero, c2 = zero;
  if constexpr (MODE == kUpdNhU) {
    c1 = mk<T>(T(st->cu1[0]), T(st->cu1[1]));
    c2 = mk<T>(T(st->cu2[0]), T(st->cu2[1]));
  } else if constexpr (MODE == kUpdNhV) {
    c1 = mk<T>(T(st->cv1[0]), T(st->cv1[1]));
    c2 = mk<T>(T(st->cv2[0]), T(st->cv2[1]));
  }
#pragma unroll
  for (int v = 0; v < TILE::NV; ++v) {
    const int b = bw + TILE::row(v, l), g = gw + TILE::col(v, l);
    if (b < nbnd && g < npwx) {
      const int64_t o = kb + (int64_t)b * npwx + g;
      const cplx<T> yn = cadd<T>(Y[o], acc.at(v));
      if constexpr (MODE == kUpdPlain || MODE == kUpdDots) Y[o] = yn;
      if constexpr (MODE == kUpdDots) {
        const cplx<T> xv = X[o], rv = yv[o];
        s0 += w * (double(xv.x) * double(yn.x) + double(xv.y) * double(yn.y));
        s1 += w * (double(rv.x) * double(xv.x) + double(rv.y) * double(xv.y));
        s2 += w * (double(rv.x) * double(xv.y) - double(rv.y) * double(xv.x));
      }
      if constexpr (MODE == kUpdNhU || MODE == kUpdNhV) {
        const cplx<T> h = cadd<T>(cmul<T>(c1, yn), cmul<T>(c2, X[o]));
        X[o] = h;
        if constexpr (MODE == kUpdNhV) {
          const cplx<T> uv = U2[o], rv = yv[o];
          s0 += w * (double(uv.x) * double(h.x) + double(uv.y) * double(h.y));
          s1 += w * (double(uv.x) * double(h.y) - double(uv.y) * double(h.x));
          s2 += w * (double(rv.x) * double(h.x) + double(rv.y) * double(h.y));
          s3 += w * (double(rv.x) * double(h.y) - double(rv.y) * double(h.x));
        }
      }
    }
  }
  if constexpr (DOTS) {
    const double sv[4] = {s0, s1, s2, s3};
#pragma unroll
    for (int r = 0; r < NR; ++r) red[r][tid] = sv[r];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
#pragma unroll
        for (int r = 0; r < NR; ++r) red[r][tid] += red[r][tid + h];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int blk = (vb.z * vb.ny + vb.y) * vb.nx + vb.x;
#pragma unroll
      for (int r = 0; r < NR; ++r) lzpart[NR * blk + r] = red[r][0];
    }
  }
}

// ---------------------------------------------------------------------------
// update: block = (G tile, band tile, k); epilogue MODE as k_proj_update
// ---------------------------------------------------------------------------
template <typename T>
struct ProjUpdateMfmaArgs {
  cplx<T>* Y;
  const cplx<T>* A;
  int P;
  int a_rows;
  const cplx<T>* C;
  int c_rows;
  int nbnd;
  int npwx;
  cplx<T>* X;
  const cplx<T>* yv;
  const cplx<T>* U2;
  const double* wk;
  double* lzpart;
  const LzDevState* st;
};

template <typename T, int MODE>
__device__ __forceinline__ void proj_update_mfma_block(cplx<T>* __restrict__ Y,
                                                       const cplx<T>* __restrict__ A, int P,
                                                       int a_rows, const cplx<T>* __restrict__ C,
                                                       int c_rows, int nbnd, int npwx,
                                                       cplx<T>* __restrict__ X,
                                                       const cplx<T>* __restrict__ yv,
                                                       const cplx<T>* __restrict__ U2,
                                                       const double* __restrict__ wk,
                                                       double* __restrict__ lzpart,
                                                       const LzDevState* st, const VBlock& vb) {
  constexpr int NR = MODE == kUpdNhV ? 4 : 3;
  if (st && st->status) return;
  constexpr int BT = kMfmaTile, KC = mfma_kc<T>(), PITCH = BT + 1;
  __shared__ cplx<T> Cs[KC * PITCH], As[KC * PITCH];
  __shared__ double red[NR][256];
  const int g0 = vb.x * BT, b0 = vb.y * BT, k = vb.z;
  const int tid = threadIdx.x, l = tid % 64, wave = tid / 64;
  const int wb = (wave / 2) * 32, wg = (wave % 2) * 32;
  const cplx<T>* Ak = A + (int64_t)k * a_rows * npwx;
  const cplx<T>* Ck = C + (int64_t)k * c_rows * nbnd;
  const cplx<T> zero = mk<T>(T(0), T(0));
  WaveTile<T> acc;
  acc.zero();
  constexpr int NPT = BT * KC / 256;
  T rcr[NPT], rci[NPT], rar[NPT], rai[NPT];  // split parts: kept in registers
  {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int kk = t / BT, j = t - kk * BT;
      const int p = (0) + kk;
      const int b = b0 + j, g = g0 + j;
      const cplx<T> cv = (p < P && b < nbnd) ? Ck[(int64_t)p * nbnd + b] : zero;
      const cplx<T> av = (p < P && g < npwx) ? Ak[(int64_t)p * npwx + g] : zero;
      rcr[i] = cv.x; rci[i] = cv.y; rar[i] = av.x; rai[i] = av.y;
    }
  }
  for (int pc = 0; pc < P; pc += KC) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int kk = t / BT, j = t - kk * BT;
      Cs[kk * PITCH + j] = mk<T>(rcr[i], rci[i]);
      As[kk * PITCH + j] = mk<T>(rar[i], rai[i]);
    }
    __syncthreads();
    if (pc + KC < P) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int kk = t / BT, j = t - kk * BT;
      const int p = (pc + KC) + kk;
      const int b = b0 + j, g = g0 + j;
      const cplx<T> cv = (p < P && b < nbnd) ? Ck[(int64_t)p * nbnd + b] : zero;
      const cplx<T> av = (p < P && g < npwx) ? Ak[(int64_t)p * npwx + g] : zero;
      rcr[i] = cv.x; rci[i] = cv.y; rar[i] = av.x; rai[i] = av.y;
    }
  }
#pragma unroll
    for (int kk = 0; kk < KC; kk += WaveTile<T>::KS) {
      acc.template step<false>(
          l, [&](int row, int kq) { return Cs[(kk + kq) * PITCH + wb + row]; },
          [&](int kq, int col) { return As[(kk + kq) * PITCH + wg + col]; });
    }
    __syncthreads();
  }
  update_epilogue<T, MODE, WaveTile<T>>(acc, Y, nbnd, npwx, X, yv, U2, wk, lzpart, st, b0 + wb,
                                        g0 + wg, k, l, red, vb);
}

template <typename T, int MODE, bool BAT = false>
__global__ __launch_bounds__(256) void k_proj_update_mfma(ProjUpdateMfmaArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (proj_update_mfma_block<T, MODE>(a_.Y, a_.A, a_.P, a_.a_rows, a_.C, a_.c_rows, a_.nbnd,
                                              a_.npwx, a_.X, a_.yv, a_.U2, a_.wk, a_.lzpart, a_.st,
                                              vb)));
}


// ---------------------------------------------------------------------------
// Split-bf16 products (precision LZ_FP32_SPLITBF16): every FP32 operand
// value x is held as x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even; x - hi is exact in FP32), and a real product
// x y as hi_x hi_y + hi_x lo_y + lo_x hi_y, three v_mfma_f32_32x32x16_bf16
// with FP32 accumulation (the dropped lo_x lo_y is 2^-16 relative).  Lane l
// supplies left[l % 32][8 (l / 32) + t] and right[8 (l / 32) + t][l % 32],
// t < 8, and holds the outputs of the f32 32x32 tile above.  Operands sit in
// LDS as four bf16 planes (re hi, re lo, im hi, im lo), k contiguous.
// ---------------------------------------------------------------------------
typedef __bf16 mfma_bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

constexpr int kB3Kc = 32;           // k per LDS round
constexpr int kB3Pitch = kB3Kc + 8; // bf16 per LDS row (16-byte aligned rows)

// four planes [4][64 rows][kB3Pitch] of bf16
struct B3Planes {
  unsigned short* base;
  __device__ __forceinline__ unsigned short* plane(int q) const { return base + q * 64 * kB3Pitch; }
  // store complex value v at (row, k): split both parts
  __device__ __forceinline__ void put(int row, int k, float2 v) const {
    const int o = row * kB3Pitch + k;
    const unsigned short rh = bf16_rne(v.x), ih = bf16_rne(v.y);
    plane(0)[o] = rh;
    plane(1)[o] = bf16_rne(v.x - bf16_value(rh));
    plane(2)[o] = ih;
    plane(3)[o] = bf16_rne(v.y - bf16_value(ih));
  }
  // eight consecutive k of one row of plane q (16 bytes)
  __device__ __forceinline__ uint4 get8(int q, int row, int k) const {
    return *reinterpret_cast<const uint4*>(plane(q) + row * kB3Pitch + k);
  }
};

__device__ __forceinline__ mfma_bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(mfma_bf16x8, v); }
__device__ __forceinline__ uint4 neg8(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

struct WaveTileB3 {
  static constexpr int KS = 16;
  static constexpr int NV = 16;
  mfma_f32x16 re, im;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int v = 0; v < 16; ++v) { re[v] = 0.f; im[v] = 0.f; }
  }
  // acc += x y over 16 k, x and y as (hi, lo) pairs
  __device__ __forceinline__ static mfma_f32x16 prod(mfma_f32x16 acc, uint4 xh, uint4 xl, uint4 yh,
                                                     uint4 yl) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(xh), as_bf16x8(yh), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(xh), as_bf16x8(yl), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(xl), as_bf16x8(yh), acc, 0, 0, 0);
    return acc;
  }
  // one k step of 16 at k0: left rows lr + l % 32 of L, right rows rr + l % 32
  // of R (R stored [col][k]); CONJ: conj(left) * right
  template <bool CONJ>
  __device__ __forceinline__ void step(int l, const B3Planes& L, int lr, const B3Planes& R, int rr,
                                       int k0) {
    const int kq = k0 + 8 * (l / 32);
    const int li = lr + l % 32, rj = rr + l % 32;
    const uint4 arh = L.get8(0, li, kq), arl = L.get8(1, li, kq);
    uint4 aih = L.get8(2, li, kq), ail = L.get8(3, li, kq);
    const uint4 brh = R.get8(0, rj, kq), brl = R.get8(1, rj, kq);
    const uint4 bih = R.get8(2, rj, kq), bil = R.get8(3, rj, kq);
    // conj: re += ar br + ai bi, im += ar bi - ai br
    // else: re += ar br - ai bi, im += ar bi + ai br
    const uint4 pih = CONJ ? aih : neg8(aih), pil = CONJ ? ail : neg8(ail);  // sign into re
    const uint4 qih = CONJ ? neg8(aih) : aih, qil = CONJ ? neg8(ail) : ail;  // sign into im
    re = prod(re, arh, arl, brh, brl);
    re = prod(re, pih, pil, bih, bil);
    im = prod(im, arh, arl, bih, bil);
    im = prod(im, qih, qil, brh, brl);
  }
  __device__ __forceinline__ static int row(int v, int l) { return 8 * (v / 4) + 4 * (l / 32) + (v % 4); }
  __device__ __forceinline__ static int col(int v, int l) { return l % 32; }
  __device__ __forceinline__ float2 at(int v) const { return make_float2(re[v], im[v]); }
};

// dot with split-bf16 products (contract of k_proj_dot_mfma, FP32)
struct ProjDotB3Args {
  const float2* A;
  int P;
  int a_rows;
  const float2* X;
  int nbnd;
  int npwx;
  int chunk;
  int nchunk;
  float2* partial;
  const LzDevState* st;
};

__device__ __forceinline__ void proj_dot_b3_block(const float2* __restrict__ A, int P, int a_rows,
                                                  const float2* __restrict__ X, int nbnd, int npwx,
                                                  int chunk, int nchunk,
                                                  float2* __restrict__ partial,
                                                  const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  constexpr int BT = kMfmaTile, KC = kB3Kc;
  __shared__ __align__(16) unsigned short lds[2 * 4 * 64 * kB3Pitch];
  const B3Planes As{lds}, Xs{lds + 4 * 64 * kB3Pitch};
  const int tilesN = (nbnd + BT - 1) / BT;
  const int p0 = (vb.x / tilesN) * BT, n0 = (vb.x % tilesN) * BT;
  const int ci = vb.y, k = vb.z;
  const int tid = threadIdx.x, l = tid % 64, wave = tid / 64;
  const int wp = (wave / 2) * 32, wn = (wave % 2) * 32;
  const float2* Ak = A + (int64_t)k * a_rows * npwx;
  const float2* Xk = X + (int64_t)k * nbnd * npwx;
  const int g_begin = ci * chunk, g_end = min(npwx, g_begin + chunk);
  const float2 zero = make_float2(0.f, 0.f);
  WaveTileB3 acc;
  acc.zero();
  constexpr int NPT = BT * KC / 256;
  float2 ra[NPT], rx[NPT];
  {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int r = t / KC, c = t - r * KC;
      const int g = (g_begin) + c;
      const int p = p0 + r, n = n0 + r;
      ra[i] = (p < P && g < g_end) ? Ak[(int64_t)p * npwx + g] : zero;
      rx[i] = (n < nbnd && g < g_end) ? Xk[(int64_t)n * npwx + g] : zero;
    }
  }
  for (int g0 = g_begin; g0 < g_end; g0 += KC) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int r = t / KC, c = t - r * KC;
      As.put(r, c, ra[i]);
      Xs.put(r, c, rx[i]);
    }
    __syncthreads();
    if (g0 + KC < g_end) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int r = t / KC, c = t - r * KC;
      const int g = (g0 + KC) + c;
      const int p = p0 + r, n = n0 + r;
      ra[i] = (p < P && g < g_end) ? Ak[(int64_t)p * npwx + g] : zero;
      rx[i] = (n < nbnd && g < g_end) ? Xk[(int64_t)n * npwx + g] : zero;
    }
  }
#pragma unroll
    for (int kk = 0; kk < KC; kk += WaveTileB3::KS) acc.step<true>(l, As, wp, Xs, wn, kk);
    __syncthreads();
  }
  float2* out = partial + ((int64_t)k * nchunk + ci) * P * nbnd;
#pragma unroll
  for (int v = 0; v < WaveTileB3::NV; ++v) {
    const int p = p0 + wp + WaveTileB3::row(v, l), n = n0 + wn + WaveTileB3::col(v, l);
    if (p < P && n < nbnd) out[(int64_t)n * P + p] = acc.at(v);
  }
}

template <bool BAT = false>
__global__ __launch_bounds__(256) void k_proj_dot_b3(ProjDotB3Args p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (proj_dot_b3_block(a_.A, a_.P, a_.a_rows, a_.X, a_.nbnd, a_.npwx, a_.chunk, a_.nchunk,
                                a_.partial, a_.st, vb)));
}

// update with split-bf16 products (contract of k_proj_update_mfma, FP32):
// C^T rows (bands) and A^T rows (plane waves) staged with p contiguous
struct ProjUpdateB3Args {
  float2* Y;
  const float2* A;
  int P;
  int a_rows;
  const float2* C;
  int c_rows;
  int nbnd;
  int npwx;
  float2* X;
  const float2* yv;
  const float2* U2;
  const double* wk;
  double* lzpart;
  const LzDevState* st;
};

template <int MODE>
__device__ __forceinline__ void proj_update_b3_block(float2* __restrict__ Y,
                                                     const float2* __restrict__ A, int P,
                                                     int a_rows, const float2* __restrict__ C,
                                                     int c_rows, int nbnd, int npwx,
                                                     float2* __restrict__ X,
                                                     const float2* __restrict__ yv,
                                                     const float2* __restrict__ U2,
                                                     const double* __restrict__ wk,
                                                     double* __restrict__ lzpart,
                                                     const LzDevState* st, const VBlock& vb) {
  constexpr int NR = MODE == kUpdNhV ? 4 : 3;
  if (st && st->status) return;
  constexpr int BT = kMfmaTile, KC = kB3Kc;
  __shared__ __align__(16) unsigned short lds[2 * 4 * 64 * kB3Pitch];
  __shared__ double red[NR][256];
  const B3Planes Cs{lds}, As{lds + 4 * 64 * kB3Pitch};
  const int g0 = vb.x * BT, b0 = vb.y * BT, k = vb.z;
  const int tid = threadIdx.x, l = tid % 64, wave = tid / 64;
  const int wb = (wave / 2) * 32, wg = (wave % 2) * 32;
  const float2* Ak = A + (int64_t)k * a_rows * npwx;
  const float2* Ck = C + (int64_t)k * c_rows * nbnd;
  const float2 zero = make_float2(0.f, 0.f);
  WaveTileB3 acc;
  acc.zero();
  constexpr int NPT = BT * KC / 256;
  float2 rc[NPT], ra[NPT];
  {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int kk = t / BT, j = t - kk * BT;
      const int p = (0) + kk;
      const int b = b0 + j, g = g0 + j;
      rc[i] = (p < P && b < nbnd) ? Ck[(int64_t)p * nbnd + b] : zero;
      ra[i] = (p < P && g < npwx) ? Ak[(int64_t)p * npwx + g] : zero;
    }
  }
  for (int pc = 0; pc < P; pc += KC) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int kk = t / BT, j = t - kk * BT;
      Cs.put(j, kk, rc[i]);
      As.put(j, kk, ra[i]);
    }
    __syncthreads();
    if (pc + KC < P) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = tid + i * 256;
      const int kk = t / BT, j = t - kk * BT;
      const int p = (pc + KC) + kk;
      const int b = b0 + j, g = g0 + j;
      rc[i] = (p < P && b < nbnd) ? Ck[(int64_t)p * nbnd + b] : zero;
      ra[i] = (p < P && g < npwx) ? Ak[(int64_t)p * npwx + g] : zero;
    }
  }
#pragma unroll
    for (int kk = 0; kk < KC; kk += WaveTileB3::KS) acc.step<false>(l, Cs, wb, As, wg, kk);
    __syncthreads();
  }
  update_epilogue<float, MODE, WaveTileB3>(acc, Y, nbnd, npwx, X, yv, U2, wk, lzpart, st,
                                           b0 + wb, g0 + wg, k, l, red, vb);
}

template <int MODE, bool BAT = false>
__global__ __launch_bounds__(256) void k_proj_update_b3(ProjUpdateB3Args p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (proj_update_b3_block<MODE>(a_.Y, a_.A, a_.P, a_.a_rows, a_.C, a_.c_rows, a_.nbnd,
                                         a_.npwx, a_.X, a_.yv, a_.U2, a_.wk, a_.lzpart, a_.st,
                                         vb)));
}

}  // namespace lz
