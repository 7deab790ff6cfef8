// Plane passes of the Liouvillian application with register-resident line
// transforms, single precision, for cubic grids N^3 with N in {24, 32, 48}
// (a line per thread) and N in {64, 72, 96} (a line per lane pair, at the end
// of this file); in double precision a line of 48 does not fit the register
// file with room to spare: the v'u pass on 48^2 planes takes lane pairs, the
// local and density passes keep the LDS-pass kernels, which were faster.  The 2-D
// transform of a z-plane of one band (Sec. 2.4: the local potential applied
// in real space to every response orbital) runs as
//   rows along i2 (only the rows that hold a stick), one line per thread;
//   columns along i1, one line per thread, where the pointwise work happens
//   between the inverse and the forward transform without leaving registers;
//   rows again, forward.
// A block of 192 threads holds 192/N planes in LDS (row pitch N + 1).  The
// local and v'u passes keep compact planes (the active rows in list order and
// a spare row).  The density pass on 48^2 planes (k_rq_density) does too,
// with the four bands of a block in the lanes of a quad; the general density
// pass (k_rl_density) keeps full planes, in which every access of a column
// thread has a compile-time offset.  Row tasks of all the planes of a block
// are packed onto the first threads, so waves without a row idle instead of
// issuing masked transforms.
#pragma once
#include "lz_fft_reg.h"
#include "lz_kernels.h"

namespace lz {

constexpr int kRegPlaneThreads = 192;

template <int N> struct RegPlane {
  static constexpr int NPB = kRegPlaneThreads / N;  // planes per block
  static constexpr int P = N + 1;                   // LDS row pitch
  static constexpr int R = (N + NPB - 1) / NPB;     // density rows per thread
};

template <typename T, int N>
__host__ __device__ constexpr bool reg_plane_ok() {
  return sizeof(T) == 4 && (N == 24 || N == 32 || N == 48);
}

// Row transforms of the planes of a block: task t < NPB * nact is row a of
// plane pp (row index row(a) in the plane's storage).
template <typename T, int N, int DIR, typename RowOf>
__device__ __forceinline__ void reg_rows(cplx<T>* planes, int pstride, int nact, int tid,
                                         RowOf row) {
  constexpr int NPB = RegPlane<N>::NPB, P = RegPlane<N>::P;
  if (tid < NPB * nact) {
    const int pp = tid / nact, a = tid - pp * nact;
    cplx<T>* r = planes + pp * pstride + row(a) * P;
    cplx<T> x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = r[j];
    reg_fft<T, N, DIR>(x);
#pragma unroll
    for (int j = 0; j < N; ++j) r[j] = x[j];
  }
}

// The sticks of one plane into its LDS rows, and back: a thread's share of
// the stick table and of the values is in flight before the first store
// (batches of kRegStickBatch strided by N cover S <= 12 N in one round).
constexpr int kRegStickBatch = 12;

template <typename T, int N>
__device__ __forceinline__ void reg_scatter(cplx<T>* pl, const cplx<T>* __restrict__ src,
                                            const int* __restrict__ soff, int S, int l) {
  for (int s0 = l; s0 < S; s0 += kRegStickBatch * N) {
    int o[kRegStickBatch];
    cplx<T> v[kRegStickBatch];
#pragma unroll
    for (int j = 0; j < kRegStickBatch; ++j) {
      const int s = s0 + j * N;
      o[j] = s < S ? soff[s] : -1;
      v[j] = s < S ? src[s] : mk<T>(T(0), T(0));
    }
#pragma unroll
    for (int j = 0; j < kRegStickBatch; ++j)
      if (o[j] >= 0) pl[o[j]] = v[j];
  }
}

template <typename T, int N, bool ADD>
__device__ __forceinline__ void reg_gather(cplx<T>* __restrict__ dst, const cplx<T>* pl,
                                           const int* __restrict__ soff, int S, int l) {
  for (int s0 = l; s0 < S; s0 += kRegStickBatch * N) {
    int o[kRegStickBatch];
    cplx<T> v[kRegStickBatch];
#pragma unroll
    for (int j = 0; j < kRegStickBatch; ++j) {
      const int s = s0 + j * N;
      o[j] = s < S ? soff[s] : -1;
      if constexpr (ADD) v[j] = s < S ? dst[s] : mk<T>(T(0), T(0));
    }
#pragma unroll
    for (int j = 0; j < kRegStickBatch; ++j) {
      const int s = s0 + j * N;
      if (o[j] >= 0) {
        const cplx<T> w = pl[o[j]];
        dst[s] = ADD ? cadd<T>(v[j], w) : w;
      }
    }
  }
}

// Column l of a compact plane (rows act[0..nact) in that order, then one
// spare row): in, with zeros for the rows that hold no stick, and out, the
// active rows.  Rows without a stick read and write the spare row, so that
// every access is unconditional (no branch per row).
template <typename T, int N>
__device__ __forceinline__ void reg_col_in(cplx<T> (&x)[N], const cplx<T>* pl,
                                           const RegPlaneArgs& a, int l) {
  constexpr int P = RegPlane<N>::P;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int r = a.slot[i];
    const cplx<T> v = pl[(r >= 0 ? r : a.nact) * P + l];
    x[i] = r >= 0 ? v : mk<T>(T(0), T(0));
  }
}
template <typename T, int N>
__device__ __forceinline__ void reg_col_out(const cplx<T> (&x)[N], cplx<T>* pl,
                                            const RegPlaneArgs& a, int l) {
  constexpr int P = RegPlane<N>::P;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int r = a.slot[i];
    pl[(r >= 0 ? r : a.nact) * P + l] = x[i];
  }
}

// ---------------------------------------------------------------------------
// D step: sticks -> IFFT2 -> V x -> FFT2 -> sticks, for nplanes planes
// (band-major, z fastest).
// ---------------------------------------------------------------------------
template <typename T>
struct RlLocalArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  RegPlaneArgs a;
  int nplanes;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rl_local_block(const cplx<T>* __restrict__ sin,
                                               cplx<T>* __restrict__ sout,
                                               const T* __restrict__ vloc, const RegPlaneArgs& a,
                                               int nplanes, const LzDevState* st,
                                               const VBlock& vb) {
  if (st && st->status) return;
  constexpr int NPB = RegPlane<N>::NPB, P = RegPlane<N>::P;
  const int pstride = (a.nact + 1) * P;  // compact planes: the active rows and a spare
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* planes = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, pp = tid / N, l = tid - pp * N;
  const int pidx = vb.x * NPB + pp;
  const bool live = pidx < nplanes;
  const int z = pidx % N;
  const int64_t so = (int64_t)pidx * a.S;
  cplx<T>* pl = planes + pp * pstride;
  for (int t = l; t < pstride; t += N) pl[t] = mk<T>(T(0), T(0));
  __syncthreads();
  if (live) reg_scatter<T, N>(pl, sin + so, a.soffc, a.S, l);
  __syncthreads();
  reg_rows<T, N, +1>(planes, pstride, a.nact, tid, [](int r) { return r; });
  __syncthreads();
  {
    // the column's potential is loaded before the transform that precedes its use
    const T* vz = vloc + (int64_t)z * N * N + l;
    T vv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) vv[i] = vz[i * N];
    cplx<T> x[N];
    reg_col_in<T, N>(x, pl, a, l);
    reg_fft<T, N, +1>(x);
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = cscale<T>(x[i], vv[i]);
    reg_fft<T, N, -1>(x);
    reg_col_out<T, N>(x, pl, a, l);
  }
  __syncthreads();
  reg_rows<T, N, -1>(planes, pstride, a.nact, tid, [](int r) { return r; });
  __syncthreads();
  if (live) reg_gather<T, N, false>(sout + so, pl, a.soffc, a.S, l);
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(kRegPlaneThreads) void k_rl_local(RlLocalArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (rl_local_block<T, N>(a_.sin, a_.sout, a_.vloc, a_.a, a_.nplanes, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// D+K step: as k_rl_local for the bands of a group at one z, NPB bands at a
// time, also accumulating the response density
//   n'(r) += bandw_b conj(u_b(r)) x_b(r)
// per group into dpart[g][z].  The column threads write their density
// products into their own plane, and after a barrier thread (pp, l) adds rows
// [pp R, pp R + R) of column l over the NPB planes in plane order into
// registers.  Rows without a stick are not cleared between bands; the column
// threads read them as zero.
// ---------------------------------------------------------------------------
template <typename T>
struct RlDensityArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  const cplx<T>* ur;
  const double* bandw;
  cplx<T>* dpart;
  int nb;
  int gsize;
  RegPlaneArgs a;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rl_density_block(const cplx<T>* __restrict__ sin,
                                                 cplx<T>* __restrict__ sout,
                                                 const T* __restrict__ vloc,
                                                 const cplx<T>* __restrict__ ur,
                                                 const double* __restrict__ bandw,
                                                 cplx<T>* __restrict__ dpart, int nb, int gsize,
                                                 const RegPlaneArgs& a, const LzDevState* st,
                                                 const VBlock& vb) {
  if (st && st->status) return;
  constexpr int NPB = RegPlane<N>::NPB, P = RegPlane<N>::P, R = RegPlane<N>::R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* planes = reinterpret_cast<cplx<T>*>(smem_raw);
  constexpr int pstride = N * P;
  const int nact = a.nact;
  const int tid = threadIdx.x, pp = tid / N, l = tid - pp * N;
  const int z = vb.x, g = vb.y;
  const int b0 = g * gsize, b1 = min(nb, b0 + gsize);
  cplx<T>* pl = planes + pp * pstride;
  cplx<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = mk<T>(T(0), T(0));
  const T* vz = vloc + (int64_t)z * N * N + l;
  for (int cb = b0; cb < b1; cb += NPB) {
    const int b = cb + pp;
    const bool live = b < b1;
    // clear the active rows, then scatter this band's sticks
    for (int t = l; t < nact * P; t += N) {
      const int ar = t / P, c = t - ar * P;
      pl[a.act[ar] * P + c] = mk<T>(T(0), T(0));
    }
    __syncthreads();
    const int64_t so = ((int64_t)(live ? b : b0) * N + z) * a.S;
    if (live) reg_scatter<T, N>(pl, sin + so, a.soff, a.S, l);
    __syncthreads();
    reg_rows<T, N, +1>(planes, pstride, nact, tid, [&](int r) { return a.act[r]; });
    __syncthreads();
    cplx<T> x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const cplx<T> v = pl[i * P + l];
      x[i] = a.slot[i] >= 0 ? v : mk<T>(T(0), T(0));
    }
    reg_fft<T, N, +1>(x);
    {
      const cplx<T>* ub = ur + ((int64_t)(live ? b : b0) * N + z) * N * N + l;
      const T wb = live ? T(bandw[b]) : T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const cplx<T> d = cmulc<T>(ub[i * N], x[i]);
        pl[i * P + l] = mk<T>(wb * d.x, wb * d.y);
        x[i] = cscale<T>(x[i], vz[i * N]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = pp * R + r;
      if (i < N) {
        cplx<T> sum = planes[i * P + l];
#pragma unroll
        for (int q = 1; q < NPB; ++q) sum = cadd<T>(sum, planes[q * pstride + i * P + l]);
        acc[r] = cadd<T>(acc[r], sum);
      }
    }
    __syncthreads();
    reg_fft<T, N, -1>(x);
#pragma unroll
    for (int i = 0; i < N; ++i) pl[i * P + l] = x[i];
    __syncthreads();
    reg_rows<T, N, -1>(planes, pstride, nact, tid, [&](int r) { return a.act[r]; });
    __syncthreads();
    if (live) reg_gather<T, N, false>(sout + so, pl, a.soff, a.S, l);
    __syncthreads();
  }
  cplx<T>* dp = dpart + ((int64_t)g * N + z) * N * N + l;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = pp * R + r;
    if (i < N) dp[i * N] = acc[r];
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(kRegPlaneThreads) void k_rl_density(RlDensityArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (rl_density_block<T, N>(a_.sin, a_.sout, a_.vloc, a_.ur, a_.bandw, a_.dpart, a_.nb,
                                     a_.gsize, a_.a, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// D+K step on 48^2 planes for a group of at most four bands, one band per
// lane of a quad: thread 4 l + pp holds column l of band b0 + pp (compact
// planes, as k_rl_local).  The density products of the four bands are added
// across the quad four rows at a time by a reduce-scatter of two lane
// permutations, after which lane pp holds row i0 + pp of the column, and
// writes it into the block's slice of the group partial.  Without the
// products of all N rows staged in LDS for the band sum (full planes, 75 KB)
// and the barriers around it, a block needs the compact planes only, and the
// register count stays within three waves per SIMD: four blocks per compute
// unit against two.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float quad_xor1(float v) {  // the value of lane pp ^ 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_xor2(float v) {  // the value of lane pp ^ 2
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}
template <typename T>
__device__ __forceinline__ cplx<T> quad_xor1(cplx<T> v) { return mk<T>(quad_xor1(v.x), quad_xor1(v.y)); }
template <typename T>
__device__ __forceinline__ cplx<T> quad_xor2(cplx<T> v) { return mk<T>(quad_xor2(v.x), quad_xor2(v.y)); }

// p0..p3: this lane's values of rows 0..3.  Returns row pp summed over the
// quad: the pairs (pp, pp ^ 1) first, then the two pair sums.
template <typename T>
__device__ __forceinline__ cplx<T> quad_reduce_scatter(cplx<T> p0, cplx<T> p1, cplx<T> p2,
                                                       cplx<T> p3, bool odd, bool high) {
  // the even lane keeps rows 0 and 2, the odd lane rows 1 and 3
  const cplx<T> r0 = cadd<T>(odd ? p1 : p0, quad_xor1<T>(odd ? p0 : p1));
  const cplx<T> r1 = cadd<T>(odd ? p3 : p2, quad_xor1<T>(odd ? p2 : p3));
  // the low lanes keep rows 0 / 1, the high lanes rows 2 / 3
  return cadd<T>(high ? r1 : r0, quad_xor2<T>(high ? r0 : r1));
}

template <typename T>
struct RqDensityArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  const cplx<T>* ur;
  const double* bandw;
  cplx<T>* dpart;
  int nb;
  int gsize;
  RegPlaneArgs a;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rq_density_block(const cplx<T>* __restrict__ sin,
                                                 cplx<T>* __restrict__ sout,
                                                 const T* __restrict__ vloc,
                                                 const cplx<T>* __restrict__ ur,
                                                 const double* __restrict__ bandw,
                                                 cplx<T>* __restrict__ dpart, int nb, int gsize,
                                                 const RegPlaneArgs& a, const LzDevState* st,
                                                 const VBlock& vb) {
  static_assert(RegPlane<N>::NPB == 4 && sizeof(T) == 4, "four single-precision bands per block");
  if (st && st->status) return;
  const int pstride = (a.nact + 1) * RegPlane<N>::P;  // compact planes
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* planes = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, pp = tid & 3, l = tid >> 2;
  const bool odd = pp & 1, high = pp & 2;
  const int z = vb.x, g = vb.y;
  const int b0 = g * gsize, b = b0 + pp;
  const bool live = b < min(nb, b0 + gsize);
  cplx<T>* pl = planes + pp * pstride;
  for (int t = l; t < pstride; t += N) pl[t] = mk<T>(T(0), T(0));
  __syncthreads();
  const int64_t so = ((int64_t)(live ? b : b0) * N + z) * a.S;
  if (live) reg_scatter<T, N>(pl, sin + so, a.soffc, a.S, l);
  __syncthreads();
  reg_rows<T, N, +1>(planes, pstride, a.nact, tid, [](int r) { return r; });
  __syncthreads();
  cplx<T> x[N];
  reg_col_in<T, N>(x, pl, a, l);
  reg_fft<T, N, +1>(x);
  {
    const cplx<T>* ub = ur + ((int64_t)(live ? b : b0) * N + z) * N * N + l;
    const T* vz = vloc + (int64_t)z * N * N + l;
    const T wb = live ? T(bandw[b]) : T(0);
    cplx<T>* o = dpart + (((int64_t)g * N + z) * N + pp) * N + l;  // rows i0 + pp
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += 4) {
      cplx<T> p[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = i0 + j;
        const cplx<T> d = cmulc<T>(ub[i * N], x[i]);
        p[j] = mk<T>(wb * d.x, wb * d.y);
        x[i] = cscale<T>(x[i], vz[i * N]);
      }
      o[(int64_t)i0 * N] = quad_reduce_scatter<T>(p[0], p[1], p[2], p[3], odd, high);
    }
  }
  // a thread reads and writes only its own column of its own plane
  reg_fft<T, N, -1>(x);
  reg_col_out<T, N>(x, pl, a, l);
  __syncthreads();
  reg_rows<T, N, -1>(planes, pstride, a.nact, tid, [](int r) { return r; });
  __syncthreads();
  if (live) reg_gather<T, N, false>(sout + so, pl, a.soffc, a.S, l);
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(kRegPlaneThreads) void k_rq_density(RqDensityArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (rq_density_block<T, N>(a_.sin, a_.sout, a_.vloc, a_.ur, a_.bandw, a_.dpart, a_.nb,
                                     a_.gsize, a_.a, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// v'(r) u_b(r) -> FFT2 -> added to the sticks of the same band
// ---------------------------------------------------------------------------
template <typename T>
struct RlVuArgs {
  const cplx<T>* ur;
  const cplx<T>* vp;
  cplx<T>* sout;
  RegPlaneArgs a;
  int nplanes;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rl_vu_block(const cplx<T>* __restrict__ ur,
                                            const cplx<T>* __restrict__ vp,
                                            cplx<T>* __restrict__ sout, const RegPlaneArgs& a,
                                            int nplanes, const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  constexpr int NPB = RegPlane<N>::NPB;
  const int pstride = (a.nact + 1) * RegPlane<N>::P;  // compact planes
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* planes = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, pp = tid / N, l = tid - pp * N;
  const int pidx = vb.x * NPB + pp;
  const bool live = pidx < nplanes;
  const int z = pidx % N;
  cplx<T>* pl = planes + pp * pstride;
  {
    const cplx<T>* ub = ur + (int64_t)(live ? pidx : 0) * N * N + l;
    const cplx<T>* vz = vp + (int64_t)z * N * N + l;
    cplx<T> x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = cmul<T>(ub[i * N], vz[i * N]);
    reg_fft<T, N, -1>(x);
    reg_col_out<T, N>(x, pl, a, l);
  }
  __syncthreads();
  reg_rows<T, N, -1>(planes, pstride, a.nact, tid, [](int r) { return r; });
  __syncthreads();
  if (live) reg_gather<T, N, true>(sout + (int64_t)pidx * a.S, pl, a.soffc, a.S, l);
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(kRegPlaneThreads) void k_rl_vu(RlVuArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br, (rl_vu_block<T, N>(a_.ur, a_.vp, a_.sout, a_.a, a_.nplanes, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// 64^2, 72^2 and 96^2 planes (single precision): one plane per 192-thread block, a
// lane pair per line (pair_fft_dit / pair_fft_dif: N/2 values per lane, a
// radix-2 step across the pair).  Rows: pair r < nact transforms compact row
// r in LDS, natural order in and out.  Columns: pair c < N reads rows 2 j + h
// of column c, transforms them to real-space rows h N/2 + k, applies the
// pointwise work there, and transforms back to rows 2 j + h (on 64^2 and
// 72^2 planes the last threads have no column).  Compact planes as above.
// ---------------------------------------------------------------------------
template <typename T> __host__ __device__ constexpr bool reg_pair_ok() { return sizeof(T) == 4; }

// Double precision on 48^2 planes takes lane pairs too in the v'u pass (24
// values per lane, the register footprint of a single-precision 48-point
// line), one plane per block of 96 threads so that every thread has a column.
template <typename T, int N> __host__ __device__ constexpr bool rp_ok() {
  return sizeof(T) == 4 ? (N == 64 || N == 72 || N == 96) : N == 48;
}
template <typename T, int N> __host__ __device__ constexpr int rp_threads() {
  return sizeof(T) == 8 && N == 48 ? 2 * N : kRegPlaneThreads;
}

template <typename T, int N, int DIR>
__device__ __forceinline__ void pair_rows(cplx<T>* pl, int nact, int tid) {
  constexpr int P = N + 1, M = N / 2;
  if (tid < 2 * nact) {
    const int h = tid & 1;
    cplx<T>* row = pl + (tid >> 1) * P;
    cplx<T> x[M];
#pragma unroll
    for (int j = 0; j < M; ++j) x[j] = row[2 * j + h];
    pair_fft_dit<T, N, DIR>(x, h);
#pragma unroll
    for (int k = 0; k < M; ++k) row[h * M + k] = x[k];
  }
}

// column c of a compact plane, rows 2 j + h in and out (spare row for the
// rows without a stick)
template <typename T, int N>
__device__ __forceinline__ void pair_col_in(cplx<T> (&x)[N / 2], const cplx<T>* pl,
                                            const RegPlaneArgs& a, int c, int h) {
  constexpr int P = N + 1;
#pragma unroll
  for (int j = 0; j < N / 2; ++j) {
    const int r = a.slot[2 * j + h];
    const cplx<T> v = pl[(r >= 0 ? r : a.nact) * P + c];
    x[j] = r >= 0 ? v : mk<T>(T(0), T(0));
  }
}
template <typename T, int N>
__device__ __forceinline__ void pair_col_out(const cplx<T> (&x)[N / 2], cplx<T>* pl,
                                             const RegPlaneArgs& a, int c, int h) {
  constexpr int P = N + 1;
#pragma unroll
  for (int j = 0; j < N / 2; ++j) {
    const int r = a.slot[2 * j + h];
    pl[(r >= 0 ? r : a.nact) * P + c] = x[j];
  }
}

// sticks of one plane into its compact LDS rows, and back, by all NT threads
template <typename T, int NT, bool ADD>
__device__ __forceinline__ void pair_gather(cplx<T>* __restrict__ dst, const cplx<T>* pl,
                                            const int* __restrict__ soff, int S, int tid) {
  reg_gather<T, NT, ADD>(dst, pl, soff, S, tid);
}

// Pointwise work f(k, v) on the N/2 values of a lane (real-space rows
// h N/2 + k), in two rounds of N/4 through a thread-private LDS area
// [N/4][NT]: the loop over a round stays rolled (U at a time), so its global
// loads are not scheduled ahead of the transforms, where they held registers.
template <typename T, int N>
__host__ __device__ constexpr size_t pair_lds(int nact) {
  const size_t plane = (size_t)(nact + 1) * (N + 1);
  const size_t stage = (size_t)(N / 4) * rp_threads<T, N>();
  return (plane > stage ? plane : stage) * sizeof(cplx<T>);
}
template <typename T, int N, int U, typename F>
__device__ __forceinline__ void pair_pointwise(cplx<T> (&x)[N / 2], cplx<T>* stg, int tid, F f) {
  constexpr int RD = N / 4, NT = rp_threads<T, N>();
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int k = 0; k < RD; ++k) stg[k * NT + tid] = x[r * RD + k];
#pragma unroll U
    for (int k = 0; k < RD; ++k) {
      cplx<T>& v = stg[k * NT + tid];
      v = f(r * RD + k, v);
    }
#pragma unroll
    for (int k = 0; k < RD; ++k) x[r * RD + k] = stg[k * NT + tid];
  }
}

template <typename T>
struct RpLocalArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  RegPlaneArgs a;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rp_local_block(const cplx<T>* __restrict__ sin,
                                               cplx<T>* __restrict__ sout,
                                               const T* __restrict__ vloc, const RegPlaneArgs& a,
                                               const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  constexpr int M = N / 2, NT = rp_threads<T, N>();
  const int pstride = (a.nact + 1) * (N + 1);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, c = tid >> 1, h = tid & 1;
  const bool col = 2 * N >= NT || c < N;  // every thread on 96^2 planes and in 96-thread blocks
  const int pidx = vb.x, z = pidx % N;
  const int64_t so = (int64_t)pidx * a.S;
  for (int t = tid; t < pstride; t += NT) pl[t] = mk<T>(T(0), T(0));
  __syncthreads();
  reg_scatter<T, NT>(pl, sin + so, a.soffc, a.S, tid);
  __syncthreads();
  pair_rows<T, N, +1>(pl, a.nact, tid);
  __syncthreads();
  {
    const T* vz = vloc + (int64_t)z * N * N + (int64_t)h * M * N + c;
    cplx<T> x[M];
    if (col) {
      pair_col_in<T, N>(x, pl, a, c, h);
      pair_fft_dit<T, N, +1>(x, h);
    }
    __syncthreads();  // every column read: the plane area becomes staging
    if (col) pair_pointwise<T, N, 8>(x, pl, tid, [&](int k, cplx<T> v) { return cscale<T>(v, vz[k * N]); });
    __syncthreads();
    if (col) {
      pair_fft_dif<T, N, -1>(x, h);
      pair_col_out<T, N>(x, pl, a, c, h);
    }
  }
  __syncthreads();
  pair_rows<T, N, -1>(pl, a.nact, tid);
  __syncthreads();
  pair_gather<T, NT, false>(sout + so, pl, a.soffc, a.S, tid);
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__((rp_threads<T, N>())) void k_rp_local(RpLocalArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br, (rp_local_block<T, N>(a_.sin, a_.sout, a_.vloc, a_.a, a_.st, vb)));
}

// A value streamed from memory once (non-temporal: kept out of the caches,
// which then hold the partial-density slices the density pass re-reads).
template <typename T>
__device__ __forceinline__ cplx<T> ld_stream(const cplx<T>* p) {
  const T* q = reinterpret_cast<const T*>(p);
  return mk<T>(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1));
}

// D+K step on 72^2 / 96^2 planes: the bands of a group one after the other at
// one z; the density products go straight into the block's slice of the
// group partial dpart[g][z] (each thread its own elements, in band order).
// Held to 168 registers (three waves per SIMD, four blocks per compute unit;
// a spill of 3 values at 96, of 15 at 72): the pass waits on memory, and
// 5.3 ms became 3.85 ms on the 96^3 cell against two blocks per unit at 172
// registers (the batched workload, with its 72^3 members, gained 7 % against
// the unbounded 181 registers at 72).
template <typename T>
struct RpDensityArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  const cplx<T>* ur;
  const double* bandw;
  cplx<T>* dpart;
  int nb;
  int gsize;
  RegPlaneArgs a;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rp_density_block(const cplx<T>* __restrict__ sin,
                                                 cplx<T>* __restrict__ sout,
                                                 const T* __restrict__ vloc,
                                                 const cplx<T>* __restrict__ ur,
                                                 const double* __restrict__ bandw,
                                                 cplx<T>* __restrict__ dpart, int nb, int gsize,
                                                 const RegPlaneArgs& a, const LzDevState* st,
                                                 const VBlock& vb) {
  if (st && st->status) return;
  constexpr int M = N / 2, NT = rp_threads<T, N>();
  const int pstride = (a.nact + 1) * (N + 1);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, c = tid >> 1, h = tid & 1;
  const bool col = 2 * N >= NT || c < N;  // every thread on 96^2 planes and in 96-thread blocks
  const int z = vb.x, g = vb.y;
  const int b0 = g * gsize, b1 = min(nb, b0 + gsize);
  const int64_t roff = (int64_t)h * M * N + (col ? c : 0);  // element (row h M, column c)
  const T* vz = vloc + (int64_t)z * N * N + roff;
  cplx<T>* dp = dpart + ((int64_t)g * N + z) * N * N + roff;
  for (int b = b0; b < b1; ++b) {
    for (int t = tid; t < pstride; t += NT) pl[t] = mk<T>(T(0), T(0));
    __syncthreads();
    const int64_t so = ((int64_t)b * N + z) * a.S;
    reg_scatter<T, NT>(pl, sin + so, a.soffc, a.S, tid);
    __syncthreads();
    pair_rows<T, N, +1>(pl, a.nact, tid);
    __syncthreads();
    // the column made opaque in each band: the row addresses of the column
    // are then formed where they are used instead of being held, loop
    // invariant, through the whole band loop
    int cb = c;
    asm volatile("" : "+v"(cb));
    cplx<T> x[M];
    if (col) {
      pair_col_in<T, N>(x, pl, a, cb, h);
      pair_fft_dit<T, N, +1>(x, h);
    }
    __syncthreads();  // every column read: the plane area becomes staging
    if (col) {
      const cplx<T>* ub = ur + ((int64_t)b * N + z) * N * N + roff;
      const T wb = T(bandw[b]);
      const bool first = b == b0;
      pair_pointwise<T, N, 12>(x, pl, tid, [&](int k, cplx<T> v) {
        const cplx<T> d = cmulc<T>(ld_stream<T>(ub + k * N), v);
        cplx<T> sacc = first ? mk<T>(T(0), T(0)) : dp[k * N];
        sacc.x += wb * d.x;
        sacc.y += wb * d.y;
        dp[k * N] = sacc;
        return cscale<T>(v, vz[k * N]);
      });
    }
    __syncthreads();
    if (col) {
      pair_fft_dif<T, N, -1>(x, h);
      pair_col_out<T, N>(x, pl, a, cb, h);
    }
    __syncthreads();
    pair_rows<T, N, -1>(pl, a.nact, tid);
    __syncthreads();
    pair_gather<T, NT, false>(sout + so, pl, a.soffc, a.S, tid);
    __syncthreads();
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__((rp_threads<T, N>())) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 3))) void k_rp_density(
    RpDensityArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (rp_density_block<T, N>(a_.sin, a_.sout, a_.vloc, a_.ur, a_.bandw, a_.dpart, a_.nb,
                                     a_.gsize, a_.a, a_.st, vb)));
}

// v'(r) u_b(r) -> FFT2 -> added to the sticks of the same band, 72^2 / 96^2
template <typename T>
struct RpVuArgs {
  const cplx<T>* ur;
  const cplx<T>* vp;
  cplx<T>* sout;
  RegPlaneArgs a;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void rp_vu_block(const cplx<T>* __restrict__ ur,
                                            const cplx<T>* __restrict__ vp,
                                            cplx<T>* __restrict__ sout, const RegPlaneArgs& a,
                                            const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  constexpr int M = N / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, c = tid >> 1, h = tid & 1;
  const int pidx = vb.x, z = pidx % N;
  if (c < N) {
    const int64_t roff = (int64_t)h * M * N + c;
    const cplx<T>* ub = ur + (int64_t)pidx * N * N + roff;
    const cplx<T>* vz = vp + (int64_t)z * N * N + roff;
    cplx<T> x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = cmul<T>(ub[k * N], vz[k * N]);
    pair_fft_dif<T, N, -1>(x, h);
    pair_col_out<T, N>(x, pl, a, c, h);
  }
  __syncthreads();
  pair_rows<T, N, -1>(pl, a.nact, tid);
  __syncthreads();
  pair_gather<T, rp_threads<T, N>(), true>(sout + (int64_t)pidx * a.S, pl, a.soffc, a.S, tid);
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__((rp_threads<T, N>())) void k_rp_vu(RpVuArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br, (rp_vu_block<T, N>(a_.ur, a_.vp, a_.sout, a_.a, a_.st, vb)));
}

}  // namespace lz
