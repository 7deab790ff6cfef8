// Linear-algebra kernels of the Liouvillian application and of the
// pseudo-Hermitian Lanczos recursion (Secs. 2.3-2.5 of the turboEELS paper):
// projector products (P_c and separable projectors), Lanczos vector updates
// and deterministic reductions, the spectrum solve, and layout permutations.
#include <algorithm>
#include <stdexcept>
#include <string>

#include "lz_kernels.h"

namespace lz {

thread_local std::vector<LaunchRec>* t_launch_rec = nullptr;

void launch_args(const void* fn, const void* fnb, dim3 grid, dim3 block, size_t lds,
                 hipStream_t s, const void* p, size_t bytes) {
  if (t_launch_rec) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    t_launch_rec->push_back(
        LaunchRec{fn, fnb, grid, block, lds, std::vector<unsigned char>(b, b + bytes)});
    return;
  }
  BatchRef br{nullptr, nullptr, 0, 0};
  void* args[2] = {const_cast<void*>(p), &br};
  const hipError_t e = hipLaunchKernel(fn, grid, block, args, lds, s);
  if (e != hipSuccess) throw std::runtime_error(std::string("kernel launch: ") + hipGetErrorString(e));
}

// complex values per thread of a 256-thread plane pass (general form)
int plane_mp(int n1, int n2) {
  const int np = n1 * n2;
  if (np <= 12 * 256) return 12;
  if (np <= 24 * 256) return 24;
  return 36;
}

template <typename T>
__device__ __forceinline__ cplx<T> czero() { return mk<T>(T(0), T(0)); }

// ---------------------------------------------------------------------------
// Projector products.  Per k the rows of A are the valence orbitals U_{k+q}
// (nbnd rows, P_c = 1 - U U^H) followed by the separable projectors beta
// (nproj rows, V_NL = beta D beta^H), all on the k+q sphere.
//
//   dot     R[k][p][n]  = sum_G conj(A[k][p][G]) X[k][n][G]   (split over G
//                         into chunk partials)
//   coef    the partials of one column n of R summed in a fixed order, and
//           the small per-k matrices turning it into update coefficients
//   update  Y[k][n][G] += sum_p A[k][p][G] C[k][p][n]
//
// With S = U^H w, B' = beta^H w and M = beta^H U (fixed), the projector of
// the separable term acting on P_c w is beta^H P_c w = B' - M S, and the
// valence overlap of beta D B is U^H beta D B = M^H (D B); one pass over w
// and one over the output then give P_c w, V_NL P_c w and P_c of the output.
// ---------------------------------------------------------------------------
constexpr int kDotK = 32;  // G per LDS tile

// Block: 256 threads as 16 x 16; thread (ty, tx) owns outputs
// (p0 + ty + 16 i, n0 + tx + 16 j), i < TPI, j < TNJ; one block covers
// `chunk` plane waves of one k.  UPD: the block first forms the Lanczos
// vector w = a*LW + b*X of its plane waves and writes it back to X (the
// host uses UPD only when one block spans every row and band of a chunk).
template <typename T>
struct ProjDotArgs {
  const cplx<T>* A;
  int P;
  int a_rows;
  cplx<T>* X;
  const cplx<T>* LW;
  int nbnd;
  int npwx;
  int chunk;
  int nchunk;
  cplx<T>* partial;
  const LzDevState* st;
};

template <typename T, int TPI, int TNJ, bool UPD>
__device__ __forceinline__ void proj_dot_block(const cplx<T>* __restrict__ A, int P, int a_rows,
                                               cplx<T>* X, const cplx<T>* __restrict__ LW, int nbnd,
                                               int npwx, int chunk, int nchunk,
                                               cplx<T>* __restrict__ partial, const LzDevState* st,
                                               const VBlock& vb) {
  if (st && st->status) return;
  constexpr int TP = 16 * TPI, TN = 16 * TNJ;
  __shared__ cplx<T> As[TP][kDotK + 1];
  __shared__ cplx<T> Xs[TN][kDotK + 1];
  const int ntn = (nbnd + TN - 1) / TN;
  const int p0 = (vb.x / ntn) * TP;
  const int n0 = (vb.x % ntn) * TN;
  const int ci = vb.y, k = vb.z;
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  T ua = T(0), ub = T(0);
  if constexpr (UPD) {
    ua = T(st->a);
    ub = T(st->b);
  }
  cplx<T> acc[TPI][TNJ];
#pragma unroll
  for (int i = 0; i < TPI; ++i)
#pragma unroll
    for (int j = 0; j < TNJ; ++j) acc[i][j] = czero<T>();
  const cplx<T>* Ak = A + (int64_t)k * a_rows * npwx;
  cplx<T>* Xk = X + (int64_t)k * nbnd * npwx;
  const cplx<T>* Lk = UPD ? LW + (int64_t)k * nbnd * npwx : nullptr;
  const int g_end = min(npwx, (ci + 1) * chunk);
  // software pipeline: the next tile's values are loaded into registers while
  // the current one is multiplied out of LDS (with UPD the Lanczos vector is
  // formed, and written back, when its tile goes to LDS)
  constexpr int NA = (TP * kDotK + 255) / 256, NX = (TN * kDotK + 255) / 256;
  cplx<T> ra[NA], rx[NX], rl[UPD ? NX : 1];
  auto load = [&](int g0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int t = threadIdx.x + i * 256;
      const int r = t / kDotK, c = t - r * kDotK;
      const int g = g0 + c, p = p0 + r;
      ra[i] = (t < TP * kDotK && p < P && g < g_end) ? Ak[(int64_t)p * npwx + g] : czero<T>();
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int t = threadIdx.x + i * 256;
      const int r = t / kDotK, c = t - r * kDotK;
      const int g = g0 + c, n = n0 + r;
      const bool in = t < TN * kDotK && n < nbnd && g < g_end;
      const int64_t o = (int64_t)n * npwx + g;
      rx[i] = in ? Xk[o] : czero<T>();
      if constexpr (UPD) rl[i] = in ? Lk[o] : czero<T>();
    }
  };
  const int g_beg = ci * chunk;
  if (g_beg < g_end) load(g_beg);
  for (int g0 = g_beg; g0 < g_end; g0 += kDotK) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int t = threadIdx.x + i * 256;
      if (t < TP * kDotK) As[t / kDotK][t % kDotK] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int t = threadIdx.x + i * 256;
      if (t < TN * kDotK) {
        const int r = t / kDotK, c = t - r * kDotK;
        cplx<T> v = rx[i];
        if constexpr (UPD) {
          const int g = g0 + c, n = n0 + r;
          v = mk<T>(ua * rl[i].x + ub * v.x, ua * rl[i].y + ub * v.y);
          if (n < nbnd && g < g_end) Xk[(int64_t)n * npwx + g] = v;
        }
        Xs[r][c] = v;
      }
    }
    __syncthreads();
    if (g0 + kDotK < g_end) load(g0 + kDotK);
#pragma unroll 4
    for (int c = 0; c < kDotK; ++c) {
      cplx<T> a[TPI], x[TNJ];
#pragma unroll
      for (int i = 0; i < TPI; ++i) a[i] = As[ty + 16 * i][c];
#pragma unroll
      for (int j = 0; j < TNJ; ++j) x[j] = Xs[tx + 16 * j][c];
#pragma unroll
      for (int i = 0; i < TPI; ++i)
#pragma unroll
        for (int j = 0; j < TNJ; ++j) acc[i][j] = cadd<T>(acc[i][j], cmulc<T>(a[i], x[j]));
    }
    __syncthreads();
  }
  cplx<T>* out = partial + ((int64_t)k * nchunk + ci) * P * nbnd;
#pragma unroll
  for (int i = 0; i < TPI; ++i)
#pragma unroll
    for (int j = 0; j < TNJ; ++j) {
      const int p = p0 + ty + 16 * i, n = n0 + tx + 16 * j;
      if (p < P && n < nbnd) out[n * P + p] = acc[i][j];
    }
}

template <typename T, int TPI, int TNJ, bool UPD, bool BAT = false>
__global__ __launch_bounds__(256, TPI * TNJ <= 3 ? 4 : 1) void k_proj_dot(ProjDotArgs<T> p,
                                                                          BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (proj_dot_block<T, TPI, TNJ, UPD>(a_.A, a_.P, a_.a_rows, a_.X, a_.LW, a_.nbnd, a_.npwx,
                                               a_.chunk, a_.nchunk, a_.partial, a_.st, vb)));
}

// Column n of R[k] (P rows) from the chunk partials [k][chunk][n][p], summed in
// double in a fixed order: lane l of a row sums chunks l, l+16, ..., then the
// 16 lane sums are added in lane order.  A round covers kRedRows rows (16
// lanes each, kRedRows / 16 rows per thread) and kRedBatch chunks per lane,
// all of their loads in flight; the result, rounded to T, is left in Rc[0..P).
constexpr int kRedRows = 64, kRedBatch = 8;

template <typename T>
__device__ __forceinline__ void reduce_column(const cplx<T>* __restrict__ partial, int nchunk,
                                              int P, int nbnd, int n, int k, cplx<T>* Rc) {
  constexpr int RB = kRedRows / 16;
  __shared__ double rx[kRedRows][17], ry[kRedRows][17];
  const int o = threadIdx.x % 16, lane = threadIdx.x / 16;
  const int64_t cs = (int64_t)P * nbnd;
  const cplx<T>* pk = partial + (int64_t)k * nchunk * cs + (int64_t)n * P;
  for (int p0 = 0; p0 < P; p0 += kRedRows) {
    double sx[RB], sy[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) sx[r] = sy[r] = 0.0;
    // kRedBatch chunks per round, all loads of a round in flight at once
    for (int c0 = lane; c0 < nchunk; c0 += 16 * kRedBatch) {
      cplx<T> v[kRedBatch][RB];
#pragma unroll
      for (int i = 0; i < kRedBatch; ++i) {
        const int c = c0 + 16 * i;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int p = p0 + o + 16 * r;
          v[i][r] = (c < nchunk && p < P) ? pk[(int64_t)c * cs + p] : czero<T>();
        }
      }
#pragma unroll
      for (int i = 0; i < kRedBatch; ++i) {
        if (c0 + 16 * i < nchunk) {
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            sx[r] += double(v[i][r].x);
            sy[r] += double(v[i][r].y);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      rx[o + 16 * r][lane] = sx[r];
      ry[o + 16 * r][lane] = sy[r];
    }
    __syncthreads();
    const int p = p0 + threadIdx.x;
    if (threadIdx.x < kRedRows && p < P) {
      double ax = 0.0, ay = 0.0;
      for (int l = 0; l < 16; ++l) {
        ax += rx[threadIdx.x][l];
        ay += ry[threadIdx.x][l];
      }
      Rc[p] = mk<T>(T(ax), T(ay));
    }
    __syncthreads();
  }
}

// Block (n, k): R[k][p][n] = column n of the reduced partials (set-up).
template <typename T>
__global__ __launch_bounds__(256) void k_reduce_plain(const cplx<T>* __restrict__ partial,
                                                      int nchunk, int P, int nbnd,
                                                      cplx<T>* __restrict__ R) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* Rc = reinterpret_cast<cplx<T>*>(smem_raw);  // [P]
  const int n = blockIdx.x, k = blockIdx.y;
  reduce_column<T>(partial, nchunk, P, nbnd, n, k, Rc);
  for (int p = threadIdx.x; p < P; p += 256) R[((int64_t)k * P + p) * nbnd + n] = Rc[p];
}

// Input side, block (n, k): R[:, n] = [S; B'][:, n] reduced, then
//   C_in[:, n] = [-S; D (B' - M S)][:, n];
// with skip_pc (the start vector, or an operator application on a vector the
// caller did not project) S is not applied: C_in = [0; D B'].
template <typename T>
struct ReduceCoefInArgs {
  const cplx<T>* partial;
  int nchunk;
  const cplx<T>* M;
  const double* dkb;
  int nbnd;
  int nproj;
  int skip_pc;
  cplx<T>* C;
  const LzDevState* st;
};

template <typename T>
__device__ __forceinline__ void reduce_coef_in_block(const cplx<T>* __restrict__ partial,
                                                     int nchunk, const cplx<T>* __restrict__ M,
                                                     const double* __restrict__ dkb, int nbnd,
                                                     int nproj, int skip_pc,
                                                     cplx<T>* __restrict__ C, const LzDevState* st,
                                                     const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* Rc = reinterpret_cast<cplx<T>*>(smem_raw);  // [P]
  const int n = vb.x, k = vb.y;
  const int P = nbnd + nproj;
  reduce_column<T>(partial, nchunk, P, nbnd, n, k, Rc);
  cplx<T>* Ck = C + (int64_t)k * P * nbnd;
  for (int p = threadIdx.x; p < P; p += 256) {
    cplx<T> out;
    if (p < nbnd) {
      out = skip_pc ? czero<T>() : mk<T>(-Rc[p].x, -Rc[p].y);
    } else {
      const int q = p - nbnd;
      double ax = double(Rc[p].x), ay = double(Rc[p].y);
      if (!skip_pc) {
        const cplx<T>* Mq = M + ((int64_t)k * nproj + q) * nbnd;
#pragma unroll 16
        for (int m = 0; m < nbnd; ++m) {
          const cplx<T> mm = Mq[m], sv = Rc[m];
          ax -= double(mm.x) * double(sv.x) - double(mm.y) * double(sv.y);
          ay -= double(mm.x) * double(sv.y) + double(mm.y) * double(sv.x);
        }
      }
      const double d = dkb[q];
      out = mk<T>(T(d * ax), T(d * ay));
    }
    Ck[p * nbnd + n] = out;
  }
}

template <typename T, bool BAT = false>
__global__ __launch_bounds__(256) void k_reduce_coef_in(ReduceCoefInArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (reduce_coef_in_block<T>(a_.partial, a_.nchunk, a_.M, a_.dkb, a_.nbnd, a_.nproj,
                                      a_.skip_pc, a_.C, a_.st, vb)));
}

// Output side, block (n, k): Rout[:, n] = (U^H Y)[:, n] reduced, DB = rows
// nbnd.. of C_in:  C_out[:, n] = [-(Rout + M^H DB); DB][:, n].
template <typename T>
struct ReduceCoefOutArgs {
  const cplx<T>* partial;
  int nchunk;
  const cplx<T>* Cin;
  const cplx<T>* M;
  int nbnd;
  int nproj;
  cplx<T>* C;
  const LzDevState* st;
};

template <typename T>
__device__ __forceinline__ void reduce_coef_out_block(const cplx<T>* __restrict__ partial,
                                                      int nchunk, const cplx<T>* __restrict__ Cin,
                                                      const cplx<T>* __restrict__ M, int nbnd,
                                                      int nproj, cplx<T>* __restrict__ C,
                                                      const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* Rc = reinterpret_cast<cplx<T>*>(smem_raw);  // [nbnd]
  const int n = vb.x, k = vb.y;
  const int P = nbnd + nproj;
  reduce_column<T>(partial, nchunk, nbnd, nbnd, n, k, Rc);
  const cplx<T>* Ck = Cin + (int64_t)k * P * nbnd;
  cplx<T>* Co = C + (int64_t)k * P * nbnd;
  for (int p = threadIdx.x; p < P; p += 256) {
    cplx<T> out;
    if (p < nbnd) {
      double ax = double(Rc[p].x), ay = double(Rc[p].y);
#pragma unroll 16
      for (int q = 0; q < nproj; ++q) {
        const cplx<T> mm = M[((int64_t)k * nproj + q) * nbnd + p];  // conj taken below
        const cplx<T> db = Ck[(nbnd + q) * nbnd + n];
        ax += double(mm.x) * double(db.x) + double(mm.y) * double(db.y);
        ay += double(mm.x) * double(db.y) - double(mm.y) * double(db.x);
      }
      out = mk<T>(T(-ax), T(-ay));
    } else {
      out = Ck[p * nbnd + n];
    }
    Co[p * nbnd + n] = out;
  }
}

template <typename T, bool BAT = false>
__global__ __launch_bounds__(256) void k_reduce_coef_out(ReduceCoefOutArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (reduce_coef_out_block<T>(a_.partial, a_.nchunk, a_.Cin, a_.M, a_.nbnd, a_.nproj, a_.C,
                                       a_.st, vb)));
}

// Y[k][n][G] += sum_{p<P} A[k][p][G] C[k][p][n], and what the recursion does
// with the updated element Y' (MODE):
//   kUpdPlain  Y <- Y'
//   kUpdDots   Y <- Y', and the pseudo-Hermitian sums of the block
//              s0 = sum w_k Re(conj(X) Y'),  s1 + i s2 = sum w_k conj(y) X
//   kUpdNhU    X <- cu1 Y' + cu2 X   (u^ of the non-Hermitian recursion formed
//              in place of the vector two steps back; Y is left as it was)
//   kUpdNhV    X <- v^ = cv1 Y' + cv2 X, and the non-Hermitian sums
//              s + i t = sum w_k conj(U2) v^,  zr + i zi = sum w_k conj(y) v^
//              (U2 = u^ of the same step, formed by a kUpdNhU launch before)
// The sums go to lzpart[block] (fixed order inside the block; 3 per block, 4
// for kUpdNhV).  A block covers 256/qn plane waves and qn x NBT bands (qn = 4
// when the coefficients fit in LDS): its qn groups of threads read the same
// rows of A (cache hits after the first), so A is fetched once per qn NBT
// bands.
constexpr int kUpdPlain = 0, kUpdDots = 1, kUpdNhU = 2, kUpdNhV = 3;

template <typename T>
struct ProjUpdateArgs {
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
  int qn;
  const LzDevState* st;
};

template <typename T, int NBT, int MODE>
__device__ __forceinline__ void proj_update_block(cplx<T>* __restrict__ Y,
                                                  const cplx<T>* __restrict__ A, int P, int a_rows,
                                                  const cplx<T>* __restrict__ C, int c_rows,
                                                  int nbnd, int npwx, cplx<T>* __restrict__ X,
                                                  const cplx<T>* __restrict__ yv,
                                                  const cplx<T>* __restrict__ U2,
                                                  const double* __restrict__ wk,
                                                  double* __restrict__ lzpart, int qn,
                                                  const LzDevState* st, const VBlock& vb) {
  constexpr bool DOTS = MODE == kUpdDots || MODE == kUpdNhV;
  constexpr int NR = MODE == kUpdNhV ? 4 : 3;
  if (st && st->status) return;
  const int NB = qn * NBT;
  const int npt = 256 / qn;  // plane waves per block
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* Cs = reinterpret_cast<cplx<T>*>(smem_raw);  // [P][NB]
  __shared__ double red[NR][256];
  const int k = vb.z;
  const int nb0 = vb.y * NB;
  const int nbb = min(NB, nbnd - nb0);
  const cplx<T>* Ck = C + (int64_t)k * c_rows * nbnd;
  for (int t = threadIdx.x; t < P * NB; t += 256) {
    const int p = t / NB, j = t - p * NB;
    Cs[t] = j < nbb ? Ck[p * nbnd + nb0 + j] : czero<T>();
  }
  __syncthreads();
  const int q = threadIdx.x / npt;
  const int g = vb.x * npt + (threadIdx.x % npt);
  const int n0 = nb0 + q * NBT;
  const int nbt = min(NBT, nbnd - n0);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (g < npwx && nbt > 0) {
    const cplx<T>* Ak = A + (int64_t)k * a_rows * npwx;
    const cplx<T>* Cq = Cs + q * NBT;
    cplx<T> acc[NBT];
#pragma unroll
    for (int j = 0; j < NBT; ++j) acc[j] = czero<T>();
    if constexpr (sizeof(T) == 8) {
      // rows of A in batches of 16 whose loads are issued before they are
      // used (faster in double precision; single precision measured faster
      // with the plain loop below)
      constexpr int kB = 16;
      for (int p0 = 0; p0 < P; p0 += kB) {
        cplx<T> a[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i)
          a[i] = p0 + i < P ? Ak[(int64_t)(p0 + i) * npwx + g] : czero<T>();
#pragma unroll
        for (int i = 0; i < kB; ++i) {
          if (p0 + i < P) {
#pragma unroll
            for (int j = 0; j < NBT; ++j)
              acc[j] = cadd<T>(acc[j], cmul<T>(a[i], Cq[(p0 + i) * NB + j]));
          }
        }
      }
    } else {
#pragma unroll 4
      for (int p = 0; p < P; ++p) {
        const cplx<T> a = Ak[(int64_t)p * npwx + g];
#pragma unroll
        for (int j = 0; j < NBT; ++j) acc[j] = cadd<T>(acc[j], cmul<T>(a, Cq[p * NB + j]));
      }
    }
    const int64_t kb = (int64_t)k * nbnd * npwx;
    const double w = DOTS ? wk[k] : 0.0;
    cplx<T> c1 = czero<T>(), c2 = czero<T>();
    if constexpr (MODE == kUpdNhU) {
      c1 = mk<T>(T(st->cu1[0]), T(st->cu1[1]));
      c2 = mk<T>(T(st->cu2[0]), T(st->cu2[1]));
    } else if constexpr (MODE == kUpdNhV) {
      c1 = mk<T>(T(st->cv1[0]), T(st->cv1[1]));
      c2 = mk<T>(T(st->cv2[0]), T(st->cv2[1]));
    }
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (j < nbt) {
        const int64_t o = kb + (int64_t)(n0 + j) * npwx + g;
        cplx<T> yv_new = cadd<T>(Y[o], acc[j]);
        if constexpr (MODE == kUpdPlain || MODE == kUpdDots) Y[o] = yv_new;
        if constexpr (MODE == kUpdDots) {
          const cplx<T> xv = X[o], rv = yv[o];
          s0 += w * (double(xv.x) * double(yv_new.x) + double(xv.y) * double(yv_new.y));
          s1 += w * (double(rv.x) * double(xv.x) + double(rv.y) * double(xv.y));
          s2 += w * (double(rv.x) * double(xv.y) - double(rv.y) * double(xv.x));
        }
        if constexpr (MODE == kUpdNhU || MODE == kUpdNhV) {
          const cplx<T> h = cadd<T>(cmul<T>(c1, yv_new), cmul<T>(c2, X[o]));
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
  }
  if constexpr (DOTS) {
    const double sv[4] = {s0, s1, s2, s3};
#pragma unroll
    for (int r = 0; r < NR; ++r) red[r][threadIdx.x] = sv[r];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) {
#pragma unroll
        for (int r = 0; r < NR; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + h];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int blk = (vb.z * vb.ny + vb.y) * vb.nx + vb.x;
#pragma unroll
      for (int r = 0; r < NR; ++r) lzpart[NR * blk + r] = red[r][0];
    }
  }
}

template <typename T, int NBT, int MODE, bool BAT = false>
__global__ __launch_bounds__(256) void k_proj_update(ProjUpdateArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (proj_update_block<T, NBT, MODE>(a_.Y, a_.A, a_.P, a_.a_rows, a_.C, a_.c_rows, a_.nbnd,
                                              a_.npwx, a_.X, a_.yv, a_.U2, a_.wk, a_.lzpart, a_.qn,
                                              a_.st, vb)));
}

}  // namespace lz
#include "lz_gemm_mfma.h"
#include "lz_small.h"
namespace lz {

// ---------------------------------------------------------------------------
// Lanczos vectors and scalars
// ---------------------------------------------------------------------------
template <typename T>
struct LzUpdateArgs {
  cplx<T>* w;
  const cplx<T>* lw;
  int64_t n;
  const LzDevState* st;
};

template <typename T>
__device__ __forceinline__ void lz_update_block(cplx<T>* __restrict__ w,
                                                const cplx<T>* __restrict__ lw, int64_t n,
                                                const LzDevState* st, const VBlock& vb) {
  if (st->status) return;
  const T a = T(st->a), b = T(st->b);
  for (int64_t i = vb.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)vb.nx * blockDim.x) {
    const cplx<T> l = lw[i], v = w[i];
    w[i] = mk<T>(a * l.x + b * v.x, a * l.y + b * v.y);
  }
}

template <typename T, bool BAT = false>
__global__ __launch_bounds__(256) void k_lz_update(LzUpdateArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br, (lz_update_block<T>(a_.w, a_.lw, a_.n, a_.st, vb)));
}

constexpr int kDotThreads = 256;

// Sum the partials and take the scalar decisions of one Lanczos step:
//   j = st->step; b2 = Re<w_j, L w_j>_w; beta_{j+1} = sqrt(b2);
//   z_{j+1} = <y, w_j>_w / beta_{j+1} for odd j (upper vector), else 0.
// Step 0 (w_0 = y) first checks for a vanished right-hand side.
struct LzFinalizeArgs {
  const double* partial;
  int nblk;
  LzDevState* st;
  double* beta;
  double* z;
  int max_steps;
  double tol;
  double yscale;
};

__device__ __forceinline__ void lz_finalize_block(const double* __restrict__ partial, int nblk,
                                                  LzDevState* __restrict__ st,
                                                  double* __restrict__ beta, double* __restrict__ z,
                                                  int max_steps, double tol, double yscale,
                                                  const VBlock& vb) {
  __shared__ double red[3][kDotThreads];
  if (st->status) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kDotThreads) {
    s0 += partial[i * 3 + 0];
    s1 += partial[i * 3 + 1];
    s2 += partial[i * 3 + 2];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int h = kDotThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
      red[2][threadIdx.x] += red[2][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double b2 = red[0][0], zr = red[1][0], zi = red[2][0];
  const int j = st->step;
  if (j >= max_steps) { st->status = 5; return; }
  if (!isfinite(b2) || !isfinite(zr) || !isfinite(zi)) { st->status = 7; return; }
  if (j == 0) {
    if (zr <= tol * tol * yscale) { st->status = 6; return; }  // y = 0: chi vanishes
    if (b2 <= 0.0) { st->status = 4; return; }
    const double bt = sqrt(b2);
    beta[0] = bt;
    z[0] = 0.0;
    z[1] = 0.0;
    st->a = 1.0 / bt;
    st->b = 0.0;
    st->beta_prev = bt;
    st->step = 1;
    return;
  }
  const double bm = st->bmax;
  if (b2 < -(tol * bm) * (tol * bm) || (b2 <= 0.0 && bm == 0.0)) { st->status = 4; return; }
  if (b2 <= (tol * bm) * (tol * bm)) { st->status = 6; return; }
  const double bt = sqrt(b2);
  beta[j] = bt;
  if (j & 1) {
    z[2 * j] = zr / bt;
    z[2 * j + 1] = zi / bt;
  } else {
    z[2 * j] = 0.0;
    z[2 * j + 1] = 0.0;
  }
  st->bmax = bm > bt ? bm : bt;
  st->a = 1.0 / bt;
  st->b = -bt / st->beta_prev;
  st->beta_prev = bt;
  st->step = j + 1;
}

template <bool BAT = false>
__global__ __launch_bounds__(256) void k_lz_finalize(LzFinalizeArgs p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (lz_finalize_block(a_.partial, a_.nblk, a_.st, a_.beta, a_.z, a_.max_steps, a_.tol,
                                a_.yscale, vb)));
}

// ---------------------------------------------------------------------------
// Non-Hermitian biorthogonal recursion (Sec. 2.5).  The two chains are kept
// unnormalised, v^_j = beta_j v_j and u^_j = conj(gamma_j) u_j, so that the
// scalings fold into the formation of the next pair:
//   v^_{j+1} = L v^_j / beta_j - (gamma_j / beta_{j-1}) v^_{j-1}
//   u^_{j+1} = L^dagger u^_j / conj(gamma_j) - (beta_j / conj(gamma_{j-1})) u^_{j-1}
//   s = (u^_{j+1}, v^_{j+1}),  beta_{j+1} = sqrt|s|,  gamma_{j+1} = s / beta_{j+1},
//   z_{j+1} = (y, v^_{j+1}) / beta_{j+1} for an upper vector, else 0.
// ---------------------------------------------------------------------------


// Block partial sums of w_k |y|^2 over the internal layout [k][n][G]
// (4 entries per block, the last three zero).
template <typename T>
__global__ __launch_bounds__(256) void k_nh_norm(const cplx<T>* __restrict__ y,
                                                 const double* __restrict__ wk, int64_t per_k,
                                                 int nks, double* __restrict__ partial) {
  __shared__ double red[256];
  const int64_t n = per_k * nks;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<T> v = y[i];
    acc += wk[i / per_k] * (double(v.x) * double(v.x) + double(v.y) * double(v.y));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[4 * blockIdx.x + 0] = red[0];
    partial[4 * blockIdx.x + 1] = 0.0;
    partial[4 * blockIdx.x + 2] = 0.0;
    partial[4 * blockIdx.x + 3] = 0.0;
  }
}

// Sum the partials (4 per block) and take the scalar decisions of one
// non-Hermitian step.  j = st->step.  j == 0: the partials hold ||y||^2;
// beta_1 = gamma_1 = ||y|| (breakdown when y vanished).  j >= 1: the
// partials hold (s, (y, v^_{j+1})); breakdown when |s| <= (tol bmax)^2 with
// bmax the largest beta_2..beta_j.  gamma and z are complex (re, im).
__global__ __launch_bounds__(256) void k_nh_finalize(const double* __restrict__ partial, int nblk,
                                                     LzDevState* __restrict__ st,
                                                     double* __restrict__ beta,
                                                     double* __restrict__ gam,
                                                     double* __restrict__ z, int max_steps,
                                                     double tol, double yscale) {
  __shared__ double red[4][kDotThreads];
  if (st->status) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += kDotThreads)
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] += partial[i * 4 + r];
#pragma unroll
  for (int r = 0; r < 4; ++r) red[r][threadIdx.x] = a[r];
  __syncthreads();
  for (int h = kDotThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
#pragma unroll
      for (int r = 0; r < 4; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double sr = red[0][0], si = red[1][0], zr = red[2][0], zi = red[3][0];
  const int j = st->step;
  if (j >= max_steps) { st->status = 5; return; }
  if (!isfinite(sr) || !isfinite(si) || !isfinite(zr) || !isfinite(zi)) { st->status = 7; return; }
  if (j == 0) {
    if (sr <= tol * tol * yscale) { st->status = 6; return; }  // y = 0: chi vanishes
    const double bt = sqrt(sr);
    beta[0] = bt;
    gam[0] = bt;
    gam[1] = 0.0;
    z[0] = 0.0;
    z[1] = 0.0;
    st->cv1[0] = 1.0 / bt; st->cv1[1] = 0.0;
    st->cu1[0] = 1.0 / bt; st->cu1[1] = 0.0;
    st->cv2[0] = st->cv2[1] = 0.0;  // no vector before the first
    st->cu2[0] = st->cu2[1] = 0.0;
    st->beta_prev = bt;
    st->gamma_prev[0] = bt;
    st->gamma_prev[1] = 0.0;
    st->bmax = 0.0;
    st->step = 1;
    return;
  }
  const double as = hypot(sr, si);
  const double bm = st->bmax;
  if (as <= (tol * bm) * (tol * bm)) { st->status = 6; return; }
  const double bt = sqrt(as);
  const double gr = sr / bt, gi = si / bt;
  beta[j] = bt;
  gam[2 * j] = gr;
  gam[2 * j + 1] = gi;
  if (j & 1) {
    z[2 * j] = zr / bt;
    z[2 * j + 1] = zi / bt;
  } else {
    z[2 * j] = 0.0;
    z[2 * j + 1] = 0.0;
  }
  // next formation: cv1 = 1/beta_{j+1}, cv2 = -gamma_{j+1}/beta_j,
  // cu1 = 1/conj(gamma_{j+1}), cu2 = -beta_{j+1}/conj(gamma_j)
  const double g2 = gr * gr + gi * gi;
  const double pr = st->gamma_prev[0], pi = st->gamma_prev[1];
  const double p2 = pr * pr + pi * pi;
  st->cv1[0] = 1.0 / bt; st->cv1[1] = 0.0;
  st->cv2[0] = -gr / st->beta_prev; st->cv2[1] = -gi / st->beta_prev;
  st->cu1[0] = gr / g2; st->cu1[1] = gi / g2;          // 1/conj(g) = g/|g|^2
  st->cu2[0] = -bt * pr / p2; st->cu2[1] = -bt * pi / p2;
  st->bmax = bm > bt ? bm : bt;
  st->beta_prev = bt;
  st->gamma_prev[0] = gr;
  st->gamma_prev[1] = gi;
  st->step = j + 1;
}

__global__ __launch_bounds__(256) void k_set_state(LzDevState* st) {
  st->step = 0;
  st->status = 0;
  st->bmax = 0.0;
  st->a = 0.0;
  st->b = 0.0;
  st->beta_prev = 0.0;
  for (int r = 0; r < 2; ++r) {
    st->cv1[r] = st->cv2[r] = st->cu1[r] = st->cu2[r] = 0.0;
    st->gamma_prev[r] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// caller order <-> internal stick-major order
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_perm_in(const cplx<T>* __restrict__ xu, cplx<T>* __restrict__ xi,
                          const int* __restrict__ perm, const int* __restrict__ npw, int nbnd,
                          int npwx) {
  const int b = blockIdx.y, k = b / nbnd;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npwx) return;
  const int64_t o = (int64_t)b * npwx;
  xi[o + i] = i < npw[k] ? xu[o + perm[(int64_t)k * npwx + i]] : czero<T>();
}

template <typename T>
__global__ __launch_bounds__(256) void k_perm_out(const cplx<T>* __restrict__ xi, cplx<T>* __restrict__ xu,
                           const int* __restrict__ perm, const int* __restrict__ npw, int nbnd,
                           int npwx) {
  const int b = blockIdx.y, k = b / nbnd;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npwx) return;
  const int64_t o = (int64_t)b * npwx;
  if (i < npw[k]) xu[o + perm[(int64_t)k * npwx + i]] = xi[o + i];
  else xu[o + i] = czero<T>();
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(cplx<T>* __restrict__ d, const cplx<T>* __restrict__ s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

// ---------------------------------------------------------------------------
// spectrum: one thread per frequency.  chi needs (Re z, (w~ - T)^-1 e_1), which
// for symmetric T equals the first component of (w~ - T)^-1 z; eliminating
// from the last row upwards, x_j = c_j x_{j-1} + d_j with
//   den_j = w~ - beta_{j+1} c_{j+1},  c_j = beta_j / den_j,
//   d_j = (z_j + beta_{j+1} d_{j+1}) / den_j,   x_1 = d_1.
// |Im den_j| >= eta keeps every division away from zero.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Backward sweep of the transposed system, one frequency per thread, over the
// m coefficients of an extended tridiagonal matrix: beta_i for i <= m0 from
// the recursion, tail[i % 2] beyond (extrapolation), z_j = 0 for j > m0.
// With gam (complex, non-Hermitian recursion) T has super-diagonal gamma:
// the transposed system then has c_j = gamma_j / den_j, and z_j is taken
// complex.  No pivoting: |Im den_j| >= eta holds only for symmetric T.
__global__ __launch_bounds__(256) void k_spectrum(const double* __restrict__ beta,
                                                  const double* __restrict__ gam,
                                                  const double* __restrict__ z, int m0, int m,
                                                  double tail_even, double tail_odd,
                                                  const double* __restrict__ tail,
                                                  const double* __restrict__ omega, int nw,
                                                  double eta, double pref, double fq,
                                                  double* __restrict__ chi,
                                                  double* __restrict__ einv,
                                                  double* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  if (tail) {  // the tail means computed on the device (k_tail_means)
    tail_even = tail[0];
    tail_odd = tail[1];
  }
  auto bet = [&](int k) {  // beta_k, 1-based
    return k <= m0 ? beta[k - 1] : ((k & 1) ? tail_odd : tail_even);
  };
  const double2 wt = make_double2(omega[i], eta);
  double2 c = make_double2(0.0, 0.0), d = make_double2(0.0, 0.0);
  for (int j = m; j >= 1; --j) {
    const double bnext = j < m ? bet(j + 1) : 0.0;  // beta_{j+1}
    const double2 den = make_double2(wt.x - bnext * c.x, wt.y - bnext * c.y);
    // pseudo-Hermitian: z_j is real in exact arithmetic; its rounding-level
    // imaginary part is dropped
    const double zj = j <= m0 ? z[2 * (j - 1)] : 0.0;
    const double zij = (gam && j <= m0) ? z[2 * (j - 1) + 1] : 0.0;
    const double2 num = make_double2(zj + bnext * d.x, zij + bnext * d.y);
    d = zdiv(num, den);
    c = zdiv(gam ? make_double2(gam[2 * (j - 1)], gam[2 * (j - 1) + 1]) : make_double2(bet(j), 0.0),
             den);
  }
  double2 ch = make_double2(0.0, 0.0);
  if (m > 0) ch = make_double2(pref * beta[0] * d.x, pref * beta[0] * d.y);
  chi[2 * i] = ch.x;
  chi[2 * i + 1] = ch.y;
  einv[2 * i] = 1.0 + fq * ch.x;
  einv[2 * i + 1] = fq * ch.y;
  loss[i] = -fq * ch.y;
}

// Tail of the extrapolated tridiagonal matrix (Sec. 3.3): the mean of
// beta_lo..beta_m0 with lo = max(2, m0/2 + 1), over all of them ('constant')
// or over those of each index parity ('osc').  One thread adds in index
// order, the order of the host form in lz_spectrum_ext, so both give the
// same bits.  out[0] is the value for even indices, out[1] for odd ones.
__global__ void k_tail_means(const double* __restrict__ beta, int m0, int osc,
                             double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int lo = m0 / 2 + 1 > 2 ? m0 / 2 + 1 : 2;
  double sum[2] = {0.0, 0.0}, all = 0.0;
  int cnt[2] = {0, 0};
  for (int k = lo; k <= m0; ++k) {
    sum[k & 1] += beta[k - 1];
    cnt[k & 1] += 1;
    all += beta[k - 1];
  }
  if (osc) {
    out[0] = sum[0] / cnt[0];
    out[1] = sum[1] / cnt[1];
  } else {
    out[0] = out[1] = all / (cnt[0] + cnt[1]);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void LaunchLin<T>::proj_dot(const void* A, int P, int a_rows, void* X, const void* LW, int nbnd,
                            int npwx, int nks, int chunk, int nchunk, void* partial,
                            const LzDevState* st, hipStream_t s, int gemm) {
  if (gemm != kGemmValu) {
    const int tiles = ((P + kMfmaTile - 1) / kMfmaTile) * ((nbnd + kMfmaTile - 1) / kMfmaTile);
    if constexpr (sizeof(T) == 4) {
      if (gemm == kGemmBf16x3) {
        lz_launch(k_proj_dot_b3<>, k_proj_dot_b3<true>, dim3(tiles, nchunk, nks), dim3(256), 0, s,
                           (const float2*)A, P, a_rows, (const float2*)X, nbnd, npwx, chunk,
                           nchunk, (float2*)partial, st);
        return;
      }
    }
    lz_launch(k_proj_dot_mfma<T>, k_proj_dot_mfma<T, true>, dim3(tiles, nchunk, nks), dim3(256), 0,
              s,
                       (const cplx<T>*)A, P, a_rows, (const cplx<T>*)X, nbnd, npwx, chunk, nchunk,
                       (cplx<T>*)partial, st);
    return;
  }
  const int tpi = P <= 16 ? 1 : P <= 32 ? 2 : P <= 48 ? 3 : 4;
  const int tnj = nbnd <= 16 ? 1 : 2;
  const int tiles = ((P + 16 * tpi - 1) / (16 * tpi)) * ((nbnd + 16 * tnj - 1) / (16 * tnj));
  const bool upd = LW != nullptr;
  dim3 grid(tiles, nchunk, nks);
#define LZ_DOT(TPI, TNJ)                                                                       \
  if (upd)                                                                                     \
    lz_launch((k_proj_dot<T, TPI, TNJ, true>), (k_proj_dot<T, TPI, TNJ, true, true>), grid, dim3(256), 0, s, (const cplx<T>*)A, \
                       P, a_rows, (cplx<T>*)X, (const cplx<T>*)LW, nbnd, npwx, chunk, nchunk,  \
                       (cplx<T>*)partial, st);                                                 \
  else                                                                                         \
    lz_launch((k_proj_dot<T, TPI, TNJ, false>), (k_proj_dot<T, TPI, TNJ, false, true>), grid, dim3(256), 0, s, (const cplx<T>*)A, \
                       P, a_rows, (cplx<T>*)X, nullptr, nbnd, npwx, chunk, nchunk,             \
                       (cplx<T>*)partial, st);
  if (tnj == 1) {
    if (tpi == 1) { LZ_DOT(1, 1) } else if (tpi == 2) { LZ_DOT(2, 1) } else if (tpi == 3) { LZ_DOT(3, 1) } else { LZ_DOT(4, 1) }
  } else {
    if (tpi == 1) { LZ_DOT(1, 2) } else if (tpi == 2) { LZ_DOT(2, 2) } else if (tpi == 3) { LZ_DOT(3, 2) } else { LZ_DOT(4, 2) }
  }
#undef LZ_DOT
}

template <typename T>
int LaunchLin<T>::mfma_chunk(int P, int nbnd, int npwx, int nks) {
  const int tiles = ((P + kMfmaTile - 1) / kMfmaTile) * ((nbnd + kMfmaTile - 1) / kMfmaTile) * nks;
  const int target = std::max(1, 1024 / tiles);
  const int kc = mfma_kc<T>();
  int chunk = (npwx + target - 1) / target;
  chunk = std::max(kc, (chunk + kc - 1) / kc * kc);
  return chunk;
}

template <typename T>
bool LaunchLin<T>::dot_single_tile(int P, int nbnd, int gemm) {
  if (gemm != kGemmValu) return false;
  const int tpi = P <= 16 ? 1 : P <= 32 ? 2 : P <= 48 ? 3 : 4;
  const int tnj = nbnd <= 16 ? 1 : 2;
  return P <= 16 * tpi && nbnd <= 16 * tnj;
}

template <typename T>
void LaunchLin<T>::reduce(const void* partial, int nchunk, int P, int nbnd, int nks, void* R,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_plain<T>, dim3(nbnd, nks), dim3(256), (size_t)P * sizeof(cplx<T>),
                     s, (const cplx<T>*)partial, nchunk, P, nbnd, (cplx<T>*)R);
}

template <typename T>
void LaunchLin<T>::reduce_coef_in(const void* partial, int nchunk, const void* M,
                                  const double* dkb, int nbnd, int nproj, int nks, bool skip_pc,
                                  void* C, const LzDevState* st, hipStream_t s) {
  const size_t lds = (size_t)(nbnd + nproj) * sizeof(cplx<T>);
  lz_launch(k_reduce_coef_in<T>, k_reduce_coef_in<T, true>, dim3(nbnd, nks), dim3(256), lds, s,
                     (const cplx<T>*)partial, nchunk, (const cplx<T>*)M, dkb, nbnd, nproj,
                     skip_pc ? 1 : 0, (cplx<T>*)C, st);
}

template <typename T>
void LaunchLin<T>::reduce_coef_out(const void* partial, int nchunk, const void* Cin,
                                   const void* M, int nbnd, int nproj, int nks, void* C,
                                   const LzDevState* st, hipStream_t s) {
  const size_t lds = (size_t)nbnd * sizeof(cplx<T>);
  lz_launch(k_reduce_coef_out<T>, k_reduce_coef_out<T, true>, dim3(nbnd, nks), dim3(256), lds, s,
                     (const cplx<T>*)partial, nchunk, (const cplx<T>*)Cin, (const cplx<T>*)M,
                     nbnd, nproj, (cplx<T>*)C, st);
}

// bands per thread of the update, and thread groups sharing a block
static int upd_bands(int nbnd) { return nbnd <= 16 ? 4 : 8; }
template <typename T>
static int upd_groups(int P, int nbt) {
  return (size_t)P * 4 * nbt * sizeof(cplx<T>) <= 65536 ? 4 : 1;
}

template <typename T>
int LaunchLin<T>::update_blocks(int P, int nbnd, int npwx, int nks, int gemm) {
  if (gemm != kGemmValu)
    return ((npwx + kMfmaTile - 1) / kMfmaTile) * ((nbnd + kMfmaTile - 1) / kMfmaTile) * nks;
  const int nbt = upd_bands(nbnd);
  const int qn = upd_groups<T>(P, nbt);
  const int npt = 256 / qn;
  return ((npwx + npt - 1) / npt) * ((nbnd + qn * nbt - 1) / (qn * nbt)) * nks;
}

template <typename T>
static void launch_update(int mode, void* Y, const void* A, int P, int a_rows, const void* C,
                          int c_rows, int nbnd, int npwx, int nks, void* X, const void* y,
                          const void* U2, const double* wk, double* lzpart, const LzDevState* st,
                          hipStream_t s, int gemm) {
  if (gemm != kGemmValu) {
    dim3 grid((npwx + kMfmaTile - 1) / kMfmaTile, (nbnd + kMfmaTile - 1) / kMfmaTile, nks);
    if constexpr (sizeof(T) == 4) {
      if (gemm == kGemmBf16x3) {
#define LZ_UPDB(MODE)                                                                            \
  lz_launch((k_proj_update_b3<MODE>), (k_proj_update_b3<MODE, true>), grid, dim3(256), 0, s, (float2*)Y,                \
                     (const float2*)A, P, a_rows, (const float2*)C, c_rows, nbnd, npwx,          \
                     (float2*)X, (const float2*)y, (const float2*)U2, wk, lzpart, st);
        switch (mode) {
          case kUpdDots: LZ_UPDB(kUpdDots) break;
          case kUpdNhU: LZ_UPDB(kUpdNhU) break;
          case kUpdNhV: LZ_UPDB(kUpdNhV) break;
          default: LZ_UPDB(kUpdPlain) break;
        }
#undef LZ_UPDB
        return;
      }
    }
#define LZ_UPDM(MODE)                                                                            \
  lz_launch((k_proj_update_mfma<T, MODE>), (k_proj_update_mfma<T, MODE, true>), grid, dim3(256), 0, s, (cplx<T>*)Y,          \
                     (const cplx<T>*)A, P, a_rows, (const cplx<T>*)C, c_rows, nbnd, npwx,        \
                     (cplx<T>*)X, (const cplx<T>*)y, (const cplx<T>*)U2, wk, lzpart, st);
    switch (mode) {
      case kUpdDots: LZ_UPDM(kUpdDots) break;
      case kUpdNhU: LZ_UPDM(kUpdNhU) break;
      case kUpdNhV: LZ_UPDM(kUpdNhV) break;
      default: LZ_UPDM(kUpdPlain) break;
    }
#undef LZ_UPDM
    return;
  }
  const int nbt = upd_bands(nbnd);
  const int qn = upd_groups<T>(P, nbt);
  const int npt = 256 / qn;
  dim3 grid((npwx + npt - 1) / npt, (nbnd + qn * nbt - 1) / (qn * nbt), nks);
  const size_t lds = (size_t)P * qn * nbt * sizeof(cplx<T>);
#define LZ_UPD(NBT, MODE)                                                                        \
  lz_launch((k_proj_update<T, NBT, MODE>), (k_proj_update<T, NBT, MODE, true>), grid, dim3(256), lds, s, (cplx<T>*)Y,        \
                     (const cplx<T>*)A, P, a_rows, (const cplx<T>*)C, c_rows, nbnd, npwx,        \
                     (cplx<T>*)X, (const cplx<T>*)y, (const cplx<T>*)U2, wk, lzpart, qn, st);
#define LZ_UPD_MODES(NBT)                                          \
  switch (mode) {                                                  \
    case kUpdDots: LZ_UPD(NBT, kUpdDots) break;                    \
    case kUpdNhU: LZ_UPD(NBT, kUpdNhU) break;                      \
    case kUpdNhV: LZ_UPD(NBT, kUpdNhV) break;                      \
    default: LZ_UPD(NBT, kUpdPlain) break;                         \
  }
  if (nbt == 4) { LZ_UPD_MODES(4) } else { LZ_UPD_MODES(8) }
#undef LZ_UPD_MODES
#undef LZ_UPD
}

template <typename T>
void LaunchLin<T>::proj_update(void* Y, const void* A, int P, int a_rows, const void* C,
                               int c_rows, int nbnd, int npwx, int nks, const void* X,
                               const void* y, const double* wk, double* lzpart,
                               const LzDevState* st, hipStream_t s, int gemm) {
  launch_update<T>(lzpart != nullptr ? kUpdDots : kUpdPlain, Y, A, P, a_rows, C, c_rows, nbnd,
                   npwx, nks, const_cast<void*>(X), y, nullptr, wk, lzpart, st, s, gemm);
}

template <typename T>
void LaunchLin<T>::nh_form(bool v_chain, void* LY, const void* A, int P, const void* C, int nbnd,
                           int npwx, int nks, void* H, const void* y, const void* U2,
                           const double* wk, double* lzpart, const LzDevState* st,
                           hipStream_t s, int gemm) {
  launch_update<T>(v_chain ? kUpdNhV : kUpdNhU, LY, A, P, P, C, P, nbnd, npwx, nks, H, y, U2, wk,
                   v_chain ? lzpart : nullptr, st, s, gemm);
}

template <typename T>
void LaunchLin<T>::lz_update(void* w, const void* lw, int64_t n, const LzDevState* st, hipStream_t s) {
  lz_launch(k_lz_update<T>, k_lz_update<T, true>, dim3(1024), dim3(256), 0, s, (cplx<T>*)w,
                     (const cplx<T>*)lw, n, st);
}

template <typename T>
void LaunchLin<T>::perm_in(const void* xu, void* xi, const int* perm, const int* npw, int nks,
                        int nbnd, int npwx, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_in<T>, dim3((npwx + 255) / 256, nks * nbnd), dim3(256), 0, s,
                     (const cplx<T>*)xu, (cplx<T>*)xi, perm, npw, nbnd, npwx);
}

template <typename T>
void LaunchLin<T>::perm_out(const void* xi, void* xu, const int* perm, const int* npw, int nks,
                         int nbnd, int npwx, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_out<T>, dim3((npwx + 255) / 256, nks * nbnd), dim3(256), 0, s,
                     (const cplx<T>*)xi, (cplx<T>*)xu, perm, npw, nbnd, npwx);
}

template <typename T>
void LaunchLin<T>::copy(void* dst, const void* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<T>, dim3(1024), dim3(256), 0, s, (cplx<T>*)dst, (const cplx<T>*)src, n);
}

void launch_lz_finalize(const double* partial, int nblk, LzDevState* st, double* beta, double* z,
                        int max_steps, double tol, double yscale, hipStream_t s) {
  lz_launch(k_lz_finalize<>, k_lz_finalize<true>, dim3(1), dim3(kDotThreads), 0, s, partial, nblk,
            st, beta, z,
                     max_steps, tol, yscale);
}

void launch_spectrum(const double* beta, const double* gam, const double* z, int m0, int m,
                     double tail_even, double tail_odd, const double* omega, int nw, double eta,
                     double pref, double fq, double* chi, double* einv, double* loss,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum, dim3((nw + 63) / 64), dim3(64), 0, s, beta, gam, z, m0, m,
                     tail_even, tail_odd, nullptr, omega, nw, eta, pref, fq, chi, einv, loss);
}

void launch_spectrum_dev_tail(const double* beta, const double* gam, const double* z, int m0,
                              int m, int osc, double* tail, const double* omega, int nw,
                              double eta, double pref, double fq, double* chi, double* einv,
                              double* loss, hipStream_t s) {
  if (m > m0) hipLaunchKernelGGL(k_tail_means, dim3(1), dim3(64), 0, s, beta, m0, osc, tail);
  hipLaunchKernelGGL(k_spectrum, dim3((nw + 63) / 64), dim3(64), 0, s, beta, gam, z, m0, m, 0.0,
                     0.0, m > m0 ? tail : nullptr, omega, nw, eta, pref, fq, chi, einv, loss);
}

template <typename T>
void launch_nh_norm(const void* y, const double* wk, int64_t per_k, int nks, double* partial,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_nh_norm<T>, dim3(kNhNormBlocks), dim3(256), 0, s, (const cplx<T>*)y, wk,
                     per_k, nks, partial);
}
template void launch_nh_norm<float>(const void*, const double*, int64_t, int, double*, hipStream_t);
template void launch_nh_norm<double>(const void*, const double*, int64_t, int, double*, hipStream_t);

void launch_nh_finalize(const double* partial, int nblk, LzDevState* st, double* beta, double* gam,
                        double* z, int max_steps, double tol, double yscale, hipStream_t s) {
  hipLaunchKernelGGL(k_nh_finalize, dim3(1), dim3(kDotThreads), 0, s, partial, nblk, st, beta, gam,
                     z, max_steps, tol, yscale);
}

void launch_set_state(LzDevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st);
}

void launch_heev(void* A, int n, int ld, double* w, void* V, int nks, hipStream_t s) {
  hipLaunchKernelGGL(k_heev_jacobi, dim3(nks), dim3(kHeevThreads), 0, s, (double2*)A, n, ld, w, (double2*)V,
                     30);
}
void launch_small_take(void* dst, const void* src, int rows, int cols, int lds, int col0,
                       int src_stride, double alpha, int nks, hipStream_t s) {
  hipLaunchKernelGGL(k_small_take, dim3(nks), dim3(256), 0, s, (double2*)dst, (const double2*)src,
                     rows, cols, lds, col0, src_stride, alpha);
}
void launch_orth_coef(const void* Q, const double* lam, int m, double tol, void* C, int* keep,
                      int nks, hipStream_t s) {
  hipLaunchKernelGGL(k_orth_coef, dim3(nks), dim3(256), 0, s, (const double2*)Q, lam, m, tol,
                     (double2*)C, keep);
}
void launch_mask_dropped(void* T, int n2, int off, int cnt, const int* keep, int nks,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_mask_dropped, dim3(nks), dim3(256), 0, s, (double2*)T, n2, off, cnt, keep);
}
void launch_gs_residual(const void* X, const void* HX, const double* theta, const void* kin, int m,
                        int npwx, int nks, double e0, void* R, void* W, hipStream_t s) {
  hipLaunchKernelGGL(k_gs_residual, dim3(1024), dim3(256), 0, s, (const double2*)X,
                     (const double2*)HX, theta, (const double*)kin, m, npwx, nks, e0, (double2*)R,
                     (double2*)W);
}

void launch_cheb_step(void* out, const void* HY, const void* Y, const void* Xold,
                      const double* coef, int m, int npwx, int nks, hipStream_t s) {
  hipLaunchKernelGGL(k_cheb_step, dim3(1024), dim3(256), 0, s, (double2*)out, (const double2*)HY,
                     (const double2*)Y, (const double2*)Xold, coef, m, npwx, nks);
}

void launch_gram_unit(void* G, int m, double* dscale, int nks, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_unit, dim3(nks), dim3(256), 0, s, (double2*)G, m, dscale);
}
void launch_row_scale(void* C, int m, const double* dscale, int nks, hipStream_t s) {
  hipLaunchKernelGGL(k_row_scale, dim3(nks), dim3(256), 0, s, (double2*)C, m, dscale);
}

void launch_ground_density(const void* ur, const double* w, int nb, int64_t np, int xc,
                           double* n0, double* fxc, hipStream_t s) {
  hipLaunchKernelGGL(k_ground_density, dim3(1024), dim3(256), 0, s, (const double2*)ur, w, nb, np,
                     xc, n0, fxc);
}

template struct LaunchLin<double>;
template struct LaunchLin<float>;

}  // namespace lz
