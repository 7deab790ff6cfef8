// FFT-based kernels of the Liouvillian application (Secs. 2.3-2.4 of the
// turboEELS paper): the local part of H_{k+q}, the response density, the
// Hartree + ALDA response potential and v'u.  Included by one translation unit
// per precision.
//
// Data layouts (per instance):
//   sphere vectors   [k][band][npwx] complex, plane waves in stick-major order
//                    (sorted by stick, then by z index): one stick is a run;
//   sticks           [band][z][S] complex after the z-direction transform;
//   real-space grids plane-major [z][i1][i2].
// A band's 3-D transform is a z pass over the S sticks that touch the sphere
// (about a fifth of the N1*N2 columns) and a 2-D pass per z-plane held in
// LDS, in which only the rows carrying a stick are transformed along i2.
//
// Every kernel has two forms selected by the template argument N: N > 0 is
// the compile-time form for cubic grids N^3 with a plan in lz_fft_ct.h, N = 0
// the general form driven by runtime plans.  Both run 256 threads per block.
// Every reduction has a fixed order, so repeated runs are bitwise identical.
#pragma once
#include <stdexcept>
#include <vector>

#include "lz_fft_ct.h"
#include "lz_kernels.h"
#include "lz_plane_reg.h"

namespace lz {

template <typename T>
__device__ __forceinline__ cplx<T> czero() { return mk<T>(T(0), T(0)); }

// LDS row pitch of a compile-time plane: 48^2 planes take N + 3 (51 complex
// values, 204 dwords = 12 mod 32 and mod 64), so that the lanes of the radix-16
// row pass (three butterflies per row) and the column passes fall in distinct
// banks; N + 1 elsewhere
template <int N> __host__ __device__ constexpr int ct_plane_pitch() {
  return N == 48 ? N + 3 : N + 1;
}

// threads of a plane block, so that the blocks the LDS admits on a compute
// unit hold about 16 waves: FP64 planes of 72^2 and 96^2 (one block per
// unit) take 1024 threads, 64^2 (two) 512; FP32 96^2 planes (two) 512; the
// rest 256.  More threads also mean fewer butterflies held per thread.
template <typename T, int N> __host__ __device__ constexpr int plane_threads() {
  return sizeof(T) == 8 ? (N >= 72 ? 1024 : N == 64 ? 512 : 256) : (N == 96 ? 512 : 256);
}

struct PlaneArgs {
  int n1, n2, n3, S, nact, pitch;
  const int* si1;
  const int* si2;
  const int* act;
  FftPlan p1, p2;
};

// LDS of a plane kernel: plane [n1][n2+1], then (compile-time form) the
// twiddle table and the list of active rows.
template <typename T, int N>
struct PlaneShm {
  cplx<T>* plane;
  const cplx<T>* tw;  // compile-time form: LDS copy; general form: unused
  const int* act;     // active rows (LDS copy in the compile-time form)
  __device__ __forceinline__ PlaneShm(unsigned char* raw, const PlaneArgs& a, const void* twg,
                                      int tid) {
    plane = reinterpret_cast<cplx<T>*>(raw);
    if constexpr (N > 0) {
      constexpr int P = ct_plane_pitch<N>();
      cplx<T>* t = plane + N * P;
      int* r = reinterpret_cast<int*>(t + ct_twsize(N));
      const cplx<T>* tg = reinterpret_cast<const cplx<T>*>(twg);
      for (int i = tid; i < ct_twsize(N); i += plane_threads<T, N>()) t[i] = tg[i];
      for (int i = tid; i < a.nact; i += plane_threads<T, N>()) r[i] = a.act[i];
      tw = t;
      act = r;
    } else {
      tw = nullptr;
      act = a.act;
    }
  }
};

template <typename T, int N>
__host__ __device__ constexpr size_t plane_shm_bytes_ct() {
  return (size_t)(N * ct_plane_pitch<N>() + ct_twsize(N)) * sizeof(cplx<T>) +
         (size_t)N * sizeof(int);
}

// 1-D transforms of a plane: rows listed in act (along i2) or all columns
// (along i1); for the general form tw1/tw2 are the runtime tables.
template <typename T, int N, int MP, int DIR>
__device__ __forceinline__ void plane_rows(const PlaneShm<T, N>& sh, const PlaneArgs& a, int nrows,
                                           bool listed, const cplx<T>* tw2, int tid) {
  if constexpr (N > 0) {
    constexpr int NT = plane_threads<T, N>(), P = ct_plane_pitch<N>();
    if (listed) ct_fft<T, N, DIR, N, LayRows<P>, NT>(sh.plane, LayRows<P>{sh.act}, nrows, sh.tw, tid);
    else ct_fft<T, N, DIR, N, LayRowsAll<P>, NT>(sh.plane, LayRowsAll<P>{}, nrows, sh.tw, tid);
  } else {
    fft_lds<T, MP, DIR>(sh.plane, Lay{1, a.pitch, listed ? sh.act : nullptr}, a.p2, nrows, tw2, tid, 256);
  }
}

template <typename T, int N, int MP, int DIR>
__device__ __forceinline__ void plane_cols(const PlaneShm<T, N>& sh, const PlaneArgs& a,
                                           const cplx<T>* tw1, int tid) {
  if constexpr (N > 0) {
    constexpr int P = ct_plane_pitch<N>();
    ct_fft<T, N, DIR, N, LayCols<P>, plane_threads<T, N>()>(sh.plane, LayCols<P>{}, N, sh.tw, tid);
  } else {
    fft_lds<T, MP, DIR>(sh.plane, Lay{a.pitch, 1, nullptr}, a.p1, a.n2, tw1, tid, 256);
  }
}

// the local potential of a z-plane as a last-pass epilogue of the inverse
// column transforms: element i1 of column i2 is scaled by V(i1, i2)
template <typename T>
struct PotentialEpilogue {
  const T* vz;
  int n2;
  template <typename U>
  __device__ __forceinline__ U load(int col, int row) const { return vz[row * n2 + col]; }
};

template <typename T, int N>
__device__ __forceinline__ void plane_zero_scatter(const PlaneShm<T, N>& sh, const PlaneArgs& a,
                                                   const cplx<T>* __restrict__ src, int tid) {
  const int n1 = N > 0 ? N : a.n1;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  constexpr int NT = N > 0 ? plane_threads<T, N>() : 256;
  for (int t = tid; t < n1 * pitch; t += NT) sh.plane[t] = czero<T>();
  __syncthreads();
  for (int s = tid; s < a.S; s += NT) sh.plane[a.si1[s] * pitch + a.si2[s]] = src[s];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// z pass, inverse: sphere -> sticks
// ---------------------------------------------------------------------------
// sticks per block of the z passes (measured: 64-stick tiles on the
// compile-time grids are slower; the passes want many small blocks)
__host__ __device__ constexpr int zpass_tile(int) { return kStickTile; }

template <typename T, int N, int ST = kStickTile>
__device__ __forceinline__ void stick_fft(cplx<T>* lds, int pitch, const FftPlan& pz, int nst,
                                          const cplx<T>* tw, int tid, int dir) {
  if constexpr (N > 0) {
    if (dir > 0) ct_fft<T, N, +1, ST>(lds, LayRowsAll<N + 1>{}, nst, tw, tid);
    else ct_fft<T, N, -1, ST>(lds, LayRowsAll<N + 1>{}, nst, tw, tid);
  } else {
    if (dir > 0) fft_lds<T, kStickMaxPt, +1>(lds, Lay{1, pitch, nullptr}, pz, nst, tw, tid, 256);
    else fft_lds<T, kStickMaxPt, -1>(lds, Lay{1, pitch, nullptr}, pz, nst, tw, tid, 256);
  }
}

// twiddles of the z plan: LDS copy behind the tile of ST lines (compile-time form)
template <typename T, int N, int ST = kStickTile>
__device__ __forceinline__ const cplx<T>* stick_tw(cplx<T>* lds, const cplx<T>* twg, int tid) {
  if constexpr (N > 0) {
    cplx<T>* t = lds + ST * (N + 1);
    for (int i = tid; i < ct_twsize(N); i += 256) t[i] = twg[i];
    return t;
  } else {
    return twg;
  }
}

template <typename T>
struct ZfftInvArgs {
  const cplx<T>* x;
  int64_t xs;
  cplx<T>* out;
  const int* map;
  int S;
  int n3_rt;
  int nbnd;
  FftPlan pz;
  const cplx<T>* twg;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void zfft_inv_block(const cplx<T>* __restrict__ x, int64_t xs,
                                               cplx<T>* __restrict__ out,
                                               const int* __restrict__ map, int S, int n3_rt,
                                               int nbnd, const FftPlan& pz,
                                               const cplx<T>* __restrict__ twg,
                                               const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  constexpr int ST = zpass_tile(N);
  const int s0 = vb.x * ST;
  const int nst = min(ST, S - s0);
  if constexpr (N > 0) {
    // bands 2 j and 2 j + 1 of k-point k (vb.y = k ceil(nbnd / 2) + j)
    // share the map of the tile: every map index, then the gathered values
    // of both bands, are in flight before the first is used; the two tiles
    // (lines [0, ST) and [ST, 2 ST)) go through one transform
    constexpr int pitch = N + 1;
    const int hp = (nbnd + 1) / 2;
    const int k = vb.y / hp, j = 2 * (vb.y - k * hp);
    const int b = k * nbnd + j;
    const bool two = j + 1 < nbnd;
    const cplx<T>* tw = stick_tw<T, N, 2 * ST>(lds, twg, tid);
    const cplx<T>* xb = x + b * xs;
    const int* mp = map + ((int64_t)k * S + s0) * N;
    constexpr int IT = (ST * N + 255) / 256;
    int idx[IT];
    cplx<T> v0[IT], v1[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * 256;
      idx[i] = t < nst * N ? mp[t] : -1;
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      v0[i] = idx[i] >= 0 ? xb[idx[i]] : czero<T>();
      v1[i] = two && idx[i] >= 0 ? xb[xs + idx[i]] : czero<T>();
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * 256;
      if (t < nst * N) {
        const int ls = t / N, z = t - ls * N;
        lds[ls * pitch + z] = v0[i];
        lds[(ST + ls) * pitch + z] = v1[i];
      }
    }
    __syncthreads();
    stick_fft<T, N, 2 * ST>(lds, pitch, pz, ST + nst, tw, tid, +1);
    cplx<T>* ob = out + (int64_t)b * N * S + s0;
    for (int t = tid; t < nst * N; t += 256) {
      const int z = t / nst, ls = t - z * nst;
      ob[(int64_t)z * S + ls] = lds[ls * pitch + z];
      if (two) ob[(int64_t)(N + z) * S + ls] = lds[(ST + ls) * pitch + z];
    }
    return;
  }
  const int n3 = N > 0 ? N : n3_rt;
  const int b = vb.y;
  const int k = b / nbnd;
  const int pitch = n3 + 1;
  const cplx<T>* tw = stick_tw<T, N, ST>(lds, twg, tid);
  const cplx<T>* xb = x + b * xs;
  const int* mp = map + ((int64_t)k * S + s0) * n3;
  {
    for (int t = tid; t < nst * n3; t += 256) {
      const int ls = t / n3, z = t - ls * n3;
      const int idx = mp[ls * n3 + z];
      lds[ls * pitch + z] = idx >= 0 ? xb[idx] : czero<T>();
    }
  }
  __syncthreads();
  stick_fft<T, N, ST>(lds, pitch, pz, nst, tw, tid, +1);
  cplx<T>* ob = out + (int64_t)b * n3 * S + s0;
  for (int t = tid; t < nst * n3; t += 256) {
    const int z = t / nst, ls = t - z * nst;
    ob[(int64_t)z * S + ls] = lds[ls * pitch + z];
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(256) void k_zfft_inv(ZfftInvArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (zfft_inv_block<T, N>(a_.x, a_.xs, a_.out, a_.map, a_.S, a_.n3_rt, a_.nbnd, a_.pz,
                                   a_.twg, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// z pass, forward: sticks -> sphere; y = x_fft/N + (kin - eps) x
// ---------------------------------------------------------------------------
template <typename T>
struct ZfftFwdArgs {
  const cplx<T>* sticks;
  const cplx<T>* x;
  int64_t xs;
  cplx<T>* y;
  const int* map;
  const T* kin;
  const double* eps;
  int S;
  int n3_rt;
  int nbnd;
  int npwx;
  T scale;
  FftPlan pz;
  const cplx<T>* twg;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void zfft_fwd_block(const cplx<T>* __restrict__ sticks,
                                               const cplx<T>* __restrict__ x, int64_t xs,
                                               cplx<T>* __restrict__ y, const int* __restrict__ map,
                                               const T* __restrict__ kin,
                                               const double* __restrict__ eps, int S, int n3_rt,
                                               int nbnd, int npwx, T scale, const FftPlan& pz,
                                               const cplx<T>* __restrict__ twg,
                                               const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n3 = N > 0 ? N : n3_rt;
  const int b = vb.y;
  const int k = b / nbnd;
  constexpr int ST = zpass_tile(N);
  const int s0 = vb.x * ST;
  const int nst = min(ST, S - s0);
  const int pitch = n3 + 1;
  const int tid = threadIdx.x;
  const cplx<T>* tw = stick_tw<T, N, ST>(lds, twg, tid);
  const cplx<T>* sb = sticks + (int64_t)b * n3 * S + s0;
  const int* mp = map + ((int64_t)k * S + s0) * n3;
  const cplx<T>* xb = x + b * xs;
  cplx<T>* yb = y + b * xs;
  const T* kb = kin + (int64_t)k * npwx;
  const T e = T(eps[b]);
  if constexpr (N > 0) {
    // the map, then x and the kinetic energies it points to, are loaded
    // before the transform (they do not depend on it): one memory latency
    // of the chain overlaps the stick loads and the transform
    constexpr int IT = (ST * N + 255) / 256;
    int idx[IT];
    cplx<T> xv[IT];
    T kv[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * 256;
      idx[i] = t < nst * N ? mp[t] : -1;
    }
    for (int t = tid; t < nst * n3; t += 256) {
      const int z = t / nst, ls = t - z * nst;
      lds[ls * pitch + z] = sb[(int64_t)z * S + ls];
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      xv[i] = idx[i] >= 0 ? xb[idx[i]] : czero<T>();
      kv[i] = idx[i] >= 0 ? kb[idx[i]] : T(0);
    }
    __syncthreads();
    stick_fft<T, N, ST>(lds, pitch, pz, nst, tw, tid, -1);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * 256;
      if (idx[i] >= 0) {
        const int ls = t / N, z = t - ls * N;
        const cplx<T> f = lds[ls * pitch + z];
        const T d = kv[i] - e;
        yb[idx[i]] = mk<T>(f.x * scale + d * xv[i].x, f.y * scale + d * xv[i].y);
      }
    }
  } else {
    for (int t = tid; t < nst * n3; t += 256) {
      const int z = t / nst, ls = t - z * nst;
      lds[ls * pitch + z] = sb[(int64_t)z * S + ls];
    }
    __syncthreads();
    stick_fft<T, N, ST>(lds, pitch, pz, nst, tw, tid, -1);
    for (int t = tid; t < nst * n3; t += 256) {
      const int ls = t / n3, z = t - ls * n3;
      const int idx = mp[ls * n3 + z];
      if (idx >= 0) {
        const cplx<T> f = lds[ls * pitch + z];
        const cplx<T> xv = xb[idx];
        const T d = kb[idx] - e;
        yb[idx] = mk<T>(f.x * scale + d * xv.x, f.y * scale + d * xv.y);
      }
    }
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(256) void k_zfft_fwd(ZfftFwdArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (zfft_fwd_block<T, N>(a_.sticks, a_.x, a_.xs, a_.y, a_.map, a_.kin, a_.eps, a_.S,
                                   a_.n3_rt, a_.nbnd, a_.npwx, a_.scale, a_.pz, a_.twg, a_.st,
                                   vb)));
}

// ---------------------------------------------------------------------------
// plane pass of a D step: x(r) = IFFT2 sticks, (V x)(r), FFT2 -> sticks
// ---------------------------------------------------------------------------
template <typename T>
struct PlaneLocalArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  PlaneArgs a;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
  const LzDevState* st;
};

template <typename T, int N, int MP>
__device__ __forceinline__ void plane_local_block(const cplx<T>* __restrict__ sin,
                                                  cplx<T>* __restrict__ sout,
                                                  const T* __restrict__ vloc, const PlaneArgs& a,
                                                  const cplx<T>* __restrict__ tw1,
                                                  const cplx<T>* __restrict__ tw2,
                                                  const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  constexpr int NTB = N > 0 ? plane_threads<T, N>() : 256;
  PlaneShm<T, N> sh(smem_raw, a, tw1, tid);
  const int n1 = N > 0 ? N : a.n1, n2 = N > 0 ? N : a.n2, n3 = N > 0 ? N : a.n3;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  const int z = vb.x, b = vb.y;
  const int64_t so = ((int64_t)b * n3 + z) * a.S;
  plane_zero_scatter<T, N>(sh, a, sin + so, tid);
  plane_rows<T, N, MP, +1>(sh, a, a.nact, true, tw2, tid);
  const T* vz = vloc + (int64_t)z * n1 * n2;
  if constexpr (N > 0) {
    // the potential multiplies the outputs of the last inverse column pass
    // as they are stored: no separate sweep over the plane
    ct_fft<T, N, +1, N, LayCols<ct_plane_pitch<N>()>, plane_threads<T, N>()>(
        sh.plane, LayCols<ct_plane_pitch<N>()>{}, N, sh.tw, tid, PotentialEpilogue<T>{vz, N});
  } else {
    plane_cols<T, N, MP, +1>(sh, a, tw1, tid);
    for (int p = tid; p < n1 * n2; p += NTB) {
      const int i1 = p / n2, i2 = p - i1 * n2;
      cplx<T>& c = sh.plane[i1 * pitch + i2];
      c = cscale<T>(c, vz[p]);
    }
    __syncthreads();
  }
  plane_cols<T, N, MP, -1>(sh, a, tw1, tid);
  plane_rows<T, N, MP, -1>(sh, a, a.nact, true, tw2, tid);
  for (int s = tid; s < a.S; s += NTB) sout[so + s] = sh.plane[a.si1[s] * pitch + a.si2[s]];
}

template <typename T, int N, int MP, bool BAT = false>
__global__ __launch_bounds__((plane_threads<T, N>())) void k_plane_local(PlaneLocalArgs<T> p,
                                                                    BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (plane_local_block<T, N, MP>(a_.sin, a_.sout, a_.vloc, a_.a, a_.tw1, a_.tw2, a_.st,
                                          vb)));
}

// ---------------------------------------------------------------------------
// plane pass of a D+K step: as above for a group of bands, accumulating the
// response density  n'(r) += (4 w_k / Omega) conj(u_b(r)) x_b(r)  (raw values
// of u and x, i.e. without the Omega^-1/2 factors, which bandw absorbs).
// ---------------------------------------------------------------------------
template <typename T>
struct PlaneLocalDensityArgs {
  const cplx<T>* sin;
  cplx<T>* sout;
  const T* vloc;
  const cplx<T>* ur;
  const double* bandw;
  cplx<T>* dpart;
  int nb;
  int gsize;
  PlaneArgs a;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
  const LzDevState* st;
};

template <typename T, int N, int MP>
__device__ __forceinline__ void plane_local_density_block(const cplx<T>* __restrict__ sin,
                                                          cplx<T>* __restrict__ sout,
                                                          const T* __restrict__ vloc,
                                                          const cplx<T>* __restrict__ ur,
                                                          const double* __restrict__ bandw,
                                                          cplx<T>* __restrict__ dpart, int nb,
                                                          int gsize, const PlaneArgs& a,
                                                          const cplx<T>* __restrict__ tw1,
                                                          const cplx<T>* __restrict__ tw2,
                                                          const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid0 = threadIdx.x;
  constexpr int NTB = N > 0 ? plane_threads<T, N>() : 256;
  PlaneShm<T, N> sh(smem_raw, a, tw1, tid0);
  const int n1 = N > 0 ? N : a.n1, n2 = N > 0 ? N : a.n2, n3 = N > 0 ? N : a.n3;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  // large planes (72^2 and 96^2 in double precision, 96^2 in single) keep the
  // running sums in dpart itself (the block's own slice, read and written by
  // the same thread in band order: the same sums, bitwise, as register
  // accumulators, which would spill)
  constexpr bool GACC = sizeof(T) == 8 ? N >= 72 : N >= 96;
  constexpr int NIT = N > 0 ? (N * N + NTB - 1) / NTB : MP;
  constexpr int ACC = GACC ? 1 : NIT;
  constexpr int UNR = GACC ? 4 : NIT;
  // FP64 planes of 48^2 and 96^2 load the first NPRE of a thread's orbital
  // values of a band before the band's transforms, which hide their
  // latency: on 48^2 planes 5 of 9 fill the registers of three waves per
  // SIMD (168; more leave two), on 96^2 planes (1024 threads, at most 128
  // registers) 3 of 9 fit
  constexpr bool PRE = sizeof(T) == 8 && (N == 48 || N == 96);
  constexpr int NPRE = !PRE ? 0 : N == 48 ? 5 : 3;
  const int z = vb.x, g = vb.y;
  const int np = n1 * n2;
  const T* vz = vloc + (int64_t)z * np;
  cplx<T>* dp = dpart + ((int64_t)g * n3 + z) * np;
  cplx<T> acc[ACC];
#pragma unroll
  for (int i = 0; i < ACC; ++i) acc[i] = czero<T>();
  const int b0 = g * gsize, b1 = min(nb, b0 + gsize);
  for (int b = b0; b < b1; ++b) {
    // the thread index passes through an empty asm statement on every band,
    // so that the compiler forms the transforms' LDS addresses per band
    // instead of holding all of them in registers through the loop (FP64
    // 48^2 planes: 138 registers instead of 232 before the orbital loads
    // below, three waves per SIMD instead of two)
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int64_t so = ((int64_t)b * n3 + z) * a.S;
    const cplx<T>* ub = ur + ((int64_t)b * n3 + z) * np;
    cplx<T> upre[NPRE > 0 ? NPRE : 1];
    if constexpr (PRE) {
#pragma unroll
      for (int i = 0; i < NPRE; ++i) {
        const int p = tid + i * NTB;
        upre[i] = p < np ? ub[p] : czero<T>();
      }
    }
    plane_zero_scatter<T, N>(sh, a, sin + so, tid);
    plane_rows<T, N, MP, +1>(sh, a, a.nact, true, tw2, tid);
    plane_cols<T, N, MP, +1>(sh, a, tw1, tid);
    const T wb = T(bandw[b]);
    // point i of the thread: the density product with the orbital value u,
    // then the potential
    auto point = [&](int i, const cplx<T>& u) {
      const int p = tid + i * NTB;
      const int i1 = p / n2, i2 = p - i1 * n2;
      cplx<T>& c = sh.plane[i1 * pitch + i2];
      const cplx<T> d = cmulc<T>(u, c);
      if constexpr (GACC) {
        cplx<T> s = b == b0 ? czero<T>() : dp[p];
        s.x += wb * d.x;
        s.y += wb * d.y;
        dp[p] = s;
      } else {
        acc[i].x += wb * d.x;
        acc[i].y += wb * d.y;
      }
      c = cscale<T>(c, vz[p]);
    };
#pragma unroll
    for (int i = 0; i < NPRE; ++i)
      if (tid + i * NTB < np) point(i, upre[i]);
#pragma unroll UNR
    for (int i = NPRE; i < NIT; ++i)
      if (tid + i * NTB < np) point(i, ub[tid + i * NTB]);
    __syncthreads();
    plane_cols<T, N, MP, -1>(sh, a, tw1, tid);
    plane_rows<T, N, MP, -1>(sh, a, a.nact, true, tw2, tid);
    for (int s = tid; s < a.S; s += NTB) sout[so + s] = sh.plane[a.si1[s] * pitch + a.si2[s]];
    __syncthreads();
  }
  if constexpr (!GACC) {
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
      const int p = tid0 + i * NTB;
      if (p < np) dp[p] = acc[i];
    }
  }
}

template <typename T, int N, int MP, bool BAT = false>
__global__ __launch_bounds__((plane_threads<T, N>())) void k_plane_local_density(
    PlaneLocalDensityArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (plane_local_density_block<T, N, MP>(a_.sin, a_.sout, a_.vloc, a_.ur, a_.bandw,
                                                  a_.dpart, a_.nb, a_.gsize, a_.a, a_.tw1, a_.tw2,
                                                  a_.st, vb)));
}

// sticks -> real-space plane (set-up: valence orbitals in real space)
template <typename T>
struct PlaneToRealArgs {
  const cplx<T>* sin;
  cplx<T>* rout;
  PlaneArgs a;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
};

template <typename T, int N, int MP>
__device__ __forceinline__ void plane_to_real_block(const cplx<T>* __restrict__ sin,
                                                    cplx<T>* __restrict__ rout, const PlaneArgs& a,
                                                    const cplx<T>* __restrict__ tw1,
                                                    const cplx<T>* __restrict__ tw2,
                                                    const VBlock& vb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  constexpr int NTB = N > 0 ? plane_threads<T, N>() : 256;
  PlaneShm<T, N> sh(smem_raw, a, tw1, tid);
  const int n1 = N > 0 ? N : a.n1, n2 = N > 0 ? N : a.n2, n3 = N > 0 ? N : a.n3;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  const int z = vb.x, b = vb.y;
  const int np = n1 * n2;
  plane_zero_scatter<T, N>(sh, a, sin + ((int64_t)b * n3 + z) * a.S, tid);
  plane_rows<T, N, MP, +1>(sh, a, a.nact, true, tw2, tid);
  plane_cols<T, N, MP, +1>(sh, a, tw1, tid);
  cplx<T>* ro = rout + ((int64_t)b * n3 + z) * np;
  for (int p = tid; p < np; p += NTB) {
    const int i1 = p / n2, i2 = p - i1 * n2;
    ro[p] = sh.plane[i1 * pitch + i2];
  }
}

template <typename T, int N, int MP, bool BAT = false>
__global__ __launch_bounds__((plane_threads<T, N>())) void k_plane_to_real(PlaneToRealArgs<T> p,
                                                                      BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (plane_to_real_block<T, N, MP>(a_.sin, a_.rout, a_.a, a_.tw1, a_.tw2, vb)));
}

// v'(r) u_b(r) -> FFT2 -> added to the sticks of the same band
template <typename T>
struct PlaneVuArgs {
  const cplx<T>* ur;
  const cplx<T>* vp;
  cplx<T>* sout;
  PlaneArgs a;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
  const LzDevState* st;
};

template <typename T, int N, int MP>
__device__ __forceinline__ void plane_vu_block(const cplx<T>* __restrict__ ur,
                                               const cplx<T>* __restrict__ vp,
                                               cplx<T>* __restrict__ sout, const PlaneArgs& a,
                                               const cplx<T>* __restrict__ tw1,
                                               const cplx<T>* __restrict__ tw2,
                                               const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  constexpr int NTB = N > 0 ? plane_threads<T, N>() : 256;
  PlaneShm<T, N> sh(smem_raw, a, tw1, tid);
  const int n1 = N > 0 ? N : a.n1, n2 = N > 0 ? N : a.n2, n3 = N > 0 ? N : a.n3;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  const int z = vb.x, b = vb.y;
  const int np = n1 * n2;
  const cplx<T>* ub = ur + ((int64_t)b * n3 + z) * np;
  const cplx<T>* vz = vp + (int64_t)z * np;
  for (int p = tid; p < np; p += NTB) {
    const int i1 = p / n2, i2 = p - i1 * n2;
    sh.plane[i1 * pitch + i2] = cmul<T>(ub[p], vz[p]);
  }
  __syncthreads();
  plane_cols<T, N, MP, -1>(sh, a, tw1, tid);
  plane_rows<T, N, MP, -1>(sh, a, a.nact, true, tw2, tid);
  const int64_t so = ((int64_t)b * n3 + z) * a.S;
  for (int s = tid; s < a.S; s += NTB) {
    const cplx<T> v = sh.plane[a.si1[s] * pitch + a.si2[s]];
    sout[so + s] = cadd<T>(sout[so + s], v);
  }
}

template <typename T, int N, int MP, bool BAT = false>
__global__ __launch_bounds__((plane_threads<T, N>())) void k_plane_vu(PlaneVuArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (plane_vu_block<T, N, MP>(a_.ur, a_.vp, a_.sout, a_.a, a_.tw1, a_.tw2, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// response Hartree + xc potential of one instance
// ---------------------------------------------------------------------------
// (1) n'(r) = sum over band groups (fixed order); 2-D forward transform
template <typename T>
struct HxcPlanesFwdArgs {
  const cplx<T>* dpart;
  int ngroups;
  cplx<T>* nr;
  cplx<T>* work;
  PlaneArgs a;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
  const LzDevState* st;
};

template <typename T, int N, int MP>
__device__ __forceinline__ void hxc_planes_fwd_block(const cplx<T>* __restrict__ dpart, int ngroups,
                                                     cplx<T>* __restrict__ nr,
                                                     cplx<T>* __restrict__ work, const PlaneArgs& a,
                                                     const cplx<T>* __restrict__ tw1,
                                                     const cplx<T>* __restrict__ tw2,
                                                     const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  constexpr int NTB = N > 0 ? plane_threads<T, N>() : 256;
  PlaneShm<T, N> sh(smem_raw, a, tw1, tid);
  const int n1 = N > 0 ? N : a.n1, n2 = N > 0 ? N : a.n2, n3 = N > 0 ? N : a.n3;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  const int z = vb.x;
  const int np = n1 * n2;
  const int64_t plane = (int64_t)n3 * np;
  for (int p = tid; p < np; p += NTB) {
    cplx<T> s = czero<T>();
#pragma unroll 8
    for (int g = 0; g < ngroups; ++g) s = cadd<T>(s, dpart[g * plane + (int64_t)z * np + p]);
    nr[(int64_t)z * np + p] = s;
    const int i1 = p / n2, i2 = p - i1 * n2;
    sh.plane[i1 * pitch + i2] = s;
  }
  __syncthreads();
  plane_cols<T, N, MP, -1>(sh, a, tw1, tid);
  plane_rows<T, N, MP, -1>(sh, a, n1, false, tw2, tid);
  for (int p = tid; p < np; p += NTB) {
    const int i1 = p / n2, i2 = p - i1 * n2;
    work[(int64_t)z * np + p] = sh.plane[i1 * pitch + i2];
  }
}

template <typename T, int N, int MP, bool BAT = false>
__global__ __launch_bounds__((plane_threads<T, N>())) void k_hxc_planes_fwd(HxcPlanesFwdArgs<T> p,
                                                                       BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (hxc_planes_fwd_block<T, N, MP>(a_.dpart, a_.ngroups, a_.nr, a_.work, a_.a, a_.tw1,
                                             a_.tw2, a_.st, vb)));
}

// (2) along z: forward, times 4 pi / (|q+G|^2 N), inverse
template <typename T>
struct HxcZArgs {
  cplx<T>* work;
  const T* khart;
  int np;
  int n3_rt;
  FftPlan pz;
  const cplx<T>* twg;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void hxc_z_block(cplx<T>* __restrict__ work, const T* __restrict__ khart,
                                            int np, int n3_rt, const FftPlan& pz,
                                            const cplx<T>* __restrict__ twg, const LzDevState* st,
                                            const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n3 = N > 0 ? N : n3_rt;
  const int c0 = vb.x * kColTile;
  const int nc = min(kColTile, np - c0);
  const int pitch = n3 + 1;
  const int tid = threadIdx.x;
  const cplx<T>* tw = stick_tw<T, N>(lds, twg, tid);
  for (int t = tid; t < nc * n3; t += 256) {
    const int z = t / nc, c = t - z * nc;
    lds[c * pitch + z] = work[(int64_t)z * np + c0 + c];
  }
  __syncthreads();
  stick_fft<T, N>(lds, pitch, pz, nc, tw, tid, -1);
  for (int t = tid; t < nc * n3; t += 256) {
    const int z = t / nc, c = t - z * nc;
    cplx<T>& v = lds[c * pitch + z];
    v = cscale<T>(v, khart[(int64_t)z * np + c0 + c]);
  }
  __syncthreads();
  stick_fft<T, N>(lds, pitch, pz, nc, tw, tid, +1);
  for (int t = tid; t < nc * n3; t += 256) {
    const int z = t / nc, c = t - z * nc;
    work[(int64_t)z * np + c0 + c] = lds[c * pitch + z];
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(256) void k_hxc_z(HxcZArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (hxc_z_block<T, N>(a_.work, a_.khart, a_.np, a_.n3_rt, a_.pz, a_.twg, a_.st, vb)));
}

// (3) 2-D inverse transform, v'(r) = v_H(r) + f_xc(r) n'(r)
template <typename T>
struct HxcPlanesInvArgs {
  const cplx<T>* work;
  const cplx<T>* nr;
  const T* fxc;
  int with_fxc;
  cplx<T>* vp;
  PlaneArgs a;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
  const LzDevState* st;
};

template <typename T, int N, int MP>
__device__ __forceinline__ void hxc_planes_inv_block(const cplx<T>* __restrict__ work,
                                                     const cplx<T>* __restrict__ nr,
                                                     const T* __restrict__ fxc, int with_fxc,
                                                     cplx<T>* __restrict__ vp, const PlaneArgs& a,
                                                     const cplx<T>* __restrict__ tw1,
                                                     const cplx<T>* __restrict__ tw2,
                                                     const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  constexpr int NTB = N > 0 ? plane_threads<T, N>() : 256;
  PlaneShm<T, N> sh(smem_raw, a, tw1, tid);
  const int n1 = N > 0 ? N : a.n1, n2 = N > 0 ? N : a.n2;
  const int pitch = N > 0 ? ct_plane_pitch<N>() : a.pitch;
  const int z = vb.x;
  const int np = n1 * n2;
  for (int p = tid; p < np; p += NTB) {
    const int i1 = p / n2, i2 = p - i1 * n2;
    sh.plane[i1 * pitch + i2] = work[(int64_t)z * np + p];
  }
  __syncthreads();
  plane_rows<T, N, MP, +1>(sh, a, n1, false, tw2, tid);
  plane_cols<T, N, MP, +1>(sh, a, tw1, tid);
  for (int p = tid; p < np; p += NTB) {
    const int i1 = p / n2, i2 = p - i1 * n2;
    cplx<T> v = sh.plane[i1 * pitch + i2];
    if (with_fxc) {
      const cplx<T> n = nr[(int64_t)z * np + p];
      const T f = fxc[(int64_t)z * np + p];
      v.x += f * n.x;
      v.y += f * n.y;
    }
    vp[(int64_t)z * np + p] = v;
  }
}

template <typename T, int N, int MP, bool BAT = false>
__global__ __launch_bounds__((plane_threads<T, N>())) void k_hxc_planes_inv(HxcPlanesInvArgs<T> p,
                                                                       BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (hxc_planes_inv_block<T, N, MP>(a_.work, a_.nr, a_.fxc, a_.with_fxc, a_.vp, a_.a,
                                             a_.tw1, a_.tw2, a_.st, vb)));
}

// ---------------------------------------------------------------------------
// response potential on compile-time grids: the 3-D transform of the single
// density grid runs as line passes of kLineTile lines per block (N^2/8
// blocks per pass instead of N plane blocks), i2 and i1 here, z in k_hxc_z.
// ---------------------------------------------------------------------------
constexpr int kLineTile = 8;
constexpr int kSumBatch = 16;  // group partials per round of loads in the first line pass

// n'(r) = sum over band groups (fixed order); forward transform along i2
template <typename T>
struct HxcL2FwdArgs {
  const cplx<T>* dpart;
  int ngroups;
  cplx<T>* nr;
  cplx<T>* work;
  const cplx<T>* twg;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void hxc_l2_fwd_block(const cplx<T>* __restrict__ dpart, int ngroups,
                                                 cplx<T>* __restrict__ nr,
                                                 cplx<T>* __restrict__ work,
                                                 const cplx<T>* __restrict__ twg,
                                                 const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  constexpr int P = N + 1;
  constexpr int64_t NG = (int64_t)N * N * N;
  const int tid = threadIdx.x;
  const cplx<T>* tw = stick_tw<T, N>(lds, twg, tid);
  const int64_t l0 = (int64_t)vb.x * kLineTile;
  // a thread's elements (at most EPT) summed over the groups in order, the
  // loads of kSumBatch groups of every element in flight together
  constexpr int EPT = (kLineTile * N + 255) / 256;
  cplx<T> v[EPT];
  int64_t idx[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    v[e] = czero<T>();
    const int t = tid + e * 256;
    idx[e] = t < kLineTile * N ? l0 * N + t : -1;
  }
  for (int g0 = 0; g0 < ngroups; g0 += kSumBatch) {
    cplx<T> u[EPT][kSumBatch];
#pragma unroll
    for (int e = 0; e < EPT; ++e)
#pragma unroll
      for (int j = 0; j < kSumBatch; ++j)
        u[e][j] = idx[e] >= 0 && g0 + j < ngroups ? dpart[(g0 + j) * NG + idx[e]] : czero<T>();
#pragma unroll
    for (int e = 0; e < EPT; ++e)
#pragma unroll
      for (int j = 0; j < kSumBatch; ++j)
        if (g0 + j < ngroups) v[e] = cadd<T>(v[e], u[e][j]);
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    if (idx[e] >= 0) {
      const int t = tid + e * 256;
      nr[idx[e]] = v[e];
      lds[(t / N) * P + t % N] = v[e];
    }
  }
  __syncthreads();
  ct_fft<T, N, -1, kStickTile>(lds, LayRowsAll<P>{}, kLineTile, tw, tid);
  for (int t = tid; t < kLineTile * N; t += 256) {
    const int ll = t / N, i = t - ll * N;
    work[(l0 + ll) * N + i] = lds[ll * P + i];
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(256) void k_hxc_l2_fwd(HxcL2FwdArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (hxc_l2_fwd_block<T, N>(a_.dpart, a_.ngroups, a_.nr, a_.work, a_.twg, a_.st, vb)));
}

// transform along i1 (lines (z, i2), stride N), in place
template <typename T>
struct HxcL1Args {
  cplx<T>* work;
  const cplx<T>* twg;
  const LzDevState* st;
};

template <typename T, int N, int DIR>
__device__ __forceinline__ void hxc_l1_block(cplx<T>* __restrict__ work,
                                             const cplx<T>* __restrict__ twg, const LzDevState* st,
                                             const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  constexpr int P = N + 1;
  constexpr int TPZ = N / kLineTile;
  const int tid = threadIdx.x;
  const cplx<T>* tw = stick_tw<T, N>(lds, twg, tid);
  const int z = vb.x / TPZ;
  const int i20 = (vb.x - z * TPZ) * kLineTile;
  cplx<T>* base = work + (int64_t)z * N * N + i20;
  for (int t = tid; t < kLineTile * N; t += 256) {
    const int i1 = t / kLineTile, ll = t - i1 * kLineTile;
    lds[ll * P + i1] = base[i1 * N + ll];
  }
  __syncthreads();
  ct_fft<T, N, DIR, kStickTile>(lds, LayRowsAll<P>{}, kLineTile, tw, tid);
  for (int t = tid; t < kLineTile * N; t += 256) {
    const int i1 = t / kLineTile, ll = t - i1 * kLineTile;
    base[i1 * N + ll] = lds[ll * P + i1];
  }
}

template <typename T, int N, int DIR, bool BAT = false>
__global__ __launch_bounds__(256) void k_hxc_l1(HxcL1Args<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br, (hxc_l1_block<T, N, DIR>(a_.work, a_.twg, a_.st, vb)));
}

// inverse along i2, then v'(r) = v_H(r) + f_xc(r) n'(r)
template <typename T>
struct HxcL2InvArgs {
  const cplx<T>* work;
  const cplx<T>* nr;
  const T* fxc;
  int with_fxc;
  cplx<T>* vp;
  const cplx<T>* twg;
  const LzDevState* st;
};

template <typename T, int N>
__device__ __forceinline__ void hxc_l2_inv_block(const cplx<T>* __restrict__ work,
                                                 const cplx<T>* __restrict__ nr,
                                                 const T* __restrict__ fxc, int with_fxc,
                                                 cplx<T>* __restrict__ vp,
                                                 const cplx<T>* __restrict__ twg,
                                                 const LzDevState* st, const VBlock& vb) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  constexpr int P = N + 1;
  const int tid = threadIdx.x;
  const cplx<T>* tw = stick_tw<T, N>(lds, twg, tid);
  const int64_t l0 = (int64_t)vb.x * kLineTile;
  for (int t = tid; t < kLineTile * N; t += 256) {
    const int ll = t / N, i = t - ll * N;
    lds[ll * P + i] = work[(l0 + ll) * N + i];
  }
  __syncthreads();
  ct_fft<T, N, +1, kStickTile>(lds, LayRowsAll<P>{}, kLineTile, tw, tid);
  for (int t = tid; t < kLineTile * N; t += 256) {
    const int ll = t / N, i = t - ll * N;
    const int64_t idx = (l0 + ll) * N + i;
    cplx<T> v = lds[ll * P + i];
    if (with_fxc) {
      const cplx<T> n = nr[idx];
      const T f = fxc[idx];
      v.x += f * n.x;
      v.y += f * n.y;
    }
    vp[idx] = v;
  }
}

template <typename T, int N, bool BAT = false>
__global__ __launch_bounds__(256) void k_hxc_l2_inv(HxcL2InvArgs<T> p, BatchRef br) {
  LZ_BATCHED(BAT, p, br,
             (hxc_l2_inv_block<T, N>(a_.work, a_.nr, a_.fxc, a_.with_fxc, a_.vp, a_.twg, a_.st,
                                     vb)));
}

template <typename T, int N>
static void hxc_lines(const Grid3& g, const void* dpart, int ngroups, void* nr, void* work,
                      const void* khart, const void* fxc, bool with_fxc, void* vp,
                      const LzDevState* st, hipStream_t s) {
  const int nlb = N * N / kLineTile;
  const size_t ll = (size_t)(kStickTile * (N + 1) + ct_twsize(N)) * sizeof(cplx<T>);
  const cplx<T>* tw = (const cplx<T>*)g.tw1;
  lz_launch((k_hxc_l2_fwd<T, N>), (k_hxc_l2_fwd<T, N, true>), dim3(nlb), dim3(256), ll, s,
            (const cplx<T>*)dpart,
                     ngroups, (cplx<T>*)nr, (cplx<T>*)work, tw, st);
  lz_launch((k_hxc_l1<T, N, -1>), (k_hxc_l1<T, N, -1, true>), dim3(nlb), dim3(256), ll, s,
            (cplx<T>*)work, tw, st);
  lz_launch((k_hxc_z<T, N>), (k_hxc_z<T, N, true>), dim3(N * N / kColTile), dim3(256), ll, s,
            (cplx<T>*)work,
                     (const T*)khart, N * N, N, g.p3, tw, st);
  lz_launch((k_hxc_l1<T, N, +1>), (k_hxc_l1<T, N, +1, true>), dim3(nlb), dim3(256), ll, s,
            (cplx<T>*)work, tw, st);
  lz_launch((k_hxc_l2_inv<T, N>), (k_hxc_l2_inv<T, N, true>), dim3(nlb), dim3(256), ll, s,
            (const cplx<T>*)work,
                     (const cplx<T>*)nr, (const T*)fxc, with_fxc ? 1 : 0, (cplx<T>*)vp, tw, st);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline PlaneArgs plane_args(const Grid3& g) {
  PlaneArgs a;
  a.n1 = g.n1; a.n2 = g.n2; a.n3 = g.n3; a.S = g.S; a.nact = g.nact; a.pitch = g.pitch2;
  a.si1 = g.si1; a.si2 = g.si2; a.act = g.act; a.p1 = g.p1; a.p2 = g.p2;
  return a;
}

// compile-time size of a grid (0 = general form)
static inline int ct_size(const Grid3& g) {
  return (g.n1 == g.n2 && g.n2 == g.n3 && ct_supported(g.n1)) ? g.n1 : 0;
}

// plane length n of a register-line or lane-pair kernel in precision T
// (0 = none: the LDS passes serve such planes)
template <typename T>
int reg_plane_len(int n) {
  switch (n) {
    case 24: return reg_plane_ok<T, 24>() ? 24 : 0;
    case 32: return reg_plane_ok<T, 32>() ? 32 : 0;
    case 48: return reg_plane_ok<T, 48>() ? 48 : 0;
    case 64: return reg_pair_ok<T>() ? 64 : 0;
    case 72: return reg_pair_ok<T>() ? 72 : 0;
    case 96: return reg_pair_ok<T>() ? 96 : 0;
    default: return 0;
  }
}
template int reg_plane_len<double>(int);
template int reg_plane_len<float>(int);

// size N of the register-line plane kernels for this grid (0 = not used)
template <typename T>
int reg_plane_size(const Grid3& g) {
  if (!g.soff_f || g.lds_planes) return 0;
  return reg_plane_len<T>(ct_size(g));
}
template int reg_plane_size<double>(const Grid3&);
template int reg_plane_size<float>(const Grid3&);


static inline RegPlaneArgs reg_args(const Grid3& g) {
  RegPlaneArgs a;
  a.S = g.S;
  a.nact = g.nact;
  a.soff = g.soff_f;
  a.soffc = g.soff_c;
  a.act = g.act;
  for (int i = 0; i < 128; ++i) a.slot[i] = g.slot[i];
  return a;
}

#define LZ_REG_LAUNCH(KERN, T, N, GRID, LDS, STREAM, ...)                                      \
  do {                                                                                         \
    if constexpr (reg_plane_ok<T, 48>()) {                                                     \
      switch (N) {                                                                             \
        case 24: lz_launch((KERN<T, 24>), (KERN<T, 24, true>), GRID, dim3(kRegPlaneThreads), LDS, STREAM, __VA_ARGS__); break; \
        case 32: lz_launch((KERN<T, 32>), (KERN<T, 32, true>), GRID, dim3(kRegPlaneThreads), LDS, STREAM, __VA_ARGS__); break; \
        case 48: lz_launch((KERN<T, 48>), (KERN<T, 48, true>), GRID, dim3(kRegPlaneThreads), LDS, STREAM, __VA_ARGS__); break; \
        default: throw std::logic_error("no line-per-thread plane kernel for this size");                        \
      }                                                                                        \
    }                                                                                          \
  } while (0)

template <typename T> static size_t plane_lds(const Grid3& g) {
  const int n = ct_size(g);
  switch (n) {
#define LZ_CASE(N) case N: return plane_shm_bytes_ct<T, N>();
    LZ_CT_SIZES(LZ_CASE)
#undef LZ_CASE
    default: return (size_t)g.n1 * g.pitch2 * sizeof(cplx<T>);
  }
}
template <typename T> static size_t stick_lds(const Grid3& g) {
  const int n = ct_size(g);
  return (size_t)(zpass_tile(n) * (g.n3 + 1) + (n ? ct_twsize(n) : 0)) * sizeof(cplx<T>);
}

// dispatch a plane kernel on (N, MP)
#define LZ_PLANE_LAUNCH(KERN, T, G, GRID, LDS, STREAM, ...)                                     \
  do {                                                                                          \
    switch (ct_size(G)) {                                                                       \
      case 24: lz_launch((KERN<T, 24, 0>), (KERN<T, 24, 0, true>), GRID, dim3(plane_threads<T, 24>()), LDS, STREAM, __VA_ARGS__); break; \
      case 32: lz_launch((KERN<T, 32, 0>), (KERN<T, 32, 0, true>), GRID, dim3(plane_threads<T, 32>()), LDS, STREAM, __VA_ARGS__); break; \
      case 40: lz_launch((KERN<T, 40, 0>), (KERN<T, 40, 0, true>), GRID, dim3(plane_threads<T, 40>()), LDS, STREAM, __VA_ARGS__); break; \
      case 48: lz_launch((KERN<T, 48, 0>), (KERN<T, 48, 0, true>), GRID, dim3(plane_threads<T, 48>()), LDS, STREAM, __VA_ARGS__); break; \
      case 64: lz_launch((KERN<T, 64, 0>), (KERN<T, 64, 0, true>), GRID, dim3(plane_threads<T, 64>()), LDS, STREAM, __VA_ARGS__); break; \
      case 72: lz_launch((KERN<T, 72, 0>), (KERN<T, 72, 0, true>), GRID, dim3(plane_threads<T, 72>()), LDS, STREAM, __VA_ARGS__); break; \
      case 96: lz_launch((KERN<T, 96, 0>), (KERN<T, 96, 0, true>), GRID, dim3(plane_threads<T, 96>()), LDS, STREAM, __VA_ARGS__); break; \
      default:                                                                                  \
        switch (plane_mp((G).n1, (G).n2)) {                                                     \
          case 12: lz_launch((KERN<T, 0, 12>), (KERN<T, 0, 12, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
          case 24: lz_launch((KERN<T, 0, 24>), (KERN<T, 0, 24, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
          default: lz_launch((KERN<T, 0, 36>), (KERN<T, 0, 36, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
        }                                                                                       \
    }                                                                                           \
  } while (0)

#define LZ_STICK_LAUNCH(KERN, T, G, GRID, LDS, STREAM, ...)                                   \
  do {                                                                                        \
    switch (ct_size(G)) {                                                                     \
      case 24: lz_launch((KERN<T, 24>), (KERN<T, 24, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 32: lz_launch((KERN<T, 32>), (KERN<T, 32, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 40: lz_launch((KERN<T, 40>), (KERN<T, 40, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 48: lz_launch((KERN<T, 48>), (KERN<T, 48, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 64: lz_launch((KERN<T, 64>), (KERN<T, 64, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 72: lz_launch((KERN<T, 72>), (KERN<T, 72, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 96: lz_launch((KERN<T, 96>), (KERN<T, 96, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      default: lz_launch((KERN<T, 0>), (KERN<T, 0, true>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
    }                                                                                         \
  } while (0)

template <typename T>
void LaunchFft<T>::zfft_inv(const Grid3& g, const void* x, int64_t xs, void* sticks,
                            const int* map, int nb, int nbnd, const LzDevState* st, hipStream_t s) {
  const int n = ct_size(g), tile = zpass_tile(n);
  // compile-time grids: a block per tile and pair of bands of one k-point
  const int nks = nb / nbnd;
  dim3 grid((g.S + tile - 1) / tile, n ? nks * ((nbnd + 1) / 2) : nb);
  const size_t lds = n ? (size_t)(2 * tile * (g.n3 + 1) + ct_twsize(n)) * sizeof(cplx<T>)
                       : stick_lds<T>(g);
  LZ_STICK_LAUNCH(k_zfft_inv, T, g, grid, lds, s, (const cplx<T>*)x, xs,
                  (cplx<T>*)sticks, map, g.S, g.n3, nbnd, g.p3, (const cplx<T>*)g.tw3, st);
}

template <typename T>
void LaunchFft<T>::zfft_fwd(const Grid3& g, const void* sticks, const void* x, int64_t xs, void* y,
                            const int* map, const void* kin, const double* eps, int nb, int nbnd,
                            int npwx, const LzDevState* st, hipStream_t s) {
  const T scale = T(1.0 / ((double)g.n1 * g.n2 * g.n3));
  const int tile = zpass_tile(ct_size(g));
  dim3 grid((g.S + tile - 1) / tile, nb);
  LZ_STICK_LAUNCH(k_zfft_fwd, T, g, grid, stick_lds<T>(g), s, (const cplx<T>*)sticks,
                  (const cplx<T>*)x, xs, (cplx<T>*)y, map, (const T*)kin, eps, g.S, g.n3, nbnd,
                  npwx, scale, g.p3, (const cplx<T>*)g.tw3, st);
}

template <typename T>
void LaunchFft<T>::plane_local(const Grid3& g, const void* sin, void* sout, const void* vloc,
                               int nb, const LzDevState* st, hipStream_t s) {
  if (const int n = reg_plane_size<T>(g)) {
    const int npb = n >= 64 ? 1 : kRegPlaneThreads / n, nplanes = nb * n;
    const size_t lds = (size_t)npb * (g.nact + 1) * (n + 1) * sizeof(cplx<T>);  // compact planes
    if constexpr (reg_pair_ok<T>()) {
      if (n >= 64) {
        if (n == 64)
          lz_launch((k_rp_local<T, 64>), (k_rp_local<T, 64, true>), dim3(nplanes),
                    dim3(kRegPlaneThreads),
                             (pair_lds<T, 64>(g.nact)), s, (const cplx<T>*)sin, (cplx<T>*)sout,
                             (const T*)vloc, reg_args(g), st);
        else if (n == 72)
          lz_launch((k_rp_local<T, 72>), (k_rp_local<T, 72, true>), dim3(nplanes),
                    dim3(kRegPlaneThreads),
                             (pair_lds<T, 72>(g.nact)), s, (const cplx<T>*)sin, (cplx<T>*)sout,
                             (const T*)vloc, reg_args(g), st);
        else
          lz_launch((k_rp_local<T, 96>), (k_rp_local<T, 96, true>), dim3(nplanes),
                    dim3(kRegPlaneThreads),
                             (pair_lds<T, 96>(g.nact)), s, (const cplx<T>*)sin, (cplx<T>*)sout,
                             (const T*)vloc, reg_args(g), st);
        return;
      }
    }
    LZ_REG_LAUNCH(k_rl_local, T, n, dim3((nplanes + npb - 1) / npb), lds, s, (const cplx<T>*)sin,
                  (cplx<T>*)sout, (const T*)vloc, reg_args(g), nplanes, st);
    return;
  }
  LZ_PLANE_LAUNCH(k_plane_local, T, g, dim3(g.n3, nb), plane_lds<T>(g), s, (const cplx<T>*)sin,
                  (cplx<T>*)sout, (const T*)vloc, plane_args(g), (const cplx<T>*)g.tw1,
                  (const cplx<T>*)g.tw2, st);
}

template <typename T>
void LaunchFft<T>::plane_local_density(const Grid3& g, const void* sin, void* sout,
                                       const void* vloc, const void* ur, const double* bandw,
                                       void* dpart, int nb, int gsize, const LzDevState* st,
                                       hipStream_t s) {
  const int ng = (nb + gsize - 1) / gsize;
  if (const int n = reg_plane_size<T>(g)) {
    if constexpr (reg_pair_ok<T>()) {
      if (n >= 64) {
        if (n == 64)
          lz_launch((k_rp_density<T, 64>), (k_rp_density<T, 64, true>), dim3(g.n3, ng),
                    dim3(kRegPlaneThreads),
                             (pair_lds<T, 64>(g.nact)), s, (const cplx<T>*)sin, (cplx<T>*)sout,
                             (const T*)vloc, (const cplx<T>*)ur, bandw, (cplx<T>*)dpart, nb,
                             gsize, reg_args(g), st);
        else if (n == 72)
          lz_launch((k_rp_density<T, 72>), (k_rp_density<T, 72, true>), dim3(g.n3, ng),
                    dim3(kRegPlaneThreads),
                             (pair_lds<T, 72>(g.nact)), s, (const cplx<T>*)sin, (cplx<T>*)sout,
                             (const T*)vloc, (const cplx<T>*)ur, bandw, (cplx<T>*)dpart, nb,
                             gsize, reg_args(g), st);
        else
          lz_launch((k_rp_density<T, 96>), (k_rp_density<T, 96, true>), dim3(g.n3, ng),
                    dim3(kRegPlaneThreads),
                             (pair_lds<T, 96>(g.nact)), s, (const cplx<T>*)sin, (cplx<T>*)sout,
                             (const T*)vloc, (const cplx<T>*)ur, bandw, (cplx<T>*)dpart, nb,
                             gsize, reg_args(g), st);
        return;
      }
    }
    if constexpr (reg_plane_ok<T, 48>()) {
      if (n == 48 && gsize <= 4) {  // one band per lane of a quad
        const size_t lds = (size_t)4 * (g.nact + 1) * 49 * sizeof(cplx<T>);  // compact planes
        lz_launch((k_rq_density<T, 48>), (k_rq_density<T, 48, true>), dim3(g.n3, ng),
                  dim3(kRegPlaneThreads), lds, s,
                           (const cplx<T>*)sin,
                           (cplx<T>*)sout, (const T*)vloc, (const cplx<T>*)ur, bandw,
                           (cplx<T>*)dpart, nb, gsize, reg_args(g), st);
        return;
      }
    }
    const int npb = kRegPlaneThreads / n;
    const size_t lds = (size_t)npb * n * (n + 1) * sizeof(cplx<T>);
    LZ_REG_LAUNCH(k_rl_density, T, n, dim3(g.n3, ng), lds, s, (const cplx<T>*)sin,
                  (cplx<T>*)sout, (const T*)vloc, (const cplx<T>*)ur, bandw, (cplx<T>*)dpart, nb,
                  gsize, reg_args(g), st);
    return;
  }
  LZ_PLANE_LAUNCH(k_plane_local_density, T, g, dim3(g.n3, ng), plane_lds<T>(g), s,
                  (const cplx<T>*)sin, (cplx<T>*)sout, (const T*)vloc, (const cplx<T>*)ur, bandw,
                  (cplx<T>*)dpart, nb, gsize, plane_args(g), (const cplx<T>*)g.tw1,
                  (const cplx<T>*)g.tw2, st);
}

template <typename T>
int LaunchFft<T>::density_blocks_per_cu(const Grid3& g) {
  if (reg_plane_size<T>(g) != 0) return 0;
  const void* f = nullptr;
  int threads = 256;
  switch (ct_size(g)) {
#define LZ_CASE(N)                                              \
  case N:                                                       \
    f = reinterpret_cast<const void*>(k_plane_local_density<T, N, 0>); \
    threads = plane_threads<T, N>();                               \
    break;
    LZ_CT_SIZES(LZ_CASE)
#undef LZ_CASE
    default: return 0;
  }
  int nbpc = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nbpc, f, threads, plane_lds<T>(g)) !=
      hipSuccess)
    return 0;
  return nbpc;
}

template <typename T>
void LaunchFft<T>::plane_to_real(const Grid3& g, const void* sin, void* rout, int nb,
                                 hipStream_t s) {
  LZ_PLANE_LAUNCH(k_plane_to_real, T, g, dim3(g.n3, nb), plane_lds<T>(g), s, (const cplx<T>*)sin,
                  (cplx<T>*)rout, plane_args(g), (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2);
}

template <typename T>
void LaunchFft<T>::plane_vu(const Grid3& g, const void* ur, const void* vp, void* sout, int nb,
                            const LzDevState* st, hipStream_t s) {
  if constexpr (rp_ok<T, 48>()) {
    // double precision on 48^2 planes: lane pairs (77.5 us against 86.9 for the
    // LDS pass on the 48^3 cell; the local and density passes stay on LDS,
    // where their lane-pair forms were slower: 125 and 377 us against 110 and
    // 164)
    if (ct_size(g) == 48 && g.soff_c && !g.lds_planes) {
      lz_launch((k_rp_vu<T, 48>), (k_rp_vu<T, 48, true>), dim3(nb * 48), dim3(rp_threads<T, 48>()),
                (size_t)(g.nact + 1) * 49 * sizeof(cplx<T>), s, (const cplx<T>*)ur,
                (const cplx<T>*)vp, (cplx<T>*)sout, reg_args(g), st);
      return;
    }
  }
  if (const int n = reg_plane_size<T>(g)) {
    const int npb = n >= 64 ? 1 : kRegPlaneThreads / n, nplanes = nb * n;
    const size_t lds = (size_t)npb * (g.nact + 1) * (n + 1) * sizeof(cplx<T>);  // compact planes
    if constexpr (reg_pair_ok<T>()) {
      if (n >= 64) {
        if (n == 64)
          lz_launch((k_rp_vu<T, 64>), (k_rp_vu<T, 64, true>), dim3(nplanes), dim3(kRegPlaneThreads),
                    lds, s,
                             (const cplx<T>*)ur, (const cplx<T>*)vp, (cplx<T>*)sout, reg_args(g),
                              st);
        else if (n == 72)
          lz_launch((k_rp_vu<T, 72>), (k_rp_vu<T, 72, true>), dim3(nplanes), dim3(kRegPlaneThreads),
                    lds, s,
                             (const cplx<T>*)ur, (const cplx<T>*)vp, (cplx<T>*)sout, reg_args(g),
                              st);
        else
          lz_launch((k_rp_vu<T, 96>), (k_rp_vu<T, 96, true>), dim3(nplanes), dim3(kRegPlaneThreads),
                    lds, s,
                             (const cplx<T>*)ur, (const cplx<T>*)vp, (cplx<T>*)sout, reg_args(g),
                              st);
        return;
      }
    }
    LZ_REG_LAUNCH(k_rl_vu, T, n, dim3((nplanes + npb - 1) / npb), lds, s, (const cplx<T>*)ur,
                  (const cplx<T>*)vp, (cplx<T>*)sout, reg_args(g), nplanes, st);
    return;
  }
  LZ_PLANE_LAUNCH(k_plane_vu, T, g, dim3(g.n3, nb), plane_lds<T>(g), s, (const cplx<T>*)ur,
                  (const cplx<T>*)vp, (cplx<T>*)sout, plane_args(g), (const cplx<T>*)g.tw1,
                  (const cplx<T>*)g.tw2, st);
}

template <typename T>
void LaunchFft<T>::hxc(const Grid3& g, const void* dpart, int ngroups, void* nr, void* work,
                       const void* khart, const void* fxc, bool with_fxc, void* vp,
                       const LzDevState* st, hipStream_t s) {
  switch (ct_size(g)) {
    case 24: return hxc_lines<T, 24>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    case 32: return hxc_lines<T, 32>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    case 48: return hxc_lines<T, 48>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    case 64: return hxc_lines<T, 64>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    case 40: return hxc_lines<T, 40>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    case 72: return hxc_lines<T, 72>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    case 96: return hxc_lines<T, 96>(g, dpart, ngroups, nr, work, khart, fxc, with_fxc, vp, st, s);
    default: break;
  }
  const int np = g.n1 * g.n2;
  LZ_PLANE_LAUNCH(k_hxc_planes_fwd, T, g, dim3(g.n3), plane_lds<T>(g), s, (const cplx<T>*)dpart,
                  ngroups, (cplx<T>*)nr, (cplx<T>*)work, plane_args(g), (const cplx<T>*)g.tw1,
                  (const cplx<T>*)g.tw2, st);
  const size_t zl = (size_t)(kColTile * (g.n3 + 1) + (ct_size(g) ? ct_twsize(ct_size(g)) : 0)) *
                    sizeof(cplx<T>);
  LZ_STICK_LAUNCH(k_hxc_z, T, g, dim3((np + kColTile - 1) / kColTile), zl, s, (cplx<T>*)work,
                  (const T*)khart, np, g.n3, g.p3, (const cplx<T>*)g.tw3, st);
  LZ_PLANE_LAUNCH(k_hxc_planes_inv, T, g, dim3(g.n3), plane_lds<T>(g), s, (const cplx<T>*)work,
                  (const cplx<T>*)nr, (const T*)fxc, with_fxc ? 1 : 0, (cplx<T>*)vp,
                  plane_args(g), (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2, st);
}

// Kernels whose LDS may exceed the default dynamic limit opt in once (each
// kernel and its work-list twin).
template <typename T>
hipError_t enable_large_lds_fft() {
  std::vector<const void*> fns;
#define LZ_BOTH(...) \
  fns.push_back((const void*)__VA_ARGS__>); \
  fns.push_back((const void*)__VA_ARGS__, true>);
#define LZ_PLANE_KERNS(KERN)                                                   \
  LZ_BOTH(KERN<T, 0, 12) LZ_BOTH(KERN<T, 0, 24) LZ_BOTH(KERN<T, 0, 36)       \
  LZ_BOTH(KERN<T, 24, 0) LZ_BOTH(KERN<T, 32, 0) LZ_BOTH(KERN<T, 40, 0)       \
  LZ_BOTH(KERN<T, 48, 0) LZ_BOTH(KERN<T, 64, 0) LZ_BOTH(KERN<T, 72, 0)       \
  LZ_BOTH(KERN<T, 96, 0)
  LZ_PLANE_KERNS(k_plane_local)
  LZ_PLANE_KERNS(k_plane_local_density)
  LZ_PLANE_KERNS(k_plane_to_real)
  LZ_PLANE_KERNS(k_plane_vu)
  LZ_PLANE_KERNS(k_hxc_planes_fwd)
  LZ_PLANE_KERNS(k_hxc_planes_inv)
#undef LZ_PLANE_KERNS
#define LZ_STICK_KERNS(KERN)                                                   \
  LZ_BOTH(KERN<T, 24) LZ_BOTH(KERN<T, 32) LZ_BOTH(KERN<T, 40) LZ_BOTH(KERN<T, 48) \
  LZ_BOTH(KERN<T, 64) LZ_BOTH(KERN<T, 72) LZ_BOTH(KERN<T, 96)
  LZ_STICK_KERNS(k_zfft_inv)
  LZ_STICK_KERNS(k_zfft_fwd)
#undef LZ_STICK_KERNS
  if constexpr (reg_plane_ok<T, 48>()) {
    LZ_BOTH(k_rl_local<T, 24) LZ_BOTH(k_rl_local<T, 32) LZ_BOTH(k_rl_local<T, 48)
    LZ_BOTH(k_rl_density<T, 24) LZ_BOTH(k_rl_density<T, 32) LZ_BOTH(k_rl_density<T, 48)
    LZ_BOTH(k_rl_vu<T, 24) LZ_BOTH(k_rl_vu<T, 32) LZ_BOTH(k_rl_vu<T, 48)
    LZ_BOTH(k_rq_density<T, 48)
  }
  if constexpr (rp_ok<T, 48>()) {
    LZ_BOTH(k_rp_vu<T, 48)
  }
  if constexpr (reg_pair_ok<T>()) {
    LZ_BOTH(k_rp_local<T, 64) LZ_BOTH(k_rp_density<T, 64) LZ_BOTH(k_rp_vu<T, 64)
    LZ_BOTH(k_rp_local<T, 72) LZ_BOTH(k_rp_density<T, 72) LZ_BOTH(k_rp_vu<T, 72)
    LZ_BOTH(k_rp_local<T, 96) LZ_BOTH(k_rp_density<T, 96) LZ_BOTH(k_rp_vu<T, 96)
  }
#undef LZ_BOTH
  const int big = 160 * 1024;
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lz
