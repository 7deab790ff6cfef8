// Device kernels of the Liouvillian application, the Lanczos recursion and the
// spectrum (Secs. 2.3-2.5 of the turboEELS paper), written for gfx950.
//
// Data layouts (per instance):
//   sphere vectors   [k][band][npwx] complex, plane waves in stick-major order
//                    (sorted by stick, then by z index) so that one stick is a
//                    contiguous run;
//   sticks           [band][z][S] complex after the z-direction transform;
//   real-space grids plane-major [z][i1][i2].
// The 3-D transform of a band is split into a z pass over the sticks that
// touch the sphere (about a fifth of the N1*N2 columns) and a 2-D pass per
// z-plane held entirely in LDS, in which only rows carrying a stick are
// transformed along i2.  Every reduction runs in a fixed order, so repeated
// runs are bitwise identical.
#include "lz_kernels.h"

namespace lz {

// complex values per thread of a 256-thread plane pass
int plane_mp(int n1, int n2) {
  const int np = n1 * n2;
  if (np <= 12 * 256) return 12;
  if (np <= 24 * 256) return 24;
  return 36;
}

#define LZ_PLANE_LAUNCH(KERN, T, MPV, GRID, LDS, STREAM, ...)                              \
  do {                                                                                     \
    switch (MPV) {                                                                         \
      case 12: hipLaunchKernelGGL((KERN<T, 12>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      case 24: hipLaunchKernelGGL((KERN<T, 24>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL((KERN<T, 36>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__); break; \
    }                                                                                      \
  } while (0)

template <typename T>
__device__ __forceinline__ cplx<T> czero() { return mk<T>(T(0), T(0)); }

// ---------------------------------------------------------------------------
// z pass, inverse: sphere -> sticks
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_zfft_inv(const cplx<T>* __restrict__ x, int64_t xs, cplx<T>* __restrict__ out,
                           const int* __restrict__ map, int S, int n3, int nbnd, FftPlan pz,
                           const cplx<T>* __restrict__ tw, const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int b = blockIdx.y;
  const int k = b / nbnd;
  const int s0 = blockIdx.x * kStickTile;
  const int nst = min(kStickTile, S - s0);
  const int pitch = n3 + 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const cplx<T>* xb = x + b * xs;
  const int* mp = map + ((int64_t)k * S + s0) * n3;
  for (int t = tid; t < nst * n3; t += nthr) {
    const int ls = t / n3, z = t - ls * n3;
    const int idx = mp[ls * n3 + z];
    lds[ls * pitch + z] = idx >= 0 ? xb[idx] : czero<T>();
  }
  __syncthreads();
  fft_lds<T, kStickMaxPt, +1>(lds, Lay{1, pitch, nullptr}, pz, nst, tw, tid, nthr);
  cplx<T>* ob = out + (int64_t)b * n3 * S + s0;
  for (int t = tid; t < nst * n3; t += nthr) {
    const int z = t / nst, ls = t - z * nst;
    ob[(int64_t)z * S + ls] = lds[ls * pitch + z];
  }
}

// ---------------------------------------------------------------------------
// z pass, forward: sticks -> sphere; y = x_fft/N + (kin - eps) x
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_zfft_fwd(const cplx<T>* __restrict__ sticks, const cplx<T>* __restrict__ x,
                           int64_t xs, cplx<T>* __restrict__ y, const int* __restrict__ map,
                           const T* __restrict__ kin, const double* __restrict__ eps, int S,
                           int n3, int nbnd, int npwx, T scale, FftPlan pz,
                           const cplx<T>* __restrict__ tw, const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int b = blockIdx.y;
  const int k = b / nbnd;
  const int s0 = blockIdx.x * kStickTile;
  const int nst = min(kStickTile, S - s0);
  const int pitch = n3 + 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const cplx<T>* sb = sticks + (int64_t)b * n3 * S + s0;
  for (int t = tid; t < nst * n3; t += nthr) {
    const int z = t / nst, ls = t - z * nst;
    lds[ls * pitch + z] = sb[(int64_t)z * S + ls];
  }
  __syncthreads();
  fft_lds<T, kStickMaxPt, -1>(lds, Lay{1, pitch, nullptr}, pz, nst, tw, tid, nthr);
  const int* mp = map + ((int64_t)k * S + s0) * n3;
  const cplx<T>* xb = x + b * xs;
  cplx<T>* yb = y + b * xs;
  const T* kb = kin + (int64_t)k * npwx;
  const T e = T(eps[b]);
  for (int t = tid; t < nst * n3; t += nthr) {
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

// ---------------------------------------------------------------------------
// plane helpers
// ---------------------------------------------------------------------------
struct PlaneArgs {
  int n1, n2, n3, S, nact, pitch;
  const int* si1;
  const int* si2;
  const int* act;
  FftPlan p1, p2;
};

template <typename T>
__device__ __forceinline__ void plane_zero_scatter(cplx<T>* lds, const PlaneArgs& a,
                                                   const cplx<T>* __restrict__ src, int tid,
                                                   int nthr) {
  for (int t = tid; t < a.n1 * a.pitch; t += nthr) lds[t] = czero<T>();
  __syncthreads();
  for (int s = tid; s < a.S; s += nthr) lds[a.si1[s] * a.pitch + a.si2[s]] = src[s];
  __syncthreads();
}

template <typename T, int MP>
__device__ __forceinline__ void plane_inverse(cplx<T>* lds, const PlaneArgs& a,
                                              const cplx<T>* tw1, const cplx<T>* tw2, int tid,
                                              int nthr) {
  // along i2 on rows that carry sticks, then along i1 on every column
  fft_lds<T, MP, +1>(lds, Lay{1, a.pitch, a.act}, a.p2, a.nact, tw2, tid, nthr);
  fft_lds<T, MP, +1>(lds, Lay{a.pitch, 1, nullptr}, a.p1, a.n2, tw1, tid, nthr);
}

template <typename T, int MP>
__device__ __forceinline__ void plane_forward(cplx<T>* lds, const PlaneArgs& a,
                                              const cplx<T>* tw1, const cplx<T>* tw2, int tid,
                                              int nthr) {
  // along i1 on every column, then along i2 only on the rows that hold sticks
  fft_lds<T, MP, -1>(lds, Lay{a.pitch, 1, nullptr}, a.p1, a.n2, tw1, tid, nthr);
  fft_lds<T, MP, -1>(lds, Lay{1, a.pitch, a.act}, a.p2, a.nact, tw2, tid, nthr);
}

// ---------------------------------------------------------------------------
// plane pass of a D step: x(r) = IFFT2 sticks, (V x)(r), FFT2 -> sticks
// ---------------------------------------------------------------------------
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_plane_local(const cplx<T>* __restrict__ sin, cplx<T>* __restrict__ sout,
                              const T* __restrict__ vloc, PlaneArgs a,
                              const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                              const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int z = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t so = ((int64_t)b * a.n3 + z) * a.S;
  plane_zero_scatter<T>(lds, a, sin + so, tid, nthr);
  plane_inverse<T, MP>(lds, a, tw1, tw2, tid, nthr);
  const T* vz = vloc + (int64_t)z * a.n1 * a.n2;
  for (int p = tid; p < a.n1 * a.n2; p += nthr) {
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    cplx<T>& c = lds[i1 * a.pitch + i2];
    c = cscale<T>(c, vz[p]);
  }
  __syncthreads();
  plane_forward<T, MP>(lds, a, tw1, tw2, tid, nthr);
  for (int s = tid; s < a.S; s += nthr) sout[so + s] = lds[a.si1[s] * a.pitch + a.si2[s]];
}

// ---------------------------------------------------------------------------
// plane pass of a D+K step: as above for a group of bands, accumulating the
// response density  n'(r) += (4 w_k / Omega) conj(u_b(r)) x_b(r)  (raw values
// of u and x, i.e. without the Omega^-1/2 factors, which bandw absorbs).
// ---------------------------------------------------------------------------
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_plane_local_density(const cplx<T>* __restrict__ sin, cplx<T>* __restrict__ sout,
                                      const T* __restrict__ vloc, const cplx<T>* __restrict__ ur,
                                      const double* __restrict__ bandw,
                                      cplx<T>* __restrict__ dpart, int nb, int gsize, PlaneArgs a,
                                      const cplx<T>* __restrict__ tw1,
                                      const cplx<T>* __restrict__ tw2, const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int z = blockIdx.x, g = blockIdx.y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int np = a.n1 * a.n2;
  const T* vz = vloc + (int64_t)z * np;
  cplx<T> acc[MP];
#pragma unroll
  for (int i = 0; i < MP; ++i) acc[i] = czero<T>();
  const int b0 = g * gsize, b1 = min(nb, b0 + gsize);
  for (int b = b0; b < b1; ++b) {
    const int64_t so = ((int64_t)b * a.n3 + z) * a.S;
    plane_zero_scatter<T>(lds, a, sin + so, tid, nthr);
    plane_inverse<T, MP>(lds, a, tw1, tw2, tid, nthr);
    const cplx<T>* ub = ur + ((int64_t)b * a.n3 + z) * np;
    const T wb = T(bandw[b]);
#pragma unroll
    for (int i = 0; i < MP; ++i) {
      const int p = tid + i * nthr;
      if (p < np) {
        const int i1 = p / a.n2, i2 = p - i1 * a.n2;
        cplx<T>& c = lds[i1 * a.pitch + i2];
        const cplx<T> d = cmulc<T>(ub[p], c);
        acc[i].x += wb * d.x;
        acc[i].y += wb * d.y;
        c = cscale<T>(c, vz[p]);
      }
    }
    __syncthreads();
    plane_forward<T, MP>(lds, a, tw1, tw2, tid, nthr);
    for (int s = tid; s < a.S; s += nthr) sout[so + s] = lds[a.si1[s] * a.pitch + a.si2[s]];
    __syncthreads();
  }
  cplx<T>* dp = dpart + ((int64_t)g * a.n3 + z) * np;
#pragma unroll
  for (int i = 0; i < MP; ++i) {
    const int p = tid + i * nthr;
    if (p < np) dp[p] = acc[i];
  }
}

// sticks -> real-space plane (init: valence orbitals in real space)
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_plane_to_real(const cplx<T>* __restrict__ sin, cplx<T>* __restrict__ rout,
                                PlaneArgs a, const cplx<T>* __restrict__ tw1,
                                const cplx<T>* __restrict__ tw2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int z = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int np = a.n1 * a.n2;
  plane_zero_scatter<T>(lds, a, sin + ((int64_t)b * a.n3 + z) * a.S, tid, nthr);
  plane_inverse<T, MP>(lds, a, tw1, tw2, tid, nthr);
  cplx<T>* ro = rout + ((int64_t)b * a.n3 + z) * np;
  for (int p = tid; p < np; p += nthr) {
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    ro[p] = lds[i1 * a.pitch + i2];
  }
}

// v'(r) u_b(r) -> FFT2 -> added to the sticks of the same band
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_plane_vu(const cplx<T>* __restrict__ ur, const cplx<T>* __restrict__ vp,
                           cplx<T>* __restrict__ sout, PlaneArgs a,
                           const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                           const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int z = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int np = a.n1 * a.n2;
  const cplx<T>* ub = ur + ((int64_t)b * a.n3 + z) * np;
  const cplx<T>* vz = vp + (int64_t)z * np;
  for (int p = tid; p < np; p += nthr) {
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    lds[i1 * a.pitch + i2] = cmul<T>(ub[p], vz[p]);
  }
  __syncthreads();
  plane_forward<T, MP>(lds, a, tw1, tw2, tid, nthr);
  const int64_t so = ((int64_t)b * a.n3 + z) * a.S;
  for (int s = tid; s < a.S; s += nthr) {
    const cplx<T> v = lds[a.si1[s] * a.pitch + a.si2[s]];
    sout[so + s] = cadd<T>(sout[so + s], v);
  }
}

// ---------------------------------------------------------------------------
// response Hartree + xc potential of one instance
// ---------------------------------------------------------------------------
// (1) n'(r) = sum over band groups (fixed order); 2-D forward transform
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_hxc_planes_fwd(const cplx<T>* __restrict__ dpart, int ngroups,
                                 cplx<T>* __restrict__ nr, cplx<T>* __restrict__ work,
                                 PlaneArgs a, const cplx<T>* __restrict__ tw1,
                                 const cplx<T>* __restrict__ tw2, const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int z = blockIdx.x;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int np = a.n1 * a.n2;
  const int64_t plane = (int64_t)a.n3 * np;
  for (int p = tid; p < np; p += nthr) {
    cplx<T> s = czero<T>();
    for (int g = 0; g < ngroups; ++g) s = cadd<T>(s, dpart[g * plane + (int64_t)z * np + p]);
    nr[(int64_t)z * np + p] = s;
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    lds[i1 * a.pitch + i2] = s;
  }
  __syncthreads();
  fft_lds<T, MP, -1>(lds, Lay{a.pitch, 1, nullptr}, a.p1, a.n2, tw1, tid, nthr);
  fft_lds<T, MP, -1>(lds, Lay{1, a.pitch, nullptr}, a.p2, a.n1, tw2, tid, nthr);
  for (int p = tid; p < np; p += nthr) {
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    work[(int64_t)z * np + p] = lds[i1 * a.pitch + i2];
  }
}

// (2) along z: forward, times 4 pi / (|q+G|^2 N), inverse
template <typename T>
__global__ __launch_bounds__(256) void k_hxc_z(cplx<T>* __restrict__ work, const T* __restrict__ khart, int np, int n3,
                        FftPlan pz, const cplx<T>* __restrict__ tw, const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int c0 = blockIdx.x * kColTile;
  const int nc = min(kColTile, np - c0);
  const int pitch = n3 + 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < nc * n3; t += nthr) {
    const int z = t / nc, c = t - z * nc;
    lds[c * pitch + z] = work[(int64_t)z * np + c0 + c];
  }
  __syncthreads();
  fft_lds<T, kStickMaxPt, -1>(lds, Lay{1, pitch, nullptr}, pz, nc, tw, tid, nthr);
  for (int t = tid; t < nc * n3; t += nthr) {
    const int z = t / nc, c = t - z * nc;
    cplx<T>& v = lds[c * pitch + z];
    v = cscale<T>(v, khart[(int64_t)z * np + c0 + c]);
  }
  __syncthreads();
  fft_lds<T, kStickMaxPt, +1>(lds, Lay{1, pitch, nullptr}, pz, nc, tw, tid, nthr);
  for (int t = tid; t < nc * n3; t += nthr) {
    const int z = t / nc, c = t - z * nc;
    work[(int64_t)z * np + c0 + c] = lds[c * pitch + z];
  }
}

// (3) 2-D inverse transform, v'(r) = v_H(r) + f_xc(r) n'(r)
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_hxc_planes_inv(const cplx<T>* __restrict__ work, const cplx<T>* __restrict__ nr,
                                 const T* __restrict__ fxc, int with_fxc, cplx<T>* __restrict__ vp,
                                 PlaneArgs a, const cplx<T>* __restrict__ tw1,
                                 const cplx<T>* __restrict__ tw2, const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int z = blockIdx.x;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int np = a.n1 * a.n2;
  for (int p = tid; p < np; p += nthr) {
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    lds[i1 * a.pitch + i2] = work[(int64_t)z * np + p];
  }
  __syncthreads();
  fft_lds<T, MP, +1>(lds, Lay{1, a.pitch, nullptr}, a.p2, a.n1, tw2, tid, nthr);
  fft_lds<T, MP, +1>(lds, Lay{a.pitch, 1, nullptr}, a.p1, a.n2, tw1, tid, nthr);
  for (int p = tid; p < np; p += nthr) {
    const int i1 = p / a.n2, i2 = p - i1 * a.n2;
    cplx<T> v = lds[i1 * a.pitch + i2];
    if (with_fxc) {
      const cplx<T> n = nr[(int64_t)z * np + p];
      const T f = fxc[(int64_t)z * np + p];
      v.x += f * n.x;
      v.y += f * n.y;
    }
    vp[(int64_t)z * np + p] = v;
  }
}

// ---------------------------------------------------------------------------
// separable projectors and the conduction projector:
//   C[k][p][n] = coef_p sum_G conj(A[k][p][G]) X[k][n][G]    (split over G)
//   Y[k][n][G] += sum_p A[k][p][G] C[k][p][n]
// ---------------------------------------------------------------------------
constexpr int kDotTile = 32;   // output tile (p and n)
constexpr int kDotK = 32;      // G per LDS tile
constexpr int kDotChunk = 512; // G per block (split-K chunk)

template <typename T>
__global__ __launch_bounds__(256) void k_proj_dot(const cplx<T>* __restrict__ A, int P, const cplx<T>* __restrict__ X,
                           int nbnd, int npwx, int nchunk, cplx<T>* __restrict__ partial,
                           const LzDevState* st) {
  if (st && st->status) return;
  __shared__ cplx<T> As[kDotTile][kDotK + 1];
  __shared__ cplx<T> Xs[kDotTile][kDotK + 1];
  const int ntn = (nbnd + kDotTile - 1) / kDotTile;
  const int tp0 = (blockIdx.x / ntn) * kDotTile;
  const int tn0 = (blockIdx.x % ntn) * kDotTile;
  const int chunk = blockIdx.y, k = blockIdx.z;
  const int tid = threadIdx.x;  // 256 = 16 x 16, 2 x 2 outputs each
  const int ty = tid / 16, tx = tid % 16;
  cplx<T> acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = czero<T>();
  const cplx<T>* Ak = A + (int64_t)k * P * npwx;
  const cplx<T>* Xk = X + (int64_t)k * nbnd * npwx;
  const int g_end = min(npwx, (chunk + 1) * kDotChunk);
  for (int g0 = chunk * kDotChunk; g0 < g_end; g0 += kDotK) {
    for (int t = tid; t < kDotTile * kDotK; t += 256) {
      const int r = t / kDotK, c = t - r * kDotK;
      const int g = g0 + c;
      const int p = tp0 + r, n = tn0 + r;
      As[r][c] = (p < P && g < g_end) ? Ak[(int64_t)p * npwx + g] : czero<T>();
      Xs[r][c] = (n < nbnd && g < g_end) ? Xk[(int64_t)n * npwx + g] : czero<T>();
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < kDotK; ++c) {
      const cplx<T> a0 = As[ty * 2][c], a1 = As[ty * 2 + 1][c];
      const cplx<T> x0 = Xs[tx * 2][c], x1 = Xs[tx * 2 + 1][c];
      acc[0][0] = cadd<T>(acc[0][0], cmulc<T>(a0, x0));
      acc[0][1] = cadd<T>(acc[0][1], cmulc<T>(a0, x1));
      acc[1][0] = cadd<T>(acc[1][0], cmulc<T>(a1, x0));
      acc[1][1] = cadd<T>(acc[1][1], cmulc<T>(a1, x1));
    }
    __syncthreads();
  }
  cplx<T>* out = partial + ((int64_t)k * nchunk + chunk) * P * nbnd;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int p = tp0 + ty * 2 + i, n = tn0 + tx * 2 + j;
      if (p < P && n < nbnd) out[p * nbnd + n] = acc[i][j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_proj_reduce(const cplx<T>* __restrict__ partial, int nchunk, int P, int nbnd,
                              cplx<T>* __restrict__ C, const double* __restrict__ coef,
                              double coef_const, const LzDevState* st) {
  if (st && st->status) return;
  const int k = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * nbnd) return;
  const cplx<T>* pk = partial + (int64_t)k * nchunk * P * nbnd;
  double sx = 0.0, sy = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const cplx<T> v = pk[(int64_t)c * P * nbnd + i];
    sx += double(v.x);
    sy += double(v.y);
  }
  const double f = coef ? coef[i / nbnd] : coef_const;
  C[(int64_t)k * P * nbnd + i] = mk<T>(T(f * sx), T(f * sy));
}

constexpr int kUpdBands = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_proj_update(const cplx<T>* __restrict__ A, int P, const cplx<T>* __restrict__ C,
                              cplx<T>* __restrict__ Y, int nbnd, int npwx,
                              const LzDevState* st) {
  if (st && st->status) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* Cs = reinterpret_cast<cplx<T>*>(smem_raw);  // [P][kUpdBands]
  const int k = blockIdx.z;
  const int n0 = blockIdx.y * kUpdBands;
  const int nbt = min(kUpdBands, nbnd - n0);
  const cplx<T>* Ck = C + (int64_t)k * P * nbnd;
  for (int t = threadIdx.x; t < P * kUpdBands; t += blockDim.x) {
    const int p = t / kUpdBands, j = t - p * kUpdBands;
    Cs[t] = j < nbt ? Ck[p * nbnd + n0 + j] : czero<T>();
  }
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npwx) return;
  const cplx<T>* Ak = A + (int64_t)k * P * npwx;
  cplx<T> acc[kUpdBands];
#pragma unroll
  for (int j = 0; j < kUpdBands; ++j) acc[j] = czero<T>();
  for (int p = 0; p < P; ++p) {
    const cplx<T> a = Ak[(int64_t)p * npwx + g];
#pragma unroll
    for (int j = 0; j < kUpdBands; ++j) acc[j] = cadd<T>(acc[j], cmul<T>(a, Cs[p * kUpdBands + j]));
  }
  cplx<T>* Yk = Y + (int64_t)k * nbnd * npwx;
#pragma unroll
  for (int j = 0; j < kUpdBands; ++j) {
    if (j < nbt) {
      cplx<T>& yv = Yk[(int64_t)(n0 + j) * npwx + g];
      yv = cadd<T>(yv, acc[j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Lanczos vectors and scalars
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_lz_update(cplx<T>* __restrict__ w, const cplx<T>* __restrict__ lw, int64_t n,
                            const LzDevState* st) {
  if (st->status) return;
  const T a = T(st->a), b = T(st->b);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<T> l = lw[i], v = w[i];
    w[i] = mk<T>(a * l.x + b * v.x, a * l.y + b * v.y);
  }
}

constexpr int kDotThreads = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_lz_dots(const cplx<T>* __restrict__ w, const cplx<T>* __restrict__ lw,
                          const cplx<T>* __restrict__ y, const double* __restrict__ wk, int nbnd,
                          int npwx, int nks, double* __restrict__ partial,
                          const LzDevState* st) {
  if (st && st->status) return;
  __shared__ double red[3][kDotThreads];
  const int64_t per_k = (int64_t)nbnd * npwx;
  const int64_t n = per_k * nks;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kDotThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kDotThreads) {
    const double wt = wk[i / per_k];
    const cplx<T> a = w[i], l = lw[i], yv = y[i];
    s0 += wt * (double(a.x) * double(l.x) + double(a.y) * double(l.y));
    s1 += wt * (double(yv.x) * double(a.x) + double(yv.y) * double(a.y));
    s2 += wt * (double(yv.x) * double(a.y) - double(yv.y) * double(a.x));
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
  if (threadIdx.x == 0) {
    partial[blockIdx.x * 3 + 0] = red[0][0];
    partial[blockIdx.x * 3 + 1] = red[1][0];
    partial[blockIdx.x * 3 + 2] = red[2][0];
  }
}

// Sum the partials and take the scalar decisions of one Lanczos step:
//   j = st->step; b2 = Re<w_j, L w_j>_w; beta_{j+1} = sqrt(b2);
//   z_{j+1} = <y, w_j>_w / beta_{j+1} for odd j (upper vector), else 0.
// Step 0 (w_0 = y) first checks for a vanished right-hand side.
__global__ __launch_bounds__(256) void k_lz_finalize(const double* __restrict__ partial, int nblk,
                              LzDevState* __restrict__ st, double* __restrict__ beta,
                              double* __restrict__ z, int max_steps, double tol, double yscale) {
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

__global__ __launch_bounds__(256) void k_set_state(LzDevState* st) {
  st->step = 0;
  st->status = 0;
  st->bmax = 0.0;
  st->a = 0.0;
  st->b = 0.0;
  st->beta_prev = 0.0;
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
// spectrum: one thread per frequency.  chi needs (z, (w~ - T)^-1 e_1), which
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

__global__ __launch_bounds__(256) void k_spectrum(const double* __restrict__ beta, const double* __restrict__ z, int m,
                           const double* __restrict__ omega, int nw, double eta, double pref,
                           double fq, double* __restrict__ chi, double* __restrict__ einv,
                           double* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  const double2 wt = make_double2(omega[i], eta);
  double2 c = make_double2(0.0, 0.0), d = make_double2(0.0, 0.0);
  for (int j = m; j >= 1; --j) {
    const double bnext = j < m ? beta[j] : 0.0;  // beta_{j+1}
    const double2 den = make_double2(wt.x - bnext * c.x, wt.y - bnext * c.y);
    const double2 num = make_double2(z[2 * (j - 1)] + bnext * d.x, z[2 * (j - 1) + 1] + bnext * d.y);
    d = zdiv(num, den);
    c = zdiv(make_double2(beta[j - 1], 0.0), den);
  }
  double2 ch = make_double2(0.0, 0.0);
  if (m > 0) ch = make_double2(pref * beta[0] * d.x, pref * beta[0] * d.y);
  chi[2 * i] = ch.x;
  chi[2 * i + 1] = ch.y;
  einv[2 * i] = 1.0 + fq * ch.x;
  einv[2 * i + 1] = fq * ch.y;
  loss[i] = -fq * ch.y;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static PlaneArgs plane_args(const Grid3& g) {
  PlaneArgs a;
  a.n1 = g.n1; a.n2 = g.n2; a.n3 = g.n3; a.S = g.S; a.nact = g.nact; a.pitch = g.pitch2;
  a.si1 = g.si1; a.si2 = g.si2; a.act = g.act; a.p1 = g.p1; a.p2 = g.p2;
  return a;
}

template <typename T> static size_t plane_lds(const Grid3& g) {
  return (size_t)g.n1 * g.pitch2 * sizeof(cplx<T>);
}
template <typename T> static size_t stick_lds(const Grid3& g) {
  return (size_t)kStickTile * (g.n3 + 1) * sizeof(cplx<T>);
}
static int stick_threads() { return 256; }

template <typename T>
void Launch<T>::zfft_inv(const Grid3& g, const void* x, int64_t xs, void* sticks, const int* map,
                         int nb, int nbnd, const LzDevState* st, hipStream_t s) {
  dim3 grid((g.S + kStickTile - 1) / kStickTile, nb);
  hipLaunchKernelGGL(k_zfft_inv<T>, grid, dim3(stick_threads()), stick_lds<T>(g), s,
                     (const cplx<T>*)x, xs, (cplx<T>*)sticks, map, g.S, g.n3, nbnd, g.p3,
                     (const cplx<T>*)g.tw3, st);
}

template <typename T>
void Launch<T>::zfft_fwd(const Grid3& g, const void* sticks, const void* x, int64_t xs, void* y,
                         const int* map, const void* kin, const double* eps, int nb, int nbnd,
                         int npwx, const LzDevState* st, hipStream_t s) {
  dim3 grid((g.S + kStickTile - 1) / kStickTile, nb);
  const T scale = T(1.0 / ((double)g.n1 * g.n2 * g.n3));
  hipLaunchKernelGGL(k_zfft_fwd<T>, grid, dim3(stick_threads()), stick_lds<T>(g), s,
                     (const cplx<T>*)sticks, (const cplx<T>*)x, xs, (cplx<T>*)y, map,
                     (const T*)kin, eps, g.S, g.n3, nbnd, npwx, scale, g.p3,
                     (const cplx<T>*)g.tw3, st);
}

template <typename T>
void Launch<T>::plane_local(const Grid3& g, const void* sin, void* sout, const void* vloc, int nb,
                            const LzDevState* st, hipStream_t s) {
  LZ_PLANE_LAUNCH(k_plane_local, T, plane_mp(g.n1, g.n2), dim3(g.n3, nb), plane_lds<T>(g), s, (const cplx<T>*)sin, (cplx<T>*)sout, (const T*)vloc,
                     plane_args(g), (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2, st);
}

template <typename T>
void Launch<T>::plane_local_density(const Grid3& g, const void* sin, void* sout, const void* vloc,
                                    const void* ur, const double* bandw, void* dpart, int nb,
                                    int gsize, const LzDevState* st, hipStream_t s) {
  const int ng = (nb + gsize - 1) / gsize;
  LZ_PLANE_LAUNCH(k_plane_local_density, T, plane_mp(g.n1, g.n2), dim3(g.n3, ng), plane_lds<T>(g), s, (const cplx<T>*)sin, (cplx<T>*)sout, (const T*)vloc,
                     (const cplx<T>*)ur, bandw, (cplx<T>*)dpart, nb, gsize, plane_args(g),
                     (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2, st);
}

template <typename T>
void Launch<T>::plane_to_real(const Grid3& g, const void* sin, void* rout, int nb, hipStream_t s) {
  LZ_PLANE_LAUNCH(k_plane_to_real, T, plane_mp(g.n1, g.n2), dim3(g.n3, nb), plane_lds<T>(g), s, (const cplx<T>*)sin, (cplx<T>*)rout, plane_args(g),
                     (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2);
}

template <typename T>
void Launch<T>::plane_vu(const Grid3& g, const void* ur, const void* vp, void* sout, int nb,
                         const LzDevState* st, hipStream_t s) {
  LZ_PLANE_LAUNCH(k_plane_vu, T, plane_mp(g.n1, g.n2), dim3(g.n3, nb), plane_lds<T>(g), s, (const cplx<T>*)ur, (const cplx<T>*)vp, (cplx<T>*)sout,
                     plane_args(g), (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2, st);
}

template <typename T>
void Launch<T>::hxc(const Grid3& g, const void* dpart, int ngroups, void* nr, void* work,
                    const void* khart, const void* fxc, bool with_fxc, void* vp,
                    const LzDevState* st, hipStream_t s) {
  const int np = g.n1 * g.n2;
  LZ_PLANE_LAUNCH(k_hxc_planes_fwd, T, plane_mp(g.n1, g.n2), dim3(g.n3), plane_lds<T>(g), s, (const cplx<T>*)dpart, ngroups, (cplx<T>*)nr,
                     (cplx<T>*)work, plane_args(g), (const cplx<T>*)g.tw1, (const cplx<T>*)g.tw2,
                     st);
  hipLaunchKernelGGL(k_hxc_z<T>, dim3((np + kColTile - 1) / kColTile), dim3(256),
                     (size_t)kColTile * (g.n3 + 1) * sizeof(cplx<T>), s, (cplx<T>*)work,
                     (const T*)khart, np, g.n3, g.p3, (const cplx<T>*)g.tw3, st);
  LZ_PLANE_LAUNCH(k_hxc_planes_inv, T, plane_mp(g.n1, g.n2), dim3(g.n3), plane_lds<T>(g), s, (const cplx<T>*)work, (const cplx<T>*)nr, (const T*)fxc,
                     with_fxc ? 1 : 0, (cplx<T>*)vp, plane_args(g), (const cplx<T>*)g.tw1,
                     (const cplx<T>*)g.tw2, st);
}

template <typename T>
void Launch<T>::proj_dot(const void* A, int P, const void* X, int nbnd, int npwx, int nks,
                         void* partial, int nchunk, void* C, const double* coef,
                         double coef_const, const LzDevState* st, hipStream_t s) {
  const int tiles = ((P + kDotTile - 1) / kDotTile) * ((nbnd + kDotTile - 1) / kDotTile);
  hipLaunchKernelGGL(k_proj_dot<T>, dim3(tiles, nchunk, nks), dim3(256), 0, s,
                     (const cplx<T>*)A, P, (const cplx<T>*)X, nbnd, npwx, nchunk,
                     (cplx<T>*)partial, st);
  hipLaunchKernelGGL(k_proj_reduce<T>, dim3((P * nbnd + 255) / 256, nks), dim3(256), 0, s,
                     (const cplx<T>*)partial, nchunk, P, nbnd, (cplx<T>*)C, coef, coef_const, st);
}

template <typename T>
void Launch<T>::proj_update(const void* A, int P, const void* C, void* Y, int nbnd, int npwx,
                            int nks, const LzDevState* st, hipStream_t s) {
  dim3 grid((npwx + 255) / 256, (nbnd + kUpdBands - 1) / kUpdBands, nks);
  hipLaunchKernelGGL(k_proj_update<T>, grid, dim3(256), (size_t)P * kUpdBands * sizeof(cplx<T>),
                     s, (const cplx<T>*)A, P, (const cplx<T>*)C, (cplx<T>*)Y, nbnd, npwx, st);
}

template <typename T>
void Launch<T>::lz_update(void* w, const void* lw, int64_t n, const LzDevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_update<T>, dim3(1024), dim3(256), 0, s, (cplx<T>*)w,
                     (const cplx<T>*)lw, n, st);
}

template <typename T>
void Launch<T>::lz_dots(const void* w, const void* lw, const void* y, const double* wk, int nbnd,
                        int npwx, int nks, double* partial, int nblk, const LzDevState* st,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_lz_dots<T>, dim3(nblk), dim3(kDotThreads), 0, s, (const cplx<T>*)w,
                     (const cplx<T>*)lw, (const cplx<T>*)y, wk, nbnd, npwx, nks, partial, st);
}

template <typename T>
void Launch<T>::perm_in(const void* xu, void* xi, const int* perm, const int* npw, int nks,
                        int nbnd, int npwx, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_in<T>, dim3((npwx + 255) / 256, nks * nbnd), dim3(256), 0, s,
                     (const cplx<T>*)xu, (cplx<T>*)xi, perm, npw, nbnd, npwx);
}

template <typename T>
void Launch<T>::perm_out(const void* xi, void* xu, const int* perm, const int* npw, int nks,
                         int nbnd, int npwx, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_out<T>, dim3((npwx + 255) / 256, nks * nbnd), dim3(256), 0, s,
                     (const cplx<T>*)xi, (cplx<T>*)xu, perm, npw, nbnd, npwx);
}

template <typename T>
void Launch<T>::copy(void* dst, const void* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<T>, dim3(1024), dim3(256), 0, s, (cplx<T>*)dst, (const cplx<T>*)src, n);
}

void launch_lz_finalize(const double* partial, int nblk, LzDevState* st, double* beta, double* z,
                        int max_steps, double tol, double yscale, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_finalize, dim3(1), dim3(kDotThreads), 0, s, partial, nblk, st, beta, z,
                     max_steps, tol, yscale);
}

void launch_spectrum(const double* beta, const double* z, int m, const double* omega, int nw,
                     double eta, double pref, double fq, double* chi, double* einv, double* loss,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum, dim3((nw + 63) / 64), dim3(64), 0, s, beta, z, m, omega, nw, eta,
                     pref, fq, chi, einv, loss);
}

void launch_set_state(LzDevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st);
}

template struct Launch<double>;
template struct Launch<float>;

// Kernels whose LDS may exceed the default dynamic limit opt in once.
hipError_t enable_large_lds() {
  const int big = 160 * 1024;
#define LZ_LDS_ATTR(KERN)                                                          \
  {                                                                                \
    const void* fns[] = {(const void*)KERN<double, 12>, (const void*)KERN<double, 24>, \
                         (const void*)KERN<double, 36>, (const void*)KERN<float, 12>,  \
                         (const void*)KERN<float, 24>,  (const void*)KERN<float, 36>}; \
    for (const void* f : fns) {                                                    \
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big); \
      if (e != hipSuccess) return e;                                               \
    }                                                                              \
  }
  LZ_LDS_ATTR(k_plane_local)
  LZ_LDS_ATTR(k_plane_local_density)
  LZ_LDS_ATTR(k_plane_to_real)
  LZ_LDS_ATTR(k_plane_vu)
  LZ_LDS_ATTR(k_hxc_planes_fwd)
  LZ_LDS_ATTR(k_hxc_planes_inv)
#undef LZ_LDS_ATTR
  return hipSuccess;
}

}  // namespace lz
