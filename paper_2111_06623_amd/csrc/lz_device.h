// Device-side building blocks: complex arithmetic, small DFT butterflies and
// the in-place LDS Stockham pass used by every FFT kernel of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lz {

template <typename T> struct CplxOf;
template <> struct CplxOf<double> { using type = double2; };
template <> struct CplxOf<float> { using type = float2; };
template <typename T> using cplx = typename CplxOf<T>::type;

template <typename T>
__device__ __forceinline__ cplx<T> mk(T x, T y) { cplx<T> r; r.x = x; r.y = y; return r; }
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by +i (dir = +1) or -i (dir = -1)
template <typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a, int dir) {
  return dir > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// FFT plans.  A length-n transform is a product of radix passes (4, 3, 5, 2).
// Pass p with radix R and ns = product of the earlier radices maps
//   in[j + r*(n/R)] * w^{r*(j mod ns)}, w = exp(s 2 pi i / (ns R)),
//   radix-R DFT over r -> out[(j/ns)*ns*R + (j mod ns) + t*ns]
// (self-sorting Stockham formulation).  Twiddles of pass p live at
// tw[twoff[p] + k*(R-1) + (r-1)] = exp(-2 pi i k r / (ns R)); the inverse
// direction uses their conjugates.
// ---------------------------------------------------------------------------
constexpr int kMaxPass = 8;
struct FftPlan {
  int n;
  int npass;
  int radix[kMaxPass];
  int ns[kMaxPass];
  int twoff[kMaxPass];
};

// radix-R DFT of v[0..R-1] in place; DIR = -1 forward (exp(-i..)), +1 inverse.
// Radices 8 and 16 (compile-time plans only) are defined in lz_fft_ct.h; the
// runtime plans of the general form use 4, 3, 5 and 2.
template <typename T, int R, int DIR> struct Dft;

template <typename T, int DIR> struct Dft<T, 2, DIR> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  }
};

template <typename T, int DIR> struct Dft<T, 4, DIR> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    // b1 = a0 + w a1 + w^2 a2 + w^3 a3 with w = exp(DIR i pi/2) = DIR*i
    cplx<T> s02 = cadd<T>(v[0], v[2]), d02 = csub<T>(v[0], v[2]);
    cplx<T> s13 = cadd<T>(v[1], v[3]), d13 = csub<T>(v[1], v[3]);
    cplx<T> r = mul_i<T>(d13, DIR);
    v[0] = cadd<T>(s02, s13);
    v[2] = csub<T>(s02, s13);
    v[1] = cadd<T>(d02, r);
    v[3] = csub<T>(d02, r);
  }
};

template <typename T, int DIR> struct Dft<T, 3, DIR> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    // w = exp(DIR 2 pi i/3) = -1/2 + DIR i sqrt(3)/2
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    cplx<T> t1 = cadd<T>(v[1], v[2]), t2 = csub<T>(v[1], v[2]);
    cplx<T> m1 = mk<T>(v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y);
    cplx<T> m2 = cscale<T>(mul_i<T>(t2, DIR), h);
    v[0] = cadd<T>(v[0], t1);
    v[1] = cadd<T>(m1, m2);
    v[2] = csub<T>(m1, m2);
  }
};

template <typename T, int DIR> struct Dft<T, 5, DIR> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    const T c1 = T(0.30901699437494742410);   // cos(2 pi/5)
    const T c2 = T(-0.80901699437494742410);  // cos(4 pi/5)
    const T s1 = T(0.95105651629515357212);   // sin(2 pi/5)
    const T s2 = T(0.58778525229247312917);   // sin(4 pi/5)
    cplx<T> t1 = cadd<T>(v[1], v[4]), t2 = cadd<T>(v[2], v[3]);
    cplx<T> t3 = csub<T>(v[1], v[4]), t4 = csub<T>(v[2], v[3]);
    cplx<T> a0 = v[0];
    cplx<T> p1 = mk<T>(a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y);
    cplx<T> p2 = mk<T>(a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y);
    cplx<T> q1 = mk<T>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    cplx<T> q2 = mk<T>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    // forward: b1 = p1 - i q1, b4 = p1 + i q1, b2 = p2 - i q2, b3 = p2 + i q2
    cplx<T> iq1 = mul_i<T>(q1, DIR), iq2 = mul_i<T>(q2, DIR);
    v[0] = mk<T>(a0.x + t1.x + t2.x, a0.y + t1.y + t2.y);
    v[1] = cadd<T>(p1, iq1);
    v[4] = csub<T>(p1, iq1);
    v[2] = cadd<T>(p2, iq2);
    v[3] = csub<T>(p2, iq2);
  }
};

// Addressing of a batch of 1-D transforms inside an LDS buffer:
//   element i of transform b is at base(b) + i*stride,
//   base(b) = (rows ? rows[b] : b) * dist.
struct Lay {
  int stride;
  int dist;
  const int* rows;  // optional indirection (LDS or global), may be null
  __device__ __forceinline__ int base(int b) const { return (rows ? rows[b] : b) * dist; }
};

// One radix-R Stockham pass over `nbatch` transforms of length n, in place.
// Every thread first loads and transforms all of its butterflies into
// registers, the block synchronises, then every thread stores; MAXB bounds
// the butterflies a thread holds (checked by the host through launch shapes).
template <typename T, int R, int MAXB, int DIR>
__device__ __forceinline__ void fft_pass(cplx<T>* lds, Lay lay, int n, int nbatch, int ns,
                                         const cplx<T>* __restrict__ tw, int tid, int nthr) {
  const int m = n / R;
  const int total = nbatch * m;
  cplx<T> v[MAXB][R];
  int bbase[MAXB], bj[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int t = tid + i * nthr;
    if (t < total) {
      const int b = t / m;
      const int j = t - b * m;
      const int k = j % ns;
      const int base = lay.base(b);
      bbase[i] = base;
      bj[i] = j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[base + (j + r * m) * lay.stride];
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[k * (R - 1) + (r - 1)];
          if (DIR > 0) w.y = -w.y;
          v[i][r] = cmul<T>(v[i][r], w);
        }
      }
      Dft<T, R, DIR>::run(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int t = tid + i * nthr;
    if (t < total) {
      const int j = bj[i];
      const int k = j % ns;
      const int o = (j / ns) * ns * R + k;
#pragma unroll
      for (int s = 0; s < R; ++s) lds[bbase[i] + (o + s * ns) * lay.stride] = v[i][s];
    }
  }
  __syncthreads();
}

// Full transform: all passes of a plan.  MAXPT bounds the complex values a
// thread touches per pass (nbatch*n <= MAXPT*nthr).
template <typename T, int MAXPT, int DIR>
__device__ __forceinline__ void fft_lds(cplx<T>* lds, Lay lay, const FftPlan& p, int nbatch,
                                        const cplx<T>* __restrict__ tw, int tid, int nthr) {
  for (int s = 0; s < p.npass; ++s) {
    const cplx<T>* t = tw + p.twoff[s];
    switch (p.radix[s]) {
      case 4: fft_pass<T, 4, (MAXPT + 3) / 4, DIR>(lds, lay, p.n, nbatch, p.ns[s], t, tid, nthr); break;
      case 3: fft_pass<T, 3, (MAXPT + 2) / 3, DIR>(lds, lay, p.n, nbatch, p.ns[s], t, tid, nthr); break;
      case 5: fft_pass<T, 5, (MAXPT + 4) / 5, DIR>(lds, lay, p.n, nbatch, p.ns[s], t, tid, nthr); break;
      default: fft_pass<T, 2, (MAXPT + 1) / 2, DIR>(lds, lay, p.n, nbatch, p.ns[s], t, tid, nthr); break;
    }
  }
}

// Recursion state kept on the device (one per instance).
struct LzDevState {
  int step;          // completed Lanczos steps
  int status;        // 0 running, 6 breakdown, 4 not positive definite, 7 non-finite
  int pad0, pad1;
  double bmax;       // largest beta_2..beta_j so far
  double a, b;       // next update: w <- a*LW + b*w_old
  double beta_prev;  // beta of the last completed step
  // non-Hermitian recursion: complex coefficients (re, im) of the next
  // formation v^ <- cv1 L v^ + cv2 v^_old, u^ <- cu1 L^dagger u^ + cu2 u^_old,
  // and gamma of the last completed step
  double cv1[2], cv2[2], cu1[2], cu2[2];
  double gamma_prev[2];
};

}  // namespace lz
