// C ABI of the library: context construction, the Liouvillian application,
// the pseudo-Hermitian Lanczos driver and the spectrum (see include/lz.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lz.h"
#include "lz_fft_ct.h"
#include "lz_kernels.h"

using namespace lz;

// Staging area of lz_spectrum_ext_noalloc, one copy per device for the life of
// the process: the frequency grid, then chi, eps^-1 and the loss, then the two
// tail means of the extrapolation.  Host code never names it in a kernel
// argument or a copy; it uses the device address that hipGetSymbolAddress
// returns for the current device (scratch_address).
constexpr int kNoallocMaxOmega = 65536;
constexpr size_t kScratchDoubles = 6 * (size_t)kNoallocMaxOmega + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_last_error;

struct LzError {
  lz_status st;
  std::string msg;
};

[[noreturn]] void fail(lz_status st, const std::string& msg) { throw LzError{st, msg}; }

#define HIPC(call)                                                                    \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      if (e_ == hipErrorOutOfMemory) fail(LZ_ERR_OOM, std::string(#call) + ": out of device memory"); \
      fail(LZ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
    }                                                                                 \
  } while (0)

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kBreakdownTol = 1e-7;
// default number of streams for the instances of one context (the hardware
// queues a process gets by default)
constexpr int kInstStreams = 4;

// device buffer with RAII
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { if (p) (void)hipFree(p); }
  void alloc(size_t b) {
    if (p) { (void)hipFree(p); p = nullptr; }
    bytes = b ? b : 16;
    HIPC(hipMalloc(&p, bytes));
    // zero-fill and wait: later work runs on a non-blocking stream that is not
    // ordered after the null stream
    HIPC(hipMemset(p, 0, bytes));
    HIPC(hipDeviceSynchronize());
  }
  template <typename U> U* as() const { return reinterpret_cast<U*>(p); }
};

template <typename U>
void upload(DBuf& d, const std::vector<U>& h) {
  d.alloc(h.size() * sizeof(U));
  if (!h.empty()) HIPC(hipMemcpy(d.p, h.data(), h.size() * sizeof(U), hipMemcpyHostToDevice));
}

// factor n into radix passes (4, 3, 5, 2) and build the forward twiddles
bool make_plan(int n, FftPlan& p, std::vector<double>& tw_re, std::vector<double>& tw_im) {
  p.n = n;
  p.npass = 0;
  int m = n, ns = 1;
  if (ct_supported(n)) {
    // the radix list the compile-time kernels were built with
    for (int q = 0; q < ct_npass(n); ++q) {
      const int r = ct_radix(n, q);
      p.radix[p.npass] = r;
      p.ns[p.npass] = ns;
      p.twoff[p.npass] = (int)tw_re.size();
      for (int k = 0; k < ns; ++k)
        for (int t = 1; t < r; ++t) {
          const double ang = -kTwoPi * (double)k * t / ((double)ns * r);
          tw_re.push_back(std::cos(ang));
          tw_im.push_back(std::sin(ang));
        }
      ns *= r;
      m /= r;
      p.npass++;
    }
    return m == 1;
  }
  const int order[4] = {4, 3, 5, 2};
  for (int r : order) {
    while (m % r == 0) {
      if (p.npass >= kMaxPass) return false;
      p.radix[p.npass] = r;
      p.ns[p.npass] = ns;
      p.twoff[p.npass] = (int)tw_re.size();
      for (int k = 0; k < ns; ++k)
        for (int q = 1; q < r; ++q) {
          const double ang = -kTwoPi * (double)k * q / ((double)ns * r);
          tw_re.push_back(std::cos(ang));
          tw_im.push_back(std::sin(ang));
        }
      ns *= r;
      m /= r;
      p.npass++;
    }
  }
  return m == 1;
}

int centred(int i, int n) { return i >= (n + 1) / 2 ? i - n : i; }

// Stages of one Liouvillian half-application that can be timed with events.
enum Stage { ST_ZINV = 0, ST_PLANE = 1, ST_PLANE_DENS = 2, ST_HXC = 3, ST_PLANE_VU = 4,
             ST_ZFWD = 5, ST_PROJ = 6, ST_LANCZOS = 7, ST_COUNT = 8 };

struct StageTimer {
  bool on = false;
  uint32_t mask = 0;  // stages timed (bit s = stage s)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[ST_COUNT];
  double total_ms[ST_COUNT] = {0};
  int count[ST_COUNT] = {0};
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    hipEvent_t e;
    if (!pool.empty()) { e = pool.back(); pool.pop_back(); return e; }
    HIPC(hipEventCreate(&e));
    return e;
  }
  bool timed(int st) const { return on && ((mask >> st) & 1u); }
  void begin(int st, hipStream_t s, hipEvent_t& e0) {
    if (!timed(st)) return;
    e0 = get();
    HIPC(hipEventRecord(e0, s));
  }
  void end(int st, hipStream_t s, hipEvent_t e0) {
    if (!timed(st)) return;
    hipEvent_t e1 = get();
    HIPC(hipEventRecord(e1, s));
    pending[st].push_back({e0, e1});
  }
  // fold completed pairs into the totals (after a stream synchronisation)
  void collect() {
    for (int st = 0; st < ST_COUNT; ++st) {
      for (auto& pr : pending[st]) {
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, pr.first, pr.second));
        total_ms[st] += ms;
        count[st] += 1;
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      pending[st].clear();
    }
  }
  void reset() {
    for (int st = 0; st < ST_COUNT; ++st) { total_ms[st] = 0; count[st] = 0; }
  }
  ~StageTimer() {
    for (int st = 0; st < ST_COUNT; ++st)
      for (auto& pr : pending[st]) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct Instance {
  lz_precision prec;
  lz_approx approx;
  bool nh = false;  // non-Hermitian biorthogonal recursion
  bool fp64;
  size_t csz;  // bytes per complex element
  int n1, n2, n3, N;
  int nks, nbnd, nproj, npwx, nb;
  double omega, q2;
  double pref, fq;
  int max_steps;
  int S = 0, nact = 0;
  int ngroups = 1, gsize = 1;
  int ptot = 0;                // rows of the stacked projector array [U; beta]
  int chunk = 32, nchunk = 1;  // split of the projector products over G
  int gemm = kGemmValu;        // where the projector products run
  int nlzblk = 1;              // blocks of the output update (Lanczos partial sums)
  int nlzblk_nl = 1;           // the same for the update over the separable rows only
  int64_t nvec;  // complex elements of one batch
  uint64_t fingerprint = 0;  // hash of every input the operator depends on (checkpoints)
  Grid3 grid;
  DBuf si1, si2, act, map_kq, map_k, perm, npw_kq;
  DBuf soff_f, soff_c;
  DBuf tw1, tw2, tw3;
  DBuf kin, eps, wk, bandw, vloc, fxc, khart;
  DBuf U, vkb, dkb;
  DBuf Aio, Mkb, Cin, Cout;
  DBuf ur, y;
  DBuf X0, X1, LW;
  DBuf Y0, Y1, LU, gam;  // non-Hermitian recursion: the u chain and complex gamma
  DBuf sa, sb;
  DBuf dpart, nr, work, vp;
  DBuf dpartial;
  DBuf lzpart, st, beta, z;
  DBuf tin, tout, tin2, tout2;
  int steps_host = 0;
  int status_host = 0;
  StageTimer timer;
  hipGraphExec_t gpair = nullptr;  // captured pair of steps (odd, even), built on first use
  ~Instance() {
    if (gpair) (void)hipGraphExecDestroy(gpair);
  }
};

#define STAGE(I, ST, S, ...)             \
  do {                                   \
    hipEvent_t e0_ = nullptr;            \
    (I).timer.begin(ST, S, e0_);         \
    __VA_ARGS__;                         \
    (I).timer.end(ST, S, e0_);           \
  } while (0)

template <typename T>
void to_dev_real(DBuf& d, const std::vector<double>& h) {
  std::vector<T> t(h.begin(), h.end());
  upload(d, t);
}

template <typename T>
void to_dev_cplx(DBuf& d, const std::vector<double>& h /* interleaved */) {
  std::vector<T> t(h.begin(), h.end());
  upload(d, t);
}

void upload_real(Instance& I, DBuf& d, const std::vector<double>& h) {
  if (I.fp64) to_dev_real<double>(d, h); else to_dev_real<float>(d, h);
}
void upload_cplx(Instance& I, DBuf& d, const std::vector<double>& h) {
  if (I.fp64) to_dev_cplx<double>(d, h); else to_dev_cplx<float>(d, h);
}

// 64-bit fingerprint of the operator's inputs: every 8-byte word of each
// array is mixed in turn (a multiply-xorshift finaliser per word), with each
// array's length mixed in first, so that equal inputs give equal values and
// a changed word changes the value with overwhelming probability.
struct Fingerprint {
  uint64_t h = 0x243F6A8885A308D3ull;
  void word(uint64_t w) {
    h ^= w;
    h *= 0xFF51AFD7ED558CCDull;
    h ^= h >> 33;
    h *= 0xC4CEB9FE1A85EC53ull;
    h ^= h >> 29;
  }
  template <typename U>
  void array(const std::vector<U>& v) {
    word((uint64_t)v.size() * sizeof(U));
    const size_t nbytes = v.size() * sizeof(U);
    const unsigned char* b = reinterpret_cast<const unsigned char*>(v.data());
    size_t i = 0;
    for (; i + 8 <= nbytes; i += 8) {
      uint64_t w;
      std::memcpy(&w, b + i, 8);
      word(w);
    }
    if (i < nbytes) {
      uint64_t w = 0;
      std::memcpy(&w, b + i, nbytes - i);
      word(w);
    }
  }
  void scalar(double x) {
    uint64_t w;
    std::memcpy(&w, &x, 8);
    word(w);
  }
};

bool valid_len(int n) {
  if (n < 2 || n > 128) return false;
  int m = n;
  for (int r : {2, 3, 5}) while (m % r == 0) m /= r;
  return m == 1;
}

// ---------------------------------------------------------------------------
// operator application on one instance (internal order, stream-ordered)
// ---------------------------------------------------------------------------
// Input side of an application: R = [U; beta]^H x, the coefficients of the
// separable term D (beta^H P_c x) and, with project, x <- P_c x.  With lw the
// Lanczos update x <- a lw + b x is formed first (fused into the dot when one
// block spans every row and band).
template <typename T>
void input_side(Instance& I, void* x, const void* lw, bool project, const LzDevState* st,
                hipStream_t s) {
  const bool fuse = lw != nullptr && LaunchLin<T>::dot_single_tile(I.ptot, I.nbnd, I.gemm);
  if (lw != nullptr && !fuse)
    STAGE(I, ST_LANCZOS, s, LaunchLin<T>::lz_update(x, lw, I.nvec, st, s));
  STAGE(I, ST_PROJ, s,
        LaunchLin<T>::proj_dot(I.Aio.p, I.ptot, I.ptot, x, fuse ? lw : nullptr, I.nbnd, I.npwx,
                               I.nks, I.chunk, I.nchunk, I.dpartial.p, st, s, I.gemm);
        LaunchLin<T>::reduce_coef_in(I.dpartial.p, I.nchunk, I.Mkb.p, I.dkb.as<double>(),
                                     I.nbnd, I.nproj, I.nks, !project, I.Cin.p, st, s));
  if (project)
    STAGE(I, ST_PROJ, s,
          LaunchLin<T>::proj_update(x, I.Aio.p, I.nbnd, I.ptot, I.Cin.p, I.ptot, I.nbnd, I.npwx,
                                    I.nks, nullptr, nullptr, nullptr, nullptr, st, s, I.gemm));
}

// Output side: out <- P_c (out + beta D B), as out + [U; beta] C_out with
// C_out = [-(U^H out + M^H D B); D B]; with lzpart also the Lanczos sums of
// (x, out, y) per block.
template <typename T>
void output_side(Instance& I, void* out, const void* x, double* lzpart, const LzDevState* st,
                 hipStream_t s) {
  STAGE(I, ST_PROJ, s,
        LaunchLin<T>::proj_dot(I.Aio.p, I.nbnd, I.ptot, out, nullptr, I.nbnd, I.npwx, I.nks,
                               I.chunk, I.nchunk, I.dpartial.p, st, s, I.gemm);
        LaunchLin<T>::reduce_coef_out(I.dpartial.p, I.nchunk, I.Cin.p, I.Mkb.p, I.nbnd, I.nproj,
                                      I.nks, I.Cout.p, st, s);
        LaunchLin<T>::proj_update(out, I.Aio.p, I.ptot, I.ptot, I.Cout.p, I.ptot, I.nbnd, I.npwx,
                                  I.nks, x, I.y.p, I.wk.as<double>(), lzpart, st, s, I.gemm));
}

// Output side of a pseudo-Hermitian step: out <- out + beta D B (D B from the
// input side of the same step), with the Lanczos sums of (x, out, y).  P_c is
// not applied to out here: the next step forms w = a out + b x' from it and
// its input side projects w, which in exact arithmetic is the vector that
// projecting out first would give (x' is already a conduction vector), and
// the sums pair out with the conduction vector x, blind to the valence part.
template <typename T>
void output_side_nl(Instance& I, void* out, const void* x, double* lzpart, const LzDevState* st,
                    hipStream_t s) {
  const cplx<T>* A = static_cast<const cplx<T>*>(I.Aio.p) + (size_t)I.nbnd * I.npwx;
  const cplx<T>* C = static_cast<const cplx<T>*>(I.Cin.p) + (size_t)I.nbnd * I.nbnd;
  STAGE(I, ST_PROJ, s,
        LaunchLin<T>::proj_update(out, A, I.nproj, I.ptot, C, I.ptot, I.nbnd, I.npwx, I.nks, x,
                                  I.y.p, I.wk.as<double>(), lzpart, st, s, I.gemm));
}

// FFT part of one half-application: out = (H_loc - eps) in (+ v'u for an
// upper vector), before the projector terms.
template <typename T>
void apply_core(Instance& I, const void* in, void* out, bool upper, const LzDevState* st,
                hipStream_t s) {
  const Grid3& g = I.grid;
  const int64_t xs = I.npwx;
  STAGE(I, ST_ZINV, s, LaunchFft<T>::zfft_inv(g, in, xs, I.sa.p, I.map_kq.as<int>(), I.nb, I.nbnd, st, s));
  if (upper && I.approx != LZ_IPA) {
    STAGE(I, ST_PLANE_DENS, s,
          LaunchFft<T>::plane_local_density(g, I.sa.p, I.sb.p, I.vloc.p, I.ur.p,
                                            I.bandw.as<double>(), I.dpart.p, I.nb, I.gsize, st, s));
    STAGE(I, ST_HXC, s,
          LaunchFft<T>::hxc(g, I.dpart.p, I.ngroups, I.nr.p, I.work.p, I.khart.p, I.fxc.p,
                            I.approx == LZ_TDDFT, I.vp.p, st, s));
    STAGE(I, ST_PLANE_VU, s, LaunchFft<T>::plane_vu(g, I.ur.p, I.vp.p, I.sb.p, I.nb, st, s));
  } else {
    STAGE(I, ST_PLANE, s, LaunchFft<T>::plane_local(g, I.sa.p, I.sb.p, I.vloc.p, I.nb, st, s));
  }
  STAGE(I, ST_ZFWD, s,
        LaunchFft<T>::zfft_fwd(g, I.sb.p, in, xs, out, I.map_kq.as<int>(), I.kin.p,
                               I.eps.as<double>(), I.nb, I.nbnd, I.npwx, st, s));
}

// One operator application on a vector the caller owns: D (lower) or D+K
// (upper) with P_c on the output only.
template <typename T>
void apply_half(Instance& I, void* in, void* out, bool upper, hipStream_t s) {
  input_side<T>(I, in, nullptr, false, nullptr, s);
  apply_core<T>(I, in, out, upper, nullptr, s);
  output_side<T>(I, out, nullptr, nullptr, nullptr, s);
}

// P_c on a vector (set-up of the right-hand side)
template <typename T>
void project_c(Instance& I, void* x, hipStream_t s) {
  LaunchLin<T>::proj_dot(I.Aio.p, I.nbnd, I.ptot, x, nullptr, I.nbnd, I.npwx, I.nks, I.chunk,
                         I.nchunk, I.dpartial.p, nullptr, s, I.gemm);
  LaunchLin<T>::reduce_coef_in(I.dpartial.p, I.nchunk, I.Mkb.p, I.dkb.as<double>(), I.nbnd, 0,
                               I.nks, false, I.Cin.p, nullptr, s);
  LaunchLin<T>::proj_update(x, I.Aio.p, I.nbnd, I.ptot, I.Cin.p, I.nbnd, I.nbnd, I.npwx, I.nks,
                            nullptr, nullptr, nullptr, nullptr, nullptr, s, I.gemm);
}

// Lanczos step j: w_j = a LW + b w_{j-2} (j > 0), w_j <- P_c w_j, LW = L w_j,
// then beta_{j+1}, z_{j+1} from the fused sums.
template <typename T>
void lanczos_step(Instance& I, int j, hipStream_t s) {
  LzDevState* st = I.st.as<LzDevState>();
  void* X = (j & 1) ? I.X1.p : I.X0.p;
  input_side<T>(I, X, j > 0 ? I.LW.p : nullptr, j > 0, st, s);
  apply_core<T>(I, X, I.LW.p, (j & 1) != 0, st, s);
  output_side_nl<T>(I, I.LW.p, X, I.lzpart.as<double>(), st, s);
  STAGE(I, ST_LANCZOS, s,
        launch_lz_finalize(I.lzpart.as<double>(), I.nlzblk_nl, st, I.beta.as<double>(),
                           I.z.as<double>(), I.max_steps, kBreakdownTol, (double)I.nbnd, s));
}

// Non-Hermitian step j (Sec. 2.5).  Step 0 only takes ||y||.  Step j >= 1
// applies L^dagger to u^_{j-1} and L to v^_{j-1} (X/Y of parity (j-1) & 1, a
// lower vector for even j-1: L applies D to it and L^dagger D+K), and forms
// u^_j and v^_j in place of u^_{j-2}, v^_{j-2} on the output sides; the v
// formation also sums (u^_j, v^_j) and (y, v^_j) for the scalar decisions.
template <typename T>
void nh_step(Instance& I, int j, hipStream_t s) {
  LzDevState* st = I.st.as<LzDevState>();
  double* part = I.lzpart.as<double>();
  if (j == 0) {
    STAGE(I, ST_LANCZOS, s,
          launch_nh_norm<T>(I.y.p, I.wk.as<double>(), (int64_t)I.nbnd * I.npwx, I.nks, part, s);
          launch_nh_finalize(part, kNhNormBlocks, st, I.beta.as<double>(), I.gam.as<double>(),
                             I.z.as<double>(), I.max_steps, kBreakdownTol, (double)I.nbnd, s));
    return;
  }
  const int c = (j - 1) & 1;
  void* V = c ? I.X1.p : I.X0.p;
  void* Vn = c ? I.X0.p : I.X1.p;
  void* U = c ? I.Y1.p : I.Y0.p;
  void* Un = c ? I.Y0.p : I.Y1.p;
  const bool v_upper = c != 0;
  // u chain: L^dagger u^_{j-1}, then u^_j
  input_side<T>(I, U, nullptr, true, st, s);
  apply_core<T>(I, U, I.LU.p, !v_upper, st, s);
  STAGE(I, ST_PROJ, s,
        LaunchLin<T>::proj_dot(I.Aio.p, I.nbnd, I.ptot, I.LU.p, nullptr, I.nbnd, I.npwx, I.nks,
                               I.chunk, I.nchunk, I.dpartial.p, st, s, I.gemm);
        LaunchLin<T>::reduce_coef_out(I.dpartial.p, I.nchunk, I.Cin.p, I.Mkb.p, I.nbnd, I.nproj,
                                      I.nks, I.Cout.p, st, s);
        LaunchLin<T>::nh_form(false, I.LU.p, I.Aio.p, I.ptot, I.Cout.p, I.nbnd, I.npwx, I.nks, Un,
                              nullptr, nullptr, nullptr, nullptr, st, s, I.gemm));
  // v chain: L v^_{j-1}, then v^_j with the sums
  input_side<T>(I, V, nullptr, true, st, s);
  apply_core<T>(I, V, I.LW.p, v_upper, st, s);
  STAGE(I, ST_PROJ, s,
        LaunchLin<T>::proj_dot(I.Aio.p, I.nbnd, I.ptot, I.LW.p, nullptr, I.nbnd, I.npwx, I.nks,
                               I.chunk, I.nchunk, I.dpartial.p, st, s, I.gemm);
        LaunchLin<T>::reduce_coef_out(I.dpartial.p, I.nchunk, I.Cin.p, I.Mkb.p, I.nbnd, I.nproj,
                                      I.nks, I.Cout.p, st, s);
        LaunchLin<T>::nh_form(true, I.LW.p, I.Aio.p, I.ptot, I.Cout.p, I.nbnd, I.npwx, I.nks, Vn,
                              I.y.p, Un, I.wk.as<double>(), part, st, s, I.gemm));
  STAGE(I, ST_LANCZOS, s,
        launch_nh_finalize(part, I.nlzblk, st, I.beta.as<double>(), I.gam.as<double>(),
                           I.z.as<double>(), I.max_steps, kBreakdownTol, (double)I.nbnd, s));
}

template <typename T>
void any_step(Instance& I, int j, hipStream_t s) {
  if (I.nh) nh_step<T>(I, j, s);
  else lanczos_step<T>(I, j, s);
}

// Capture one odd step (D+K on the upper vector) and the following even step
// (D on the lower vector) as a graph.  Every step after the first has one of
// these two forms: the kernels read the step number and the update
// coefficients from the device state, so the same graph serves every pair.
void build_pair_graph(Instance& I, hipStream_t s) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  if (I.fp64) {
    any_step<double>(I, 1, s);
    any_step<double>(I, 2, s);
  } else {
    any_step<float>(I, 1, s);
    any_step<float>(I, 2, s);
  }
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || g == nullptr) fail(LZ_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&I.gpair, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    I.gpair = nullptr;
    fail(LZ_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
  }
}

// ---------------------------------------------------------------------------
// work-list launches over the instances of a context
// ---------------------------------------------------------------------------
// One kernel of a step, merged over the members of a group: the launch runs
// nblocks work items, item[b] naming the member and its block (lz_batch.h).
struct MergedLaunch {
  const void* fn = nullptr;
  dim3 block;
  size_t lds = 0;
  unsigned nblocks = 0;
  int stride = 0;
  DBuf tab, item;
  std::vector<unsigned char> args0;  // argument bytes of the first member (the kernel's P slot)
};

// Instances whose steps issue the same kernels (with the same block shapes),
// advanced together: the merged launches of a first step (j = 0, no update),
// an odd step (D+K on an upper vector) and an even step (D).
struct BatchGroup {
  std::vector<int> members;
  std::vector<std::unique_ptr<MergedLaunch>> plan[3];
};

int plan_of_step(int j) { return j == 0 ? 0 : (j & 1) ? 1 : 2; }

// The launches step j of instance I issues, recorded instead of run.  The
// recording runs inside a capture of the private stream s, so that anything
// issued around the recorder would land in the captured graph rather than on
// the device; a non-empty graph is an error.
std::vector<LaunchRec> record_step(Instance& I, int j, hipStream_t s) {
  std::vector<LaunchRec> rec;
  HIPC(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  t_launch_rec = &rec;
  try {
    if (I.fp64) lanczos_step<double>(I, j, s);
    else lanczos_step<float>(I, j, s);
  } catch (...) {
    t_launch_rec = nullptr;
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  t_launch_rec = nullptr;
  hipGraph_t g = nullptr;
  HIPC(hipStreamEndCapture(s, &g));
  size_t nodes = 0;
  const hipError_t e = hipGraphGetNodes(g, nullptr, &nodes);
  (void)hipGraphDestroy(g);
  HIPC(e);
  if (nodes != 0) fail(LZ_ERR_HIP, "a step issued work outside the launch recorder");
  return rec;
}

bool same_kernels(const std::vector<LaunchRec>& a, const std::vector<LaunchRec>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].fn != b[i].fn || a[i].fnb != b[i].fnb || a[i].block.x != b[i].block.x || a[i].block.y != b[i].block.y ||
        a[i].block.z != b[i].block.z || a[i].args.size() != b[i].args.size())
      return false;
  return true;
}

// Launch l of the recorded sequences of the members, merged.
std::unique_ptr<MergedLaunch> merge_launch(const std::vector<const std::vector<LaunchRec>*>& recs,
                                           size_t l) {
  auto m = std::make_unique<MergedLaunch>();
  const LaunchRec& r0 = (*recs[0])[l];
  if (!r0.fnb) fail(LZ_ERR_HIP, "a kernel of the step has no work-list form");
  m->fn = r0.fnb;
  m->block = r0.block;
  m->args0 = r0.args;
  m->stride = (int)((sizeof(BatchGrid) + r0.args.size() + 15) / 16 * 16);
  std::vector<unsigned char> tab(recs.size() * (size_t)m->stride, 0);
  std::vector<unsigned> item;
  for (size_t i = 0; i < recs.size(); ++i) {
    const LaunchRec& r = (*recs[i])[l];
    const BatchGrid g{(int)r.grid.x, (int)r.grid.y, (int)r.grid.z, 0};
    std::memcpy(tab.data() + i * m->stride, &g, sizeof(g));
    std::memcpy(tab.data() + i * m->stride + sizeof(g), r.args.data(), r.args.size());
    const uint64_t nb = (uint64_t)r.grid.x * r.grid.y * r.grid.z;
    if (nb > kBatchLocalMask) fail(LZ_ERR_ARG, "an instance's launch exceeds 2^24 blocks");
    for (unsigned b = 0; b < (unsigned)nb; ++b) item.push_back(((unsigned)i << 24) | b);
    m->lds = std::max(m->lds, r.lds);
  }
  m->nblocks = (unsigned)item.size();
  upload(m->tab, tab);
  upload(m->item, item);
  return m;
}

// Group the instances by the kernels of their three kinds of step and merge
// each group's launches (once, after the autotuner has fixed every launch
// configuration; the argument structs hold only buffers and sizes that do
// not change later, the step's coefficients are read from device state).
void build_batch(lz_ctx* c);

// ---------------------------------------------------------------------------
// launch configurations and the autotuner
// ---------------------------------------------------------------------------
struct LaunchCfg {
  int gemm;     // projector products: kGemmValu, kGemmMfma, kGemmBf16x3
  int chunk;    // plane waves per partial of a projector dot
  int nchunk;
  int nlzblk;   // blocks of the output update (Lanczos partial sums)
  int nlzblk_nl;  // the same for the update over the separable rows only
  int gsize;    // bands per group of the density pass
  int ngroups;
  int lds_planes;  // 1: LDS Stockham plane kernels in place of register lines / lane pairs
};

void set_cfg(Instance& I, const LaunchCfg& c) {
  I.grid.lds_planes = c.lds_planes;
  I.gemm = c.gemm;
  I.chunk = c.chunk;
  I.nchunk = c.nchunk;
  I.nlzblk = c.nlzblk;
  I.nlzblk_nl = c.nlzblk_nl;
  I.gsize = c.gsize;
  I.ngroups = c.ngroups;
}

LaunchCfg make_cfg(const Instance& I, int gemm, int gsize, int chunk = kProjChunk,
                   int lds_planes = 0) {
  LaunchCfg c;
  c.gemm = gemm;
  c.lds_planes = lds_planes;
  if (gemm != kGemmValu)
    c.chunk = I.fp64 ? LaunchLin<double>::mfma_chunk(I.ptot, I.nbnd, I.npwx, I.nks)
                     : LaunchLin<float>::mfma_chunk(I.ptot, I.nbnd, I.npwx, I.nks);
  else
    c.chunk = chunk;
  c.nchunk = (I.npwx + c.chunk - 1) / c.chunk;
  c.nlzblk = I.fp64 ? LaunchLin<double>::update_blocks(I.ptot, I.nbnd, I.npwx, I.nks, gemm)
                    : LaunchLin<float>::update_blocks(I.ptot, I.nbnd, I.npwx, I.nks, gemm);
  c.nlzblk_nl = I.fp64 ? LaunchLin<double>::update_blocks(I.nproj, I.nbnd, I.npwx, I.nks, gemm)
                       : LaunchLin<float>::update_blocks(I.nproj, I.nbnd, I.npwx, I.nks, gemm);
  c.gsize = std::max(1, std::min(gsize, I.nb));
  c.ngroups = (I.nb + c.gsize - 1) / c.gsize;
  return c;
}

// The heuristic configuration first:
//  - projector products on the matrix cores for many bands and rows (or as
//    asked; the split-bf16 precision always takes them);
//  - density band groups of about four blocks per compute unit, or on the
//    register-line kernels up to N = 48 one chunk of 192/N bands per block
//    (the block count is then a multiple of what the compute units hold at
//    once);
// then, for the autotuner, the other projector path (unless one was asked
// for), groups of twice the bands, on the vector ALU dot chunks of 128 and
// 256 plane waves, and the other schedule of the 2-D plane transforms
// (register lines or lane pairs against LDS Stockham passes) where both exist.
int heuristic_group(const Instance& I, int rn) {
  if (rn && rn < 64) return 192 / rn;
  if (rn || I.n3 >= 72) {
    // a band at a time per block (the lane-pair kernels of 96^2 planes, and
    // the LDS kernels of large planes, which add into their slice of the
    // group partial): groups of 8 bands give n3 x N_b/8 blocks, so that the
    // last round of blocks is not a small remainder of a few long blocks (the
    // group partials then take N_b/8 grids)
    return std::min(I.nb, 8);
  }
  // LDS kernels
  const int ng = std::max(1, std::min(I.nb, (1024 + I.n3 - 1) / I.n3));
  return (I.nb + ng - 1) / ng;
}

// Band-group size of a density pass whose blocks (one per z-plane and group)
// each take time in proportion to their bands, run in rounds of `slots`
// blocks: the fewest rounds x bands per block, plus a small cost per group
// for the partial the Hartree pass reads back (0.05 of a band's work; ties
// go to the larger group).  On the 48^3 cell in FP64 (128 band-k products,
// 3 blocks per compute unit) it picks 8: 768 blocks, one round.  Measured
// there: the density pass takes the same time for groups of 4 to 13 (it is
// not bound by the rounds), the Hartree pass reads fewer partials from
// larger groups (36 us at 8, 41 us at 4), and 16 (two rounds) is 1.5x slower.
int round_group(const Instance& I, int slots) {
  int best = 1;
  double best_t = 1e300;
  for (int g = 1; g <= std::min(I.nb, 16); ++g) {
    const int ng = (I.nb + g - 1) / g;
    const int64_t blocks = (int64_t)I.n3 * ng;
    const double t = (double)((blocks + slots - 1) / slots) * g + 0.05 * ng;
    if (t <= best_t + 1e-9) {
      best_t = t;
      best = g;
    }
  }
  return best;
}

std::vector<LaunchCfg> launch_candidates(Instance& I, const lz_options& opt) {
  const bool mc = opt.projector_gemm == LZ_GEMM_MFMA ||
                  (opt.projector_gemm == LZ_GEMM_AUTO && I.nbnd >= 32 && I.ptot >= 64);
  const int gemm0 = I.prec == LZ_FP32_SPLITBF16 ? kGemmBf16x3 : mc ? kGemmMfma : kGemmValu;
  // register-line / lane-pair kernels exist for this grid and precision?
  I.grid.lds_planes = 0;
  const int rn_reg = I.fp64 ? reg_plane_size<double>(I.grid) : reg_plane_size<float>(I.grid);
  const bool reg_avail = rn_reg != 0 || (I.fp64 && I.n1 == 48 && I.n2 == 48 && I.n3 == 48 &&
                                         I.grid.soff_c != nullptr);
  const int lds0 = opt.fft_planes == 2 ? 1 : 0;
  int g_reg = heuristic_group(I, rn_reg), g_lds = heuristic_group(I, 0);
  {
    // the LDS density pass: groups that fill whole rounds of the blocks the
    // device holds at once
    const int saved = I.grid.lds_planes;
    I.grid.lds_planes = 1;
    const int bpc = I.fp64 ? LaunchFft<double>::density_blocks_per_cu(I.grid)
                           : LaunchFft<float>::density_blocks_per_cu(I.grid);
    I.grid.lds_planes = saved;
    int dev = 0, ncu = 0;
    if (bpc > 0 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
      g_lds = round_group(I, bpc * ncu);
  }
  // where no register-line kernel exists, the density pass is the LDS one in both forms
  if (rn_reg == 0) g_reg = g_lds;
  int g0 = lds0 ? g_lds : g_reg;
  // a group size or a dot chunk the caller fixes replaces the heuristic and is not tuned
  if (opt.density_group_bands > 0) g0 = opt.density_group_bands;
  const int ch0 = opt.projector_chunk > 0 ? opt.projector_chunk : kProjChunk;
  std::vector<LaunchCfg> c{make_cfg(I, gemm0, g0, ch0, lds0)};
  if (!opt.autotune) return c;
  std::vector<int> gemms{gemm0};
  if (opt.projector_gemm == LZ_GEMM_AUTO && I.prec != LZ_FP32_SPLITBF16)
    gemms.push_back(gemm0 == kGemmValu ? kGemmMfma : kGemmValu);
  std::vector<int> sizes{g0}, chunks{ch0};
  if (opt.density_group_bands == 0) sizes.push_back(2 * g0);
  if (opt.projector_chunk == 0) chunks = {kProjChunk, 2 * kProjChunk, 4 * kProjChunk};
  for (int gm : gemms)
    for (int gs : sizes) {
      if (gs > I.nb && gs != g0) continue;
      for (int ch : chunks) {
        if (gm != kGemmValu && ch != ch0) continue;  // the matrix-core dot sizes its own
        if (gm == gemm0 && gs == g0 && ch == ch0) continue;
        c.push_back(make_cfg(I, gm, gs, ch, lds0));
      }
    }
  if (opt.fft_planes == 0 && reg_avail)
    c.push_back(make_cfg(I, gemm0, opt.density_group_bands > 0 ? g0 : g_lds, ch0, 1));
  return c;
}

// Time every candidate on D and D+K applications of the right-hand side
// (an untimed pair, then three trials of three pairs between events on the
// stream; a candidate's time is its fastest trial) and keep the heuristic
// configuration unless another is faster by more than 3 % (short timings
// vary by a few percent; a smaller margin let the choice flip between runs).
template <typename T>
void autotune(Instance& I, const std::vector<LaunchCfg>& cands, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  const size_t vb = (size_t)I.nvec * I.csz;
  float best = 0.f;
  size_t bi = 0;
  auto pair = [&]() {
    HIPC(hipMemcpyAsync(I.tin.p, I.y.p, vb, hipMemcpyDeviceToDevice, s));
    HIPC(hipMemcpyAsync(I.tin2.p, I.y.p, vb, hipMemcpyDeviceToDevice, s));
    apply_half<T>(I, I.tin.p, I.tout.p, false, s);
    apply_half<T>(I, I.tin2.p, I.tout2.p, true, s);
  };
  for (size_t i = 0; i < cands.size(); ++i) {
    set_cfg(I, cands[i]);
    pair();
    float t_min = 0.f;
    for (int trial = 0; trial < 3; ++trial) {
      HIPC(hipEventRecord(e0, s));
      for (int rep = 0; rep < 3; ++rep) pair();
      HIPC(hipEventRecord(e1, s));
      HIPC(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, e0, e1));
      if (trial == 0 || ms < t_min) t_min = ms;
    }
    if (i == 0 || t_min < 0.97f * best) {
      best = t_min;
      bi = i;
    }
  }
  set_cfg(I, cands[bi]);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// ---------------------------------------------------------------------------
// construction of one instance
// ---------------------------------------------------------------------------
template <typename T>
void build_device_tables(Instance& I, hipStream_t s, const std::vector<double>& evc_k_in) {
  // valence orbitals in real space: sphere (caller order) -> sticks -> planes
  DBuf uk;
  upload_cplx(I, uk, evc_k_in);
  LaunchFft<T>::zfft_inv(I.grid, uk.p, I.npwx, I.sa.p, I.map_k.as<int>(), I.nb, I.nbnd, nullptr, s);
  LaunchFft<T>::plane_to_real(I.grid, I.sa.p, I.ur.p, I.nb, s);
  // M = beta^H U per k (fixed overlaps of the separable projectors)
  if (I.nproj > 0) {
    const void* beta = (const char*)I.Aio.p + (size_t)I.nbnd * I.npwx * I.csz;
    LaunchLin<T>::proj_dot(beta, I.nproj, I.ptot, I.U.p, nullptr, I.nbnd, I.npwx, I.nks, I.chunk,
                           I.nchunk, I.dpartial.p, nullptr, s, I.gemm);
    LaunchLin<T>::reduce(I.dpartial.p, I.nchunk, I.nproj, I.nbnd, I.nks, I.Mkb.p, s);
  }
  // y = P_c (shifted u)
  project_c<T>(I, I.y.p, s);
  HIPC(hipStreamSynchronize(s));
}

std::unique_ptr<Instance> build_instance(const lz_system& sys, const lz_options& opt,
                                         hipStream_t s) {
  auto Ip = std::make_unique<Instance>();
  Instance& I = *Ip;
  I.prec = opt.prec;
  I.approx = opt.approx;
  I.nh = opt.algorithm == LZ_NON_HERMITIAN;
  I.fp64 = opt.prec == LZ_FP64;
  I.csz = I.fp64 ? 16 : 8;
  I.max_steps = opt.max_steps;
  // ---- validation
  for (int i = 0; i < 3; ++i)
    if (!valid_len(sys.nr[i])) fail(LZ_ERR_ARG, "nr[" + std::to_string(i) + "] must factor into 2,3,5 and lie in [2,128]");
  I.n1 = sys.nr[0]; I.n2 = sys.nr[1]; I.n3 = sys.nr[2];
  // only cubic grids are validated against the oracle (every workload here
  // is cubic); other shapes are refused rather than run unchecked
  if (I.n1 != I.n2 || I.n2 != I.n3) fail(LZ_ERR_ARG, "the FFT grid must be cubic (N1 = N2 = N3)");
  if (I.n1 * I.n2 > 36 * 256) fail(LZ_ERR_ARG, "N1*N2 exceeds 9216");
  I.N = I.n1 * I.n2 * I.n3;
  if (sys.nks < 1 || sys.nbnd < 1 || sys.nproj < 0 || sys.npwx < 1)
    fail(LZ_ERR_ARG, "nks, nbnd, npwx must be >= 1 and nproj >= 0");
  I.nks = sys.nks; I.nbnd = sys.nbnd; I.nproj = sys.nproj; I.npwx = sys.npwx;
  I.nb = I.nks * I.nbnd;
  if (!sys.xk || !sys.wk || !sys.npw_k || !sys.npw_kq || !sys.nl_k || !sys.nl_kq || !sys.evc_k ||
      !sys.evc_kq || !sys.et_k || !sys.vloc_r)
    fail(LZ_ERR_ARG, "a required array pointer is NULL");
  if (opt.approx == LZ_TDDFT && !sys.fxc_r) fail(LZ_ERR_ARG, "fxc_r is required for TDDFT");
  if (I.nproj > 0 && (!sys.vkb_kq || !sys.dkb)) fail(LZ_ERR_ARG, "vkb_kq and dkb are required when nproj > 0");
  const double* at = sys.at;
  const double det = at[0] * (at[4] * at[8] - at[5] * at[7]) - at[1] * (at[3] * at[8] - at[5] * at[6]) +
                     at[2] * (at[3] * at[7] - at[4] * at[6]);
  if (!(std::fabs(det) > 0)) fail(LZ_ERR_ARG, "lattice vectors are singular");
  I.omega = std::fabs(det);
  // reciprocal rows b_j: b = 2 pi inv(at)^T
  double bg[9];
  {
    double inv[9];
    inv[0] = (at[4] * at[8] - at[5] * at[7]) / det;
    inv[1] = -(at[1] * at[8] - at[2] * at[7]) / det;
    inv[2] = (at[1] * at[5] - at[2] * at[4]) / det;
    inv[3] = -(at[3] * at[8] - at[5] * at[6]) / det;
    inv[4] = (at[0] * at[8] - at[2] * at[6]) / det;
    inv[5] = -(at[0] * at[5] - at[2] * at[3]) / det;
    inv[6] = (at[3] * at[7] - at[4] * at[6]) / det;
    inv[7] = -(at[0] * at[7] - at[1] * at[6]) / det;
    inv[8] = (at[0] * at[4] - at[1] * at[3]) / det;
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) bg[j * 3 + c] = kTwoPi * inv[c * 3 + j];
  }
  auto gcart = [&](int m1, int m2, int m3, double* out) {
    for (int c = 0; c < 3; ++c) out[c] = m1 * bg[c] + m2 * bg[3 + c] + m3 * bg[6 + c];
  };
  double Q[3];
  gcart(sys.g0[0], sys.g0[1], sys.g0[2], Q);
  for (int c = 0; c < 3; ++c) Q[c] += sys.q[c];
  I.q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  if (!(I.q2 > 0)) fail(LZ_ERR_ARG, "Q = q + G0 must be nonzero");
  I.pref = 4.0 / I.omega;
  I.fq = 4.0 * M_PI / I.q2;
  double wsum = 0;
  for (int k = 0; k < I.nks; ++k) {
    if (!(sys.wk[k] >= 0)) fail(LZ_ERR_ARG, "negative k weight");
    wsum += sys.wk[k];
  }
  if (std::fabs(wsum - 1.0) > 1e-10) fail(LZ_ERR_ARG, "k weights must sum to 1");
  for (int k = 0; k < I.nks; ++k) {
    if (sys.npw_k[k] < 1 || sys.npw_k[k] > I.npwx || sys.npw_kq[k] < 1 || sys.npw_kq[k] > I.npwx)
      fail(LZ_ERR_ARG, "npw out of range [1, npwx]");
    if (sys.npw_kq[k] <= I.nbnd) fail(LZ_ERR_ARG, "npw_kq must exceed nbnd");
  }
  // ---- sticks: union of the (i1, i2) columns of every sphere
  auto split = [&](int idx, int& i1, int& i2, int& i3) {
    i3 = idx % I.n3;
    i2 = (idx / I.n3) % I.n2;
    i1 = idx / (I.n2 * I.n3);
  };
  std::vector<char> col(I.n1 * I.n2, 0);
  auto scan = [&](const int32_t* nl, const int32_t* npw) {
    for (int k = 0; k < I.nks; ++k) {
      std::vector<char> seen(I.N, 0);
      for (int i = 0; i < npw[k]; ++i) {
        const int idx = nl[(int64_t)k * I.npwx + i];
        if (idx < 0 || idx >= I.N) fail(LZ_ERR_ARG, "plane-wave index outside the grid");
        if (seen[idx]) fail(LZ_ERR_ARG, "duplicate plane wave in a sphere");
        seen[idx] = 1;
        int i1, i2, i3;
        split(idx, i1, i2, i3);
        col[i1 * I.n2 + i2] = 1;
      }
    }
  };
  scan(sys.nl_k, sys.npw_k);
  scan(sys.nl_kq, sys.npw_kq);
  std::vector<int> sid(I.n1 * I.n2, -1), si1, si2, act;
  std::vector<char> rowact(I.n1, 0);
  for (int c = 0; c < I.n1 * I.n2; ++c)
    if (col[c]) {
      sid[c] = (int)si1.size();
      si1.push_back(c / I.n2);
      si2.push_back(c % I.n2);
      rowact[c / I.n2] = 1;
    }
  for (int r = 0; r < I.n1; ++r)
    if (rowact[r]) act.push_back(r);
  I.S = (int)si1.size();
  I.nact = (int)act.size();
  // ---- internal (stick-major) order of the k+q spheres
  std::vector<int> perm((size_t)I.nks * I.npwx, 0), npwkq(I.nks);
  std::vector<int> map_kq((size_t)I.nks * I.S * I.n3, -1), map_k((size_t)I.nks * I.S * I.n3, -1);
  std::vector<double> kin((size_t)I.nks * I.npwx, 0.0);
  for (int k = 0; k < I.nks; ++k) {
    const int npw = sys.npw_kq[k];
    npwkq[k] = npw;
    std::vector<std::pair<int64_t, int>> key(npw);
    for (int i = 0; i < npw; ++i) {
      const int idx = sys.nl_kq[(int64_t)k * I.npwx + i];
      int i1, i2, i3;
      split(idx, i1, i2, i3);
      key[i] = {(int64_t)sid[i1 * I.n2 + i2] * I.n3 + i3, i};
    }
    std::sort(key.begin(), key.end());
    const double* xk = sys.xk + 3 * k;
    for (int ii = 0; ii < npw; ++ii) {
      const int i = key[ii].second;
      perm[(size_t)k * I.npwx + ii] = i;
      const int idx = sys.nl_kq[(int64_t)k * I.npwx + i];
      int i1, i2, i3;
      split(idx, i1, i2, i3);
      map_kq[((size_t)k * I.S + sid[i1 * I.n2 + i2]) * I.n3 + i3] = ii;
      double g[3];
      gcart(centred(i1, I.n1), centred(i2, I.n2), centred(i3, I.n3), g);
      double e = 0;
      for (int c = 0; c < 3; ++c) {
        const double v = xk[c] + sys.q[c] + g[c];
        e += v * v;
      }
      kin[(size_t)k * I.npwx + ii] = 0.5 * e;
    }
    for (int i = 0; i < sys.npw_k[k]; ++i) {
      const int idx = sys.nl_k[(int64_t)k * I.npwx + i];
      int i1, i2, i3;
      split(idx, i1, i2, i3);
      map_k[((size_t)k * I.S + sid[i1 * I.n2 + i2]) * I.n3 + i3] = i;
    }
  }
  // ---- complex arrays in internal order (interleaved doubles on the host)
  const size_t nv = (size_t)I.nks * I.nbnd * I.npwx;
  I.nvec = (int64_t)nv;
  std::vector<double> U(2 * nv, 0.0), Y(2 * nv, 0.0), EK(2 * nv, 0.0);
  for (int k = 0; k < I.nks; ++k) {
    // y_nk(G') = u_nk at the grid point G' - G0 (the grid product e^{iG0.r} u)
    std::unordered_map<int, int> kpos;
    for (int i = 0; i < sys.npw_k[k]; ++i) kpos[sys.nl_k[(int64_t)k * I.npwx + i]] = i;
    for (int n = 0; n < I.nbnd; ++n) {
      const size_t row = ((size_t)k * I.nbnd + n) * I.npwx;
      for (int ii = 0; ii < npwkq[k]; ++ii) {
        const int i = perm[(size_t)k * I.npwx + ii];
        U[2 * (row + ii)] = sys.evc_kq[2 * (row + i)];
        U[2 * (row + ii) + 1] = sys.evc_kq[2 * (row + i) + 1];
        const int idx = sys.nl_kq[(int64_t)k * I.npwx + i];
        int i1, i2, i3;
        split(idx, i1, i2, i3);
        const int j1 = ((i1 - sys.g0[0]) % I.n1 + I.n1) % I.n1;
        const int j2 = ((i2 - sys.g0[1]) % I.n2 + I.n2) % I.n2;
        const int j3 = ((i3 - sys.g0[2]) % I.n3 + I.n3) % I.n3;
        auto it = kpos.find((j1 * I.n2 + j2) * I.n3 + j3);
        if (it != kpos.end()) {
          Y[2 * (row + ii)] = sys.evc_k[2 * (row + it->second)];
          Y[2 * (row + ii) + 1] = sys.evc_k[2 * (row + it->second) + 1];
        }
      }
      for (int i = 0; i < sys.npw_k[k]; ++i) {
        EK[2 * (row + i)] = sys.evc_k[2 * (row + i)];
        EK[2 * (row + i) + 1] = sys.evc_k[2 * (row + i) + 1];
      }
    }
  }
  std::vector<double> VKB;
  std::vector<double> dkb(I.nproj);
  if (I.nproj > 0) {
    VKB.assign(2 * (size_t)I.nks * I.nproj * I.npwx, 0.0);
    for (int k = 0; k < I.nks; ++k)
      for (int p = 0; p < I.nproj; ++p) {
        const size_t row = ((size_t)k * I.nproj + p) * I.npwx;
        for (int ii = 0; ii < npwkq[k]; ++ii) {
          const int i = perm[(size_t)k * I.npwx + ii];
          VKB[2 * (row + ii)] = sys.vkb_kq[2 * (row + i)];
          VKB[2 * (row + ii) + 1] = sys.vkb_kq[2 * (row + i) + 1];
        }
      }
    for (int p = 0; p < I.nproj; ++p) dkb[p] = sys.dkb[p];
  }
  // ---- real-space grids in plane-major order [i3][i1][i2]; Hartree kernel
  std::vector<double> vl(I.N), fx(I.N, 0.0), kh(I.N, 0.0);
  bool singular = false;
  for (int i1 = 0; i1 < I.n1; ++i1)
    for (int i2 = 0; i2 < I.n2; ++i2)
      for (int i3 = 0; i3 < I.n3; ++i3) {
        const int src = (i1 * I.n2 + i2) * I.n3 + i3;
        const int dst = (i3 * I.n1 + i1) * I.n2 + i2;
        vl[dst] = sys.vloc_r[src];
        if (sys.fxc_r) fx[dst] = sys.fxc_r[src];
        double g[3];
        gcart(centred(i1, I.n1), centred(i2, I.n2), centred(i3, I.n3), g);
        double qg2 = 0;
        for (int c = 0; c < 3; ++c) {
          const double v = sys.q[c] + g[c];
          qg2 += v * v;
        }
        if (qg2 == 0.0) singular = true;
        else kh[dst] = 4.0 * M_PI / (qg2 * (double)I.N);
      }
  if (singular && I.approx != LZ_IPA) fail(LZ_ERR_ARG, "q + G = 0 on the grid: the Hartree kernel is singular");
  // ---- fingerprint of the operator (refuses checkpoints of another one)
  {
    Fingerprint f;
    f.word(((uint64_t)I.n1 << 40) | ((uint64_t)I.n2 << 20) | (uint64_t)I.n3);
    f.word(((uint64_t)I.nks << 32) | (uint64_t)I.nbnd);
    f.word(((uint64_t)I.nproj << 32) | (uint64_t)I.npwx);
    f.word((uint64_t)I.approx);
    f.scalar(I.omega);
    f.scalar(I.q2);
    f.array(perm);
    f.array(map_kq);
    f.array(map_k);
    f.array(kin);
    f.array(U);
    f.array(Y);
    f.array(EK);
    f.array(VKB);
    f.array(dkb);
    f.array(vl);
    if (I.approx == LZ_TDDFT) f.array(fx);
    if (I.approx != LZ_IPA) f.array(kh);
    f.array(std::vector<double>(sys.et_k, sys.et_k + I.nb));
    f.array(std::vector<double>(sys.wk, sys.wk + I.nks));
    I.fingerprint = f.h;
  }
  // ---- plans
  std::vector<double> tr, ti;
  FftPlan p1, p2, p3;
  std::vector<double> tws[3];
  int lens[3] = {I.n1, I.n2, I.n3};
  FftPlan* plans[3] = {&p1, &p2, &p3};
  DBuf* twb[3] = {&I.tw1, &I.tw2, &I.tw3};
  for (int a = 0; a < 3; ++a) {
    tr.clear(); ti.clear();
    if (!make_plan(lens[a], *plans[a], tr, ti)) fail(LZ_ERR_ARG, "unsupported FFT length");
    std::vector<double> il(2 * tr.size());
    for (size_t i = 0; i < tr.size(); ++i) { il[2 * i] = tr[i]; il[2 * i + 1] = ti[i]; }
    upload_cplx(I, *twb[a], il);
  }
  // ---- device uploads
  upload(I.si1, si1);
  upload(I.si2, si2);
  upload(I.act, act);
  upload(I.map_kq, map_kq);
  upload(I.map_k, map_k);
  upload(I.perm, perm);
  upload(I.npw_kq, npwkq);
  upload_real(I, I.kin, kin);
  std::vector<double> eps(sys.et_k, sys.et_k + I.nb), wk(sys.wk, sys.wk + I.nks), bw(I.nb);
  for (int b = 0; b < I.nb; ++b) bw[b] = 4.0 * wk[b / I.nbnd] / I.omega;
  upload(I.eps, eps);
  upload(I.wk, wk);
  upload(I.bandw, bw);
  upload_real(I, I.vloc, vl);
  upload_real(I, I.fxc, fx);
  upload_real(I, I.khart, kh);
  upload_cplx(I, I.U, U);
  upload_cplx(I, I.y, Y);
  // stacked rows per k: U (nbnd rows) then beta (nproj rows)
  I.ptot = I.nbnd + I.nproj;
  {
    std::vector<double> A(2 * (size_t)I.nks * I.ptot * I.npwx, 0.0);
    for (int k = 0; k < I.nks; ++k) {
      for (int n = 0; n < I.nbnd; ++n)
        std::memcpy(&A[2 * (((size_t)k * I.ptot + n) * I.npwx)], &U[2 * (((size_t)k * I.nbnd + n) * I.npwx)],
                    2 * sizeof(double) * I.npwx);
      for (int p = 0; p < I.nproj; ++p)
        std::memcpy(&A[2 * (((size_t)k * I.ptot + I.nbnd + p) * I.npwx)],
                    &VKB[2 * (((size_t)k * I.nproj + p) * I.npwx)], 2 * sizeof(double) * I.npwx);
    }
    upload_cplx(I, I.Aio, A);
  }
  if (I.nproj > 0) upload(I.dkb, dkb);
  else I.dkb.alloc(sizeof(double));
  I.grid.n1 = I.n1; I.grid.n2 = I.n2; I.grid.n3 = I.n3;
  I.grid.S = I.S; I.grid.nact = I.nact; I.grid.pitch2 = I.n2 + 1;
  I.grid.si1 = I.si1.as<int>(); I.grid.si2 = I.si2.as<int>(); I.grid.act = I.act.as<int>();
  I.grid.p1 = p1; I.grid.p2 = p2; I.grid.p3 = p3;
  I.grid.tw1 = I.tw1.p; I.grid.tw2 = I.tw2.p; I.grid.tw3 = I.tw3.p;
  // row tables of the register-line plane kernels (cubic grids up to 96)
  I.grid.soff_f = nullptr;
  I.grid.soff_c = nullptr;
  I.grid.lds_planes = 0;
  for (int i = 0; i < 128; ++i) I.grid.slot[i] = -1;
  if (I.n1 == I.n2 && I.n2 == I.n3 && I.n1 <= 96) {
    const int pitch = I.n1 + 1;
    for (int a = 0; a < I.nact; ++a) I.grid.slot[act[a]] = (signed char)a;
    std::vector<int> sf(I.S), sc(I.S);
    for (int t = 0; t < I.S; ++t) {
      sf[t] = si1[t] * pitch + si2[t];
      sc[t] = I.grid.slot[si1[t]] * pitch + si2[t];
    }
    upload(I.soff_f, sf);
    upload(I.soff_c, sc);
    I.grid.soff_f = I.soff_f.as<int>();
    I.grid.soff_c = I.soff_c.as<int>();
  }
  // ---- work buffers
  const size_t vb = nv * I.csz;
  I.X0.alloc(vb); I.X1.alloc(vb); I.LW.alloc(vb);
  I.tin.alloc(vb); I.tout.alloc(vb); I.tin2.alloc(vb); I.tout2.alloc(vb);
  I.sa.alloc((size_t)I.nb * I.n3 * I.S * I.csz);
  I.sb.alloc((size_t)I.nb * I.n3 * I.S * I.csz);
  I.ur.alloc((size_t)I.nb * I.N * I.csz);
  // launch configurations: the heuristic default first, then (autotune)
  // the alternatives; buffers are sized for every candidate
  std::vector<LaunchCfg> cands = launch_candidates(I, opt);
  int max_groups = 0, max_chunks = 0, max_blk = kNhNormBlocks;
  for (const LaunchCfg& c : cands) {
    max_groups = std::max(max_groups, c.ngroups);
    max_chunks = std::max(max_chunks, c.nchunk);
    max_blk = std::max(max_blk, std::max(c.nlzblk, c.nlzblk_nl));
  }
  set_cfg(I, cands[0]);
  I.dpart.alloc((size_t)max_groups * I.N * I.csz);
  I.nr.alloc((size_t)I.N * I.csz);
  I.work.alloc((size_t)I.N * I.csz);
  I.vp.alloc((size_t)I.N * I.csz);
  I.dpartial.alloc((size_t)I.nks * max_chunks * I.ptot * I.nbnd * I.csz);
  I.Cin.alloc((size_t)I.nks * I.ptot * I.nbnd * I.csz);
  I.Cout.alloc((size_t)I.nks * I.ptot * I.nbnd * I.csz);
  I.Mkb.alloc((size_t)I.nks * std::max(1, I.nproj) * I.nbnd * I.csz);
  I.lzpart.alloc((size_t)max_blk * 4 * sizeof(double));
  I.st.alloc(sizeof(LzDevState));
  I.beta.alloc((size_t)I.max_steps * sizeof(double));
  I.z.alloc((size_t)I.max_steps * 2 * sizeof(double));
  if (I.nh) {
    I.Y0.alloc(vb); I.Y1.alloc(vb); I.LU.alloc(vb);
    I.gam.alloc((size_t)I.max_steps * 2 * sizeof(double));
  }
  if (I.fp64) build_device_tables<double>(I, s, EK);
  else build_device_tables<float>(I, s, EK);
  if (opt.autotune && cands.size() > 1) {
    if (I.fp64) autotune<double>(I, cands, s);
    else autotune<float>(I, cands, s);
  }
  return Ip;
}

}  // namespace

struct lz_ctx {
  int device = 0;
  double* scratch = nullptr;  // device address of this device's staging area
  hipStream_t user = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // streams on which lz_step runs the instances side by side (empty: every
  // instance on `stream`, one after another); instance i uses qs[i % size]
  std::vector<hipStream_t> qs;
  std::vector<hipEvent_t> qdone;
  hipEvent_t ev_fork = nullptr;
  lz_options opt{};
  std::vector<std::unique_ptr<Instance>> inst;
  bool started = false;
  // work-list launches (opt.batched): groups of instances and their merged
  // steps, built at the first batched lz_step
  std::vector<std::unique_ptr<BatchGroup>> groups;
  bool batch_built = false;
  hipStream_t capture = nullptr;  // private stream of the launch recorder
  hipGraphExec_t batch_pair = nullptr;  // a pair of batched steps (use_graph)
  ~lz_ctx() {
    if (batch_pair) (void)hipGraphExecDestroy(batch_pair);
    groups.clear();
    inst.clear();
    if (capture) (void)hipStreamDestroy(capture);
    for (auto e : qdone) (void)hipEventDestroy(e);
    for (auto q : qs) (void)hipStreamDestroy(q);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
  }
  // order the private stream after the caller's stream
  void enter() {
    HIPC(hipEventRecord(ev_in, user));
    HIPC(hipStreamWaitEvent(stream, ev_in, 0));
  }
  void leave() {
    HIPC(hipEventRecord(ev_out, stream));
    HIPC(hipStreamWaitEvent(user, ev_out, 0));
  }
};

namespace {

template <typename F>
lz_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return LZ_OK;
  } catch (const LzError& e) {
    g_last_error = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LZ_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown failure";
    return LZ_ERR_HIP;
  }
}

// Device address of the staging area on the current device, looked up once
// per device (the first lz_init on it) and kept until the process ends.
double* scratch_address(int device) {
  static std::mutex mu;
  static double* addr[64] = {nullptr};
  if (device < 0 || device >= 64) fail(LZ_ERR_ARG, "device index beyond 63");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(LZ_ERR_HIP, "no device address for the staging area");
    addr[device] = static_cast<double*>(p);
  }
  return addr[device];
}

void start_recursion(lz_ctx* c) {
  for (auto& ip : c->inst) {
    Instance& I = *ip;
    launch_set_state(I.st.as<LzDevState>(), c->stream);
    HIPC(hipMemcpyAsync(I.X0.p, I.y.p, (size_t)I.nvec * I.csz, hipMemcpyDeviceToDevice, c->stream));
    HIPC(hipMemsetAsync(I.X1.p, 0, (size_t)I.nvec * I.csz, c->stream));
    if (I.nh) {
      HIPC(hipMemcpyAsync(I.Y0.p, I.y.p, (size_t)I.nvec * I.csz, hipMemcpyDeviceToDevice, c->stream));
      HIPC(hipMemsetAsync(I.Y1.p, 0, (size_t)I.nvec * I.csz, c->stream));
    }
    I.steps_host = 0;
    I.status_host = 0;
  }
  c->started = true;
}

void read_state(lz_ctx* c) {
  HIPC(hipStreamSynchronize(c->stream));
  for (auto& ip : c->inst) {
    ip->timer.collect();
    LzDevState h;
    HIPC(hipMemcpy(&h, ip->st.p, sizeof(h), hipMemcpyDeviceToHost));
    ip->steps_host = h.step;
    ip->status_host = h.status;
  }
}

void build_batch(lz_ctx* c) {
  c->groups.clear();
  if (!c->capture) HIPC(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  const int ni = (int)c->inst.size();
  std::vector<std::vector<LaunchRec>> rec[3];
  for (int k = 0; k < 3; ++k) rec[k].resize(ni);
  for (int i = 0; i < ni; ++i)
    for (int k = 0; k < 3; ++k) rec[k][i] = record_step(*c->inst[i], k, c->capture);
  std::vector<int> group_of(ni, -1);
  for (int i = 0; i < ni; ++i) {
    for (size_t g = 0; g < c->groups.size() && group_of[i] < 0; ++g) {
      const int r = c->groups[g]->members[0];
      if ((int)c->groups[g]->members.size() < kBatchMaxInst && same_kernels(rec[0][i], rec[0][r]) &&
          same_kernels(rec[1][i], rec[1][r]) && same_kernels(rec[2][i], rec[2][r])) {
        c->groups[g]->members.push_back(i);
        group_of[i] = (int)g;
      }
    }
    if (group_of[i] < 0) {
      c->groups.push_back(std::make_unique<BatchGroup>());
      c->groups.back()->members.push_back(i);
      group_of[i] = (int)c->groups.size() - 1;
    }
  }
  for (auto& gp : c->groups) {
    for (int k = 0; k < 3; ++k) {
      std::vector<const std::vector<LaunchRec>*> recs;
      for (int i : gp->members) recs.push_back(&rec[k][i]);
      for (size_t l = 0; l < recs[0]->size(); ++l) gp->plan[k].push_back(merge_launch(recs, l));
    }
  }
  c->batch_built = true;
}

// One step of every member of group g (all at step j) on stream s.
void batched_step(const BatchGroup& g, int j, hipStream_t s) {
  for (const auto& m : g.plan[plan_of_step(j)]) {
    if (m->nblocks == 0) continue;
    BatchRef br{m->tab.as<unsigned char>(), m->item.as<unsigned>(), m->stride, 0};
    void* args[2] = {const_cast<unsigned char*>(m->args0.data()), &br};
    HIPC(hipLaunchKernel(m->fn, dim3(m->nblocks), m->block, args, m->lds, s));
  }
}

// The work-list path serves a step of the pseudo-Hermitian recursion when
// every running instance is at the same step and no stage timer is on.
bool batch_applies(const lz_ctx* c) {
  if (!c->opt.batched) return false;
  int j = -1;
  for (const auto& ip : c->inst) {
    if (ip->nh || ip->timer.on) return false;
    if (ip->status_host != 0) continue;
    if (j >= 0 && ip->steps_host != j) return false;
    j = ip->steps_host;
  }
  return true;
}

}  // namespace

extern "C" {

lz_status lz_init(const lz_system* sys, int32_t n_inst, const lz_options* opt, int32_t device,
                  void* hip_stream, lz_ctx** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!sys || !opt || !out) fail(LZ_ERR_ARG, "null argument");
    if (n_inst < 1) fail(LZ_ERR_ARG, "n_inst must be >= 1");
    if (opt->max_steps < 1) fail(LZ_ERR_ARG, "max_steps must be >= 1");
    if (opt->autotune != 0 && opt->autotune != 1) fail(LZ_ERR_ARG, "autotune must be 0 or 1");
    if (opt->prec != LZ_FP64 && opt->prec != LZ_FP32 && opt->prec != LZ_FP32_SPLITBF16)
      fail(LZ_ERR_ARG, "unknown precision");
    if (opt->approx != LZ_TDDFT && opt->approx != LZ_RPA && opt->approx != LZ_IPA)
      fail(LZ_ERR_ARG, "unknown approximation");
    if (opt->algorithm != LZ_PSEUDO_HERMITIAN && opt->algorithm != LZ_NON_HERMITIAN)
      fail(LZ_ERR_ARG, "unknown Lanczos algorithm");
    if (opt->streams < 0 || opt->streams > 64) fail(LZ_ERR_ARG, "streams must lie in [0, 64]");
    if (opt->projector_gemm != LZ_GEMM_AUTO && opt->projector_gemm != LZ_GEMM_VALU &&
        opt->projector_gemm != LZ_GEMM_MFMA)
      fail(LZ_ERR_ARG, "unknown projector_gemm");
    if (opt->density_group_bands < 0) fail(LZ_ERR_ARG, "density_group_bands must be >= 0");
    if (opt->batched != 0 && opt->batched != 1) fail(LZ_ERR_ARG, "batched must be 0 or 1");
    if (opt->fft_planes < 0 || opt->fft_planes > 2) fail(LZ_ERR_ARG, "fft_planes must be 0, 1 or 2");
    if (opt->projector_chunk != 0 && opt->projector_chunk != kProjChunk &&
        opt->projector_chunk != 2 * kProjChunk && opt->projector_chunk != 4 * kProjChunk)
      fail(LZ_ERR_ARG, "projector_chunk must be 0, 64, 128 or 256");
    int ndev = 0;
    HIPC(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(LZ_ERR_ARG, "no such device");
    HIPC(hipSetDevice(device));
    auto c = std::make_unique<lz_ctx>();
    c->device = device;
    c->scratch = scratch_address(device);
    c->opt = *opt;
    c->user = (hipStream_t)hip_stream;
    HIPC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIPC(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIPC(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    {
      const int nq = std::min(n_inst, opt->streams > 0 ? (int)opt->streams : kInstStreams);
      if (nq > 1) {
        HIPC(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        for (int i = 0; i < nq; ++i) {
          hipStream_t q = nullptr;
          hipEvent_t e = nullptr;
          HIPC(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
          c->qs.push_back(q);
          HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
          c->qdone.push_back(e);
        }
      }
    }
    HIPC(enable_large_lds_fft<double>());
    HIPC(enable_large_lds_fft<float>());
    c->enter();
    for (int i = 0; i < n_inst; ++i) c->inst.push_back(build_instance(sys[i], *opt, c->stream));
    start_recursion(c.get());
    c->leave();
    HIPC(hipStreamSynchronize(c->stream));
    *out = c.release();
  });
}

lz_status lz_apply_liouvillian(lz_ctx* c, const void* q_in, const void* p_in, void* q_out,
                               void* p_out) {
  return guarded([&] {
    if (!c) fail(LZ_ERR_ARG, "null context");
    if ((q_in == nullptr) != (p_out == nullptr) || (p_in == nullptr) != (q_out == nullptr))
      fail(LZ_ERR_ARG, "each half needs both its input and its output (or neither)");
    HIPC(hipSetDevice(c->device));
    c->enter();
    // instances side by side on their streams, as in lz_step
    const bool fork = !c->qs.empty();
    if (fork) {
      HIPC(hipEventRecord(c->ev_fork, c->stream));
      for (auto q : c->qs) HIPC(hipStreamWaitEvent(q, c->ev_fork, 0));
    }
    size_t off = 0;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
      Instance& I = *c->inst[ii];
      hipStream_t sq = fork ? c->qs[ii % c->qs.size()] : c->stream;
      const size_t bytes_off = off * I.csz;
      auto at = [&](const void* p) { return p ? (const char*)p + bytes_off : nullptr; };
      auto atw = [&](void* p) { return p ? (char*)p + bytes_off : nullptr; };
      const void* qi = at(q_in);
      const void* pi = at(p_in);
      void* qo = atw(q_out);
      void* po = atw(p_out);
      if (I.fp64) {
        if (pi) {
          LaunchLin<double>::perm_in(pi, I.tin.p, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
          apply_half<double>(I, I.tin.p, I.tout.p, false, sq);
          LaunchLin<double>::perm_out(I.tout.p, qo, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
        }
        if (qi) {
          LaunchLin<double>::perm_in(qi, I.tin2.p, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
          apply_half<double>(I, I.tin2.p, I.tout2.p, true, sq);
          LaunchLin<double>::perm_out(I.tout2.p, po, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
        }
      } else {
        if (pi) {
          LaunchLin<float>::perm_in(pi, I.tin.p, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
          apply_half<float>(I, I.tin.p, I.tout.p, false, sq);
          LaunchLin<float>::perm_out(I.tout.p, qo, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
        }
        if (qi) {
          LaunchLin<float>::perm_in(qi, I.tin2.p, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
          apply_half<float>(I, I.tin2.p, I.tout2.p, true, sq);
          LaunchLin<float>::perm_out(I.tout2.p, po, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, sq);
        }
      }
      off += (size_t)I.nvec;
    }
    if (fork) {
      for (size_t q = 0; q < c->qs.size(); ++q) {
        HIPC(hipEventRecord(c->qdone[q], c->qs[q]));
        HIPC(hipStreamWaitEvent(c->stream, c->qdone[q], 0));
      }
    }
    HIPC(hipGetLastError());
    c->leave();
  });
}

lz_status lz_reset(lz_ctx* c) {
  return guarded([&] {
    if (!c) fail(LZ_ERR_ARG, "null context");
    HIPC(hipSetDevice(c->device));
    c->enter();
    start_recursion(c);
    HIPC(hipGetLastError());
    c->leave();
  });
}

lz_status lz_step(lz_ctx* c, int32_t n_steps, int32_t* steps_done) {
  lz_status ret = LZ_OK;
  lz_status g = guarded([&] {
    if (!c) fail(LZ_ERR_ARG, "null context");
    if (n_steps < 0) fail(LZ_ERR_ARG, "n_steps must be >= 0");
    HIPC(hipSetDevice(c->device));
    for (auto& ip : c->inst)
      if (ip->status_host == 0 && ip->steps_host + n_steps > ip->max_steps)
        fail(LZ_ERR_STATE, "max_steps would be exceeded");
    c->enter();
    const int ni = (int)c->inst.size();
    if (batch_applies(c)) {
      // work-list launches: one launch per kernel of the step over every
      // member of a group (groups side by side on the context's streams)
      if (!c->batch_built) build_batch(c);
      int j0 = -1;
      for (auto& ip : c->inst)
        if (ip->status_host == 0) j0 = ip->steps_host;
      const int ng = (int)c->groups.size();
      const bool gfork = ng > 1 && !c->qs.empty();
      // steps j .. j + n - 1 of every group, forked from and joined back to
      // the context stream
      auto issue = [&](int j, int n) {
        if (gfork) {
          HIPC(hipEventRecord(c->ev_fork, c->stream));
          for (auto q : c->qs) HIPC(hipStreamWaitEvent(q, c->ev_fork, 0));
        }
        for (int jj = j; jj < j + n; ++jj)
          for (int g = 0; g < ng; ++g)
            batched_step(*c->groups[g], jj, gfork ? c->qs[g % c->qs.size()] : c->stream);
        if (gfork) {
          for (size_t q = 0; q < c->qs.size(); ++q) {
            HIPC(hipEventRecord(c->qdone[q], c->qs[q]));
            HIPC(hipStreamWaitEvent(c->stream, c->qdone[q], 0));
          }
        }
      };
      const int end = j0 + n_steps;
      for (int j = j0; j0 >= 0 && j < end;) {
        if (c->opt.use_graph && (j & 1) && j + 1 < end) {
          // an odd and an even step of every group as one captured graph
          // (the kernels read the step from the device state: one graph
          // serves every pair)
          if (!c->batch_pair) {
            hipGraph_t gr = nullptr;
            HIPC(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
            issue(1, 2);
            HIPC(hipStreamEndCapture(c->stream, &gr));
            const hipError_t ei = hipGraphInstantiate(&c->batch_pair, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (ei != hipSuccess) {
              c->batch_pair = nullptr;
              fail(LZ_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
            }
          }
          HIPC(hipGraphLaunch(c->batch_pair, c->stream));
          j += 2;
        } else {
          issue(j, 1);
          ++j;
        }
      }
    } else {
    // With several streams the instances advance side by side: their steps
    // are issued round-robin, one unit (a step or a replayed pair) per
    // instance per round, each instance on its own stream, so the small
    // kernels of one instance overlap with the work of the others.
    const bool fork = !c->qs.empty();
    if (fork) {
      HIPC(hipEventRecord(c->ev_fork, c->stream));
      for (auto q : c->qs) HIPC(hipStreamWaitEvent(q, c->ev_fork, 0));
    }
    std::vector<int> jj(ni), end(ni);
    for (int i = 0; i < ni; ++i) {
      jj[i] = c->inst[i]->steps_host;
      end[i] = c->inst[i]->status_host == 0 ? jj[i] + n_steps : jj[i];
    }
    // one unit of instance i on stream s; returns false when it has none left
    auto issue = [&](int i, hipStream_t s) {
      Instance& I = *c->inst[i];
      int& j = jj[i];
      if (j >= end[i]) return false;
      const bool graphs = c->opt.use_graph != 0 && !I.timer.on;
      if (graphs && (j & 1) && j + 1 < end[i]) {
        if (!I.gpair) build_pair_graph(I, s);
        HIPC(hipGraphLaunch(I.gpair, s));
        j += 2;
      } else {
        if (I.fp64) any_step<double>(I, j, s);
        else any_step<float>(I, j, s);
        ++j;
      }
      return true;
    };
    if (fork) {
      for (bool more = true; more;) {
        more = false;
        for (int i = 0; i < ni; ++i) more |= issue(i, c->qs[i % c->qs.size()]);
      }
      for (size_t q = 0; q < c->qs.size(); ++q) {
        HIPC(hipEventRecord(c->qdone[q], c->qs[q]));
        HIPC(hipStreamWaitEvent(c->stream, c->qdone[q], 0));
      }
    } else {
      for (int i = 0; i < ni; ++i)
        while (issue(i, c->stream)) {
        }
    }
    }
    HIPC(hipGetLastError());
    c->leave();
    read_state(c);
    for (auto& ip : c->inst) {
      if (ip->status_host == 4 || ip->status_host == 7) ret = LZ_ERR_NOT_PD;
      else if (ip->status_host == 6 && ret == LZ_OK) ret = LZ_BREAKDOWN;
    }
    if (steps_done) *steps_done = c->inst[0]->steps_host;
    if (ret == LZ_ERR_NOT_PD) g_last_error = "beta^2 <= 0 or non-finite: the metric is not positive definite";
    if (ret == LZ_BREAKDOWN) g_last_error = "Krylov space exhausted (lucky breakdown)";
  });
  if (g != LZ_OK) return g;
  return ret;
}

lz_status lz_get_state(lz_ctx* c, int32_t inst, int32_t* steps_done, int32_t* status) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    if (steps_done) *steps_done = I.steps_host;
    if (status) *status = I.status_host == 0 ? 0 : (I.status_host == 6 ? LZ_BREAKDOWN : LZ_ERR_NOT_PD);
  });
}

lz_status lz_get_coefficients(lz_ctx* c, int32_t inst, int32_t first, int32_t count, double* beta,
                              double* gamma, double* z) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    if (first < 0 || count < 0) fail(LZ_ERR_ARG, "negative range");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    if (first + count > I.steps_host) fail(LZ_ERR_STATE, "coefficients not computed yet");
    if (gamma && I.nh) fail(LZ_ERR_ARG, "gamma is complex in the non-Hermitian recursion: use lz_get_gamma");
    if (count == 0) return;
    if (beta) HIPC(hipMemcpy(beta, I.beta.as<double>() + first, count * sizeof(double), hipMemcpyDeviceToHost));
    if (gamma) HIPC(hipMemcpy(gamma, I.beta.as<double>() + first, count * sizeof(double), hipMemcpyDeviceToHost));
    if (z) HIPC(hipMemcpy(z, I.z.as<double>() + 2 * first, 2 * count * sizeof(double), hipMemcpyDeviceToHost));
  });
}

lz_status lz_get_tuning(lz_ctx* c, int32_t inst, int32_t* projector_gemm,
                        int32_t* density_group_bands, int32_t* projector_chunks,
                        int32_t* fft_planes) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    const Instance& I = *c->inst[inst];
    if (fft_planes) *fft_planes = I.grid.lds_planes ? 2 : 1;
    if (projector_gemm) *projector_gemm = I.gemm == kGemmValu ? LZ_GEMM_VALU : LZ_GEMM_MFMA;
    if (density_group_bands) *density_group_bands = I.gsize;
    if (projector_chunks) *projector_chunks = I.nchunk;
  });
}

lz_status lz_launch_plan(int32_t n, int32_t prec, int32_t nbnd, int32_t nks, int32_t npwx,
                         int32_t nproj, int32_t slots, int32_t* out) {
  return guarded([&] {
    if (!out) fail(LZ_ERR_ARG, "out is NULL");
    if (!valid_len(n)) fail(LZ_ERR_ARG, "n must factor into 2,3,5 and lie in [2,128]");
    if (n * n > 36 * 256) fail(LZ_ERR_ARG, "N1*N2 exceeds 9216");
    if (prec != LZ_FP64 && prec != LZ_FP32 && prec != LZ_FP32_SPLITBF16)
      fail(LZ_ERR_ARG, "unknown precision");
    if (nks < 1 || nbnd < 1 || nproj < 0 || npwx < 1)
      fail(LZ_ERR_ARG, "nks, nbnd, npwx must be >= 1 and nproj >= 0");
    if ((int64_t)nks * nbnd > (1 << 24) || (int64_t)nbnd + nproj > (1 << 24))
      fail(LZ_ERR_ARG, "band or projector counts too large");
    if (slots < 0) fail(LZ_ERR_ARG, "slots must be >= 0");
    // the fields of an instance the host-side helpers read; nothing else is set
    Instance I;
    I.prec = (lz_precision)prec;
    I.fp64 = prec == LZ_FP64;
    I.n1 = I.n2 = I.n3 = n;
    I.N = n * n * n;
    I.nks = nks;
    I.nbnd = nbnd;
    I.nproj = nproj;
    I.npwx = npwx;
    I.nb = nks * nbnd;
    I.ptot = nbnd + nproj;
    const int ct = ct_supported(n) ? n : 0;
    const int rn = ct ? (I.fp64 ? reg_plane_len<double>(ct) : reg_plane_len<float>(ct)) : 0;
    // as launch_candidates: the LDS form by the round rule where the slots
    // are known, the register form's own heuristic where it exists
    const int g_lds = slots > 0 ? round_group(I, slots) : heuristic_group(I, 0);
    out[0] = ct;
    out[1] = rn;
    out[2] = rn ? heuristic_group(I, rn) : g_lds;
    out[3] = g_lds;
    out[4] = slots > 0 ? round_group(I, slots) : 0;
    const LaunchCfg v = make_cfg(I, kGemmValu, out[2]);
    const LaunchCfg m = make_cfg(I, prec == LZ_FP32_SPLITBF16 ? kGemmBf16x3 : kGemmMfma, out[2]);
    out[5] = v.chunk;
    out[6] = v.nchunk;
    out[7] = v.nlzblk;
    out[8] = v.nlzblk_nl;
    out[9] = m.chunk;
    out[10] = m.nchunk;
    out[11] = m.nlzblk;
    out[12] = m.nlzblk_nl;
    out[13] = v.gsize;
    out[14] = v.ngroups;
  });
}

lz_status lz_get_gamma(lz_ctx* c, int32_t inst, int32_t first, int32_t count, double* gamma) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    if (first < 0 || count < 0) fail(LZ_ERR_ARG, "negative range");
    if (count > 0 && !gamma) fail(LZ_ERR_ARG, "null gamma");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    if (first + count > I.steps_host) fail(LZ_ERR_STATE, "coefficients not computed yet");
    if (count == 0) return;
    if (I.nh) {
      HIPC(hipMemcpy(gamma, I.gam.as<double>() + 2 * first, 2 * count * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      std::vector<double> b(count);
      HIPC(hipMemcpy(b.data(), I.beta.as<double>() + first, count * sizeof(double), hipMemcpyDeviceToHost));
      for (int i = 0; i < count; ++i) { gamma[2 * i] = b[i]; gamma[2 * i + 1] = 0.0; }
    }
  });
}

lz_status lz_spectrum_ext(lz_ctx* c, int32_t inst, int32_t m0, int32_t m,
                          int32_t extrapolation, const double* omega, int32_t n_omega, double eta,
                          double* chi, double* eps_inv, double* loss) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    if (n_omega < 0 || (n_omega > 0 && !omega)) fail(LZ_ERR_ARG, "bad frequency grid");
    if (!(eta > 0)) fail(LZ_ERR_ARG, "eta must be > 0");
    if (extrapolation != LZ_EXTRAP_NONE && extrapolation != LZ_EXTRAP_CONSTANT &&
        extrapolation != LZ_EXTRAP_OSC)
      fail(LZ_ERR_ARG, "unknown extrapolation scheme");
    if (extrapolation == LZ_EXTRAP_NONE) m = m0;
    if (m < m0) fail(LZ_ERR_ARG, "m must be >= m0");
    if (m > m0 && m0 < 4) fail(LZ_ERR_ARG, "extrapolation needs at least 4 computed coefficients");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    if (m0 < 0 || m0 > I.steps_host) fail(LZ_ERR_STATE, "m0 exceeds the completed steps");
    if (I.nh && m > m0) fail(LZ_ERR_ARG, "extrapolation is defined for the pseudo-Hermitian recursion only");
    if (n_omega == 0) return;
    // tail of the extended matrix: means over the last half of beta_2..beta_m0
    double tail[2] = {0.0, 0.0};
    if (m > m0) {
      std::vector<double> b(m0);
      HIPC(hipMemcpy(b.data(), I.beta.p, m0 * sizeof(double), hipMemcpyDeviceToHost));
      const int lo = std::max(2, m0 / 2 + 1);
      double sum[2] = {0.0, 0.0}, all = 0.0;
      int cnt[2] = {0, 0};
      for (int k = lo; k <= m0; ++k) {
        sum[k & 1] += b[k - 1];
        cnt[k & 1] += 1;
        all += b[k - 1];
      }
      if (extrapolation == LZ_EXTRAP_OSC) {
        tail[0] = sum[0] / cnt[0];
        tail[1] = sum[1] / cnt[1];
      } else {
        tail[0] = tail[1] = all / (cnt[0] + cnt[1]);
      }
    }
    DBuf dw, dchi, dei, dl;
    dw.alloc(n_omega * sizeof(double));
    dchi.alloc(2 * n_omega * sizeof(double));
    dei.alloc(2 * n_omega * sizeof(double));
    dl.alloc(n_omega * sizeof(double));
    HIPC(hipMemcpyAsync(dw.p, omega, n_omega * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_spectrum(I.beta.as<double>(), I.nh ? I.gam.as<double>() : nullptr, I.z.as<double>(),
                    m0, m, tail[0], tail[1],
                    dw.as<double>(), n_omega, eta, I.pref, I.fq, dchi.as<double>(),
                    dei.as<double>(), dl.as<double>(), c->stream);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(c->stream));
    if (chi) HIPC(hipMemcpy(chi, dchi.p, 2 * n_omega * sizeof(double), hipMemcpyDeviceToHost));
    if (eps_inv) HIPC(hipMemcpy(eps_inv, dei.p, 2 * n_omega * sizeof(double), hipMemcpyDeviceToHost));
    if (loss) HIPC(hipMemcpy(loss, dl.p, n_omega * sizeof(double), hipMemcpyDeviceToHost));
  });
}

lz_status lz_spectrum(lz_ctx* c, int32_t inst, int32_t m, const double* omega, int32_t n_omega,
                      double eta, double* chi, double* eps_inv, double* loss) {
  return lz_spectrum_ext(c, inst, m, m, LZ_EXTRAP_NONE, omega, n_omega, eta, chi, eps_inv, loss);
}

lz_status lz_spectrum_ext_noalloc(lz_ctx* c, int32_t inst, int32_t m0, int32_t m,
                                  int32_t extrapolation, const double* omega, int32_t n_omega,
                                  double eta, double* chi, double* eps_inv, double* loss) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    if (n_omega < 0 || (n_omega > 0 && !omega)) fail(LZ_ERR_ARG, "bad frequency grid");
    if (n_omega > kNoallocMaxOmega) fail(LZ_ERR_ARG, "n_omega exceeds 65536 (the staging area)");
    if (!(eta > 0)) fail(LZ_ERR_ARG, "eta must be > 0");
    if (extrapolation != LZ_EXTRAP_NONE && extrapolation != LZ_EXTRAP_CONSTANT &&
        extrapolation != LZ_EXTRAP_OSC)
      fail(LZ_ERR_ARG, "unknown extrapolation scheme");
    if (extrapolation == LZ_EXTRAP_NONE) m = m0;
    if (m < m0) fail(LZ_ERR_ARG, "m must be >= m0");
    if (m > m0 && m0 < 4) fail(LZ_ERR_ARG, "extrapolation needs at least 4 computed coefficients");
    HIPC(hipSetDevice(c->device));
    Instance& I = *c->inst[inst];
    // the completed steps, read without the stage-timer bookkeeping
    HIPC(hipStreamSynchronize(c->stream));
    LzDevState h;
    HIPC(hipMemcpy(&h, I.st.p, sizeof(h), hipMemcpyDeviceToHost));
    if (m0 < 0 || m0 > h.step) fail(LZ_ERR_STATE, "m0 exceeds the completed steps");
    if (I.nh && m > m0) fail(LZ_ERR_ARG, "extrapolation is defined for the pseudo-Hermitian recursion only");
    if (n_omega == 0) return;
    double* dw = c->scratch;
    double* dchi = dw + n_omega;
    double* dei = dchi + 2 * (size_t)n_omega;
    double* dl = dei + 2 * (size_t)n_omega;
    double* dtail = c->scratch + 6 * (size_t)kNoallocMaxOmega;
    HIPC(hipMemcpyAsync(dw, omega, n_omega * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_spectrum_dev_tail(I.beta.as<double>(), I.nh ? I.gam.as<double>() : nullptr,
                             I.z.as<double>(), m0, m, extrapolation == LZ_EXTRAP_OSC, dtail, dw,
                             n_omega, eta, I.pref, I.fq, dchi, dei, dl, c->stream);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(c->stream));
    if (chi) HIPC(hipMemcpy(chi, dchi, 2 * n_omega * sizeof(double), hipMemcpyDeviceToHost));
    if (eps_inv) HIPC(hipMemcpy(eps_inv, dei, 2 * n_omega * sizeof(double), hipMemcpyDeviceToHost));
    if (loss) HIPC(hipMemcpy(loss, dl, n_omega * sizeof(double), hipMemcpyDeviceToHost));
  });
}

lz_status lz_get_rhs(lz_ctx* c, int32_t inst, void* y_out) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size() || !y_out) fail(LZ_ERR_ARG, "bad argument");
    HIPC(hipSetDevice(c->device));
    c->enter();
    Instance& I = *c->inst[inst];
    if (I.fp64) LaunchLin<double>::perm_out(I.y.p, y_out, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, c->stream);
    else LaunchLin<float>::perm_out(I.y.p, y_out, I.perm.as<int>(), I.npw_kq.as<int>(), I.nks, I.nbnd, I.npwx, c->stream);
    HIPC(hipGetLastError());
    c->leave();
  });
}

lz_status lz_stage_timer(lz_ctx* c, int32_t mask) {
  return guarded([&] {
    if (!c) fail(LZ_ERR_ARG, "null context");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    for (auto& ip : c->inst) {
      ip->timer.mask = (uint32_t)mask & ((1u << ST_COUNT) - 1u);
      ip->timer.on = ip->timer.mask != 0;
      ip->timer.reset();
    }
  });
}

lz_status lz_stage_times(lz_ctx* c, int32_t inst, double* total_ms, int32_t* count) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) fail(LZ_ERR_ARG, "bad context or instance");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    for (int s = 0; s < ST_COUNT; ++s) {
      if (total_ms) total_ms[s] = I.timer.total_ms[s];
      if (count) count[s] = I.timer.count[s];
    }
  });
}

// ---- checkpoint / restart of the recursion state of one instance ----------
namespace {
constexpr uint64_t kCkptMagic = 0x4C5A434B50543033ull;  // "LZCKPT03"
struct CkptHeader {
  uint64_t magic;
  int32_t prec, nks, nbnd, nproj, npwx, n1, n2, n3;
  int32_t step, alg;
  int64_t nvec;
  int32_t approx, pad;
  uint64_t fingerprint;  // of the operator's inputs (Instance::fingerprint)
  LzDevState st;
};
// pseudo-Hermitian: beta, z and the vectors X0, X1, LW; non-Hermitian: beta,
// gamma, z and the two chains X0, X1, Y0, Y1
uint64_t ckpt_bytes(const Instance& I, int step) {
  const uint64_t coef = I.nh ? 5 : 3, vecs = I.nh ? 4 : 3;
  return sizeof(CkptHeader) + (uint64_t)step * coef * sizeof(double) + vecs * I.nvec * I.csz;
}
struct CkptVectors {
  DBuf* v[4];
  int n;
  DBuf** begin() { return v; }
  DBuf** end() { return v + n; }
};
CkptVectors ckpt_vectors(Instance& I) {
  if (I.nh) return {{&I.X0, &I.X1, &I.Y0, &I.Y1}, 4};
  return {{&I.X0, &I.X1, &I.LW, nullptr}, 3};
}
}  // namespace

lz_status lz_checkpoint_size(lz_ctx* c, int32_t inst, uint64_t* bytes) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size() || !bytes) fail(LZ_ERR_ARG, "bad argument");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    const Instance& I = *c->inst[inst];
    *bytes = ckpt_bytes(I, I.steps_host);
  });
}

lz_status lz_checkpoint_save(lz_ctx* c, int32_t inst, void* buf, uint64_t bytes) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size() || !buf) fail(LZ_ERR_ARG, "bad argument");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    const int step = I.steps_host;
    if (bytes < ckpt_bytes(I, step)) fail(LZ_ERR_ARG, "checkpoint buffer too small");
    CkptHeader h{};
    h.magic = kCkptMagic;
    h.prec = I.prec; h.nks = I.nks; h.nbnd = I.nbnd; h.nproj = I.nproj; h.npwx = I.npwx;
    h.n1 = I.n1; h.n2 = I.n2; h.n3 = I.n3; h.step = step; h.nvec = I.nvec;
    h.alg = I.nh ? LZ_NON_HERMITIAN : LZ_PSEUDO_HERMITIAN;
    h.approx = I.approx;
    h.fingerprint = I.fingerprint;
    HIPC(hipMemcpy(&h.st, I.st.p, sizeof(LzDevState), hipMemcpyDeviceToHost));
    char* o = static_cast<char*>(buf);
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    if (step > 0) {
      HIPC(hipMemcpy(o, I.beta.p, step * sizeof(double), hipMemcpyDeviceToHost));
      o += step * sizeof(double);
      if (I.nh) {
        HIPC(hipMemcpy(o, I.gam.p, 2 * step * sizeof(double), hipMemcpyDeviceToHost));
        o += 2 * step * sizeof(double);
      }
      HIPC(hipMemcpy(o, I.z.p, 2 * step * sizeof(double), hipMemcpyDeviceToHost));
      o += 2 * step * sizeof(double);
    }
    const size_t vb = (size_t)I.nvec * I.csz;
    for (DBuf* d : ckpt_vectors(I)) {
      HIPC(hipMemcpy(o, d->p, vb, hipMemcpyDeviceToHost));
      o += vb;
    }
  });
}

lz_status lz_checkpoint_load(lz_ctx* c, int32_t inst, const void* buf, uint64_t bytes) {
  return guarded([&] {
    if (!c || inst < 0 || inst >= (int)c->inst.size() || !buf) fail(LZ_ERR_ARG, "bad argument");
    if (bytes < sizeof(CkptHeader)) fail(LZ_ERR_ARG, "checkpoint truncated");
    HIPC(hipSetDevice(c->device));
    read_state(c);
    Instance& I = *c->inst[inst];
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (h.magic != kCkptMagic) fail(LZ_ERR_ARG, "not a checkpoint of this library");
    if (h.prec != I.prec || h.nks != I.nks || h.nbnd != I.nbnd || h.nproj != I.nproj ||
        h.npwx != I.npwx || h.n1 != I.n1 || h.n2 != I.n2 || h.n3 != I.n3 || h.nvec != I.nvec)
      fail(LZ_ERR_ARG, "checkpoint of a different system or precision");
    if (h.alg != (I.nh ? LZ_NON_HERMITIAN : LZ_PSEUDO_HERMITIAN))
      fail(LZ_ERR_ARG, "checkpoint of the other Lanczos algorithm");
    if (h.approx != I.approx) fail(LZ_ERR_ARG, "checkpoint of another level of theory");
    if (h.fingerprint != I.fingerprint)
      fail(LZ_ERR_ARG, "checkpoint of another system (the operator's inputs differ)");
    if (h.step < 0 || h.step > I.max_steps) fail(LZ_ERR_ARG, "checkpoint exceeds max_steps");
    if (bytes < ckpt_bytes(I, h.step)) fail(LZ_ERR_ARG, "checkpoint truncated");
    const char* o = static_cast<const char*>(buf) + sizeof(h);
    HIPC(hipMemcpy(I.st.p, &h.st, sizeof(LzDevState), hipMemcpyHostToDevice));
    if (h.step > 0) {
      HIPC(hipMemcpy(I.beta.p, o, h.step * sizeof(double), hipMemcpyHostToDevice));
      o += h.step * sizeof(double);
      if (I.nh) {
        HIPC(hipMemcpy(I.gam.p, o, 2 * h.step * sizeof(double), hipMemcpyHostToDevice));
        o += 2 * h.step * sizeof(double);
      }
      HIPC(hipMemcpy(I.z.p, o, 2 * h.step * sizeof(double), hipMemcpyHostToDevice));
      o += 2 * h.step * sizeof(double);
    }
    const size_t vb = (size_t)I.nvec * I.csz;
    for (DBuf* d : ckpt_vectors(I)) {
      HIPC(hipMemcpy(d->p, o, vb, hipMemcpyHostToDevice));
      o += vb;
    }
    HIPC(hipDeviceSynchronize());
    I.steps_host = h.step;
    I.status_host = h.st.status;
    c->started = true;
  });
}

}  // extern "C"

namespace {

// LOBPCG (Knyazev 2001) for the lowest m eigenpairs of H on the k+q spheres
// of an internal instance with no valence manifold (P_c = 1) and zero band
// energies, whose D applications are then H x.  Per iteration, with X the
// Ritz block, P the previous search direction and theta the Ritz values:
//   R = H X - X theta, W = precond(R)             (k_gs_residual)
//   Z = [W, P], Z <- Z - X (X^H Z) twice
//   Z' = Z Q lam^{-1/2} over the directions Z spans (Jacobi on Z^H Z), twice
//   H Z' applied explicitly (products of H by combinations of earlier
//   blocks drift once the Gram matrices are ill-conditioned)
//   V = [X, Z'], T = V^H H V, T Y = Y theta       (Jacobi)
//   X = V Y[:, :m], H X = H V Y[:, :m], P = Z' Y[m:, :m]
// All in double precision on the device; the host reads only the residual
// norms to stop.
struct GsBuffers {
  DBuf X, HX, R, W, HW, P, HP, Z, HZ, Zc, HZc, V, HV, part, G, Tm, Ym, Cm, wv, keep, theta;
};

// Block products of the eigensolver run on the matrix cores once both sides
// hold many vectors (the 128-band large cell: Gram matrices of order 396 over
// 51k plane waves), on the vector ALU for the small blocks.
int gs_gemm(int P, int nb) { return P >= 64 && nb >= 32 ? kGemmMfma : kGemmValu; }
int gs_chunk(const Instance& I, int P, int nb) {
  return gs_gemm(P, nb) == kGemmMfma ? LaunchLin<double>::mfma_chunk(P, nb, I.npwx, I.nks)
                                     : kProjChunk;
}
// partials of a Gram product of P x nb (complex elements)
size_t gs_part_elems(const Instance& I, int P, int nb) {
  const int ch = gs_chunk(I, P, nb);
  return (size_t)I.nks * ((I.npwx + ch - 1) / ch) * P * nb;
}

void gs_gram(Instance& I, GsBuffers& b, const void* A, int P, const void* B, int nb, void* out,
             hipStream_t s) {
  const int gm = gs_gemm(P, nb), ch = gs_chunk(I, P, nb), nch = (I.npwx + ch - 1) / ch;
  LaunchLin<double>::proj_dot(A, P, P, const_cast<void*>(B), nullptr, nb, I.npwx, I.nks, ch, nch,
                              b.part.p, nullptr, s, gm);
  LaunchLin<double>::reduce(b.part.p, nch, P, nb, I.nks, out, s);
}

// Y[k][nb] (+)= A[k][P]^T C[k][P][nb]
void gs_comb(Instance& I, void* Y, const void* A, int P, const void* C, int nb, bool accumulate,
             hipStream_t s) {
  if (!accumulate)
    HIPC(hipMemsetAsync(Y, 0, (size_t)I.nks * nb * I.npwx * sizeof(double2), s));
  LaunchLin<double>::proj_update(Y, A, P, P, C, P, nb, I.npwx, I.nks, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, s, gs_gemm(P, nb));
}

// rows [0, ra) of V[k] = A[k], rows [ra, ra + rb) = B[k]
void gs_stack(Instance& I, void* V, const void* A, int ra, const void* B, int rb, hipStream_t s) {
  const size_t row = (size_t)I.npwx * sizeof(double2);
  const size_t pitch = (size_t)(ra + rb) * row;
  HIPC(hipMemcpy2DAsync(V, pitch, A, ra * row, ra * row, I.nks, hipMemcpyDeviceToDevice, s));
  HIPC(hipMemcpy2DAsync((char*)V + ra * row, pitch, B, rb * row, rb * row, I.nks,
                        hipMemcpyDeviceToDevice, s));
}

// Rayleigh-Ritz of LOBPCG up to this order (3 (nbnd + n_extra)); larger
// blocks take the Chebyshev-filtered subspace iteration, whose dense problems
// are of the block's own order
constexpr int kLobpcgOrderMax = 256;
constexpr int kChebDegree = 40;
constexpr int kChebMinDegree = 4;

// Chebyshev-filtered subspace iteration (Zhou and Saad, 2007) for the lowest
// m eigenpairs, from the Ritz block (X, HX, theta) left by the start: each
// iteration applies a Chebyshev polynomial of H (degree up to kChebDegree) that is
// small on [a, ub] (a the largest Ritz value of the block, ub an upper bound
// of the spectrum) and normalised at the lowest Ritz value, then
// orthonormalises the block (Jacobi on its Gram matrix) and does
// Rayleigh-Ritz in its span.  Only products by H and dense problems of order
// m.  ub = max kinetic energy of the sphere + max V_loc + a Gershgorin bound
// of sum_p max(D_p, 0) |beta_p><beta_p| (Weyl: the three are Hermitian).
void chebyshev_ground_state(const lz_system& sys, Instance& I, GsBuffers& b, int m, int nb_out,
                            const std::vector<double>& kin, double tol, int max_iter, int& it,
                            double& worst, hipStream_t s) {
  const int nks = I.nks, npwx = I.npwx;
  // the upper bound per sphere
  std::vector<double> ub(nks, 0.0);
  double vmax = -1e300;
  for (int i = 0; i < I.N; ++i) vmax = std::max(vmax, sys.vloc_r[i]);
  std::vector<double> gersh(nks, 0.0);
  if (I.nproj > 0) {
    const int np = I.nproj;
    DBuf bc, gram;
    bc.alloc((size_t)nks * np * npwx * sizeof(double2));
    gram.alloc((size_t)nks * np * np * sizeof(double2));
    const size_t row = (size_t)npwx * sizeof(double2);
    HIPC(hipMemcpy2DAsync(bc.p, np * row, (const char*)I.Aio.p + (size_t)m * row, I.ptot * row,
                          np * row, nks, hipMemcpyDeviceToDevice, s));
    DBuf part;
    part.alloc(gs_part_elems(I, np, np) * sizeof(double2));
    std::swap(part.p, b.part.p);
    gs_gram(I, b, bc.p, np, bc.p, np, gram.p, s);
    std::swap(part.p, b.part.p);
    std::vector<double2> g((size_t)nks * np * np);
    std::vector<double> dkb(np);
    HIPC(hipMemcpyAsync(g.data(), gram.p, g.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(dkb.data(), I.dkb.p, np * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int k = 0; k < nks; ++k)
      for (int p = 0; p < np; ++p) {
        double r = 0.0;
        for (int q = 0; q < np; ++q) {
          const double2 x = g[((size_t)k * np + p) * np + q];
          r += std::sqrt(std::max(dkb[p], 0.0) * std::max(dkb[q], 0.0)) * std::hypot(x.x, x.y);
        }
        gersh[k] = std::max(gersh[k], r);
      }
  }
  for (int k = 0; k < nks; ++k) {
    double kmax = 0.0;
    for (int i = 0; i < sys.npw_kq[k]; ++i) kmax = std::max(kmax, kin[(size_t)k * npwx + i]);
    ub[k] = 1.01 * (kmax + std::max(vmax, 0.0) + gersh[k]) + 0.01;
  }
  std::vector<double> theta((size_t)nks * m), coef((size_t)kChebDegree * nks * 3);
  std::vector<double2> rr((size_t)nks * m * m);
  DBuf dcoef, dscale;
  dcoef.alloc(coef.size() * sizeof(double));
  dscale.alloc((size_t)nks * m * sizeof(double));
  for (it = 0;; ++it) {
    // residual norms of the wanted pairs
    launch_gs_residual(b.X.p, b.HX.p, b.theta.as<double>(), I.kin.p, m, npwx, nks, 1.0, b.R.p,
                       b.W.p, s);
    gs_gram(I, b, b.R.p, m, b.R.p, m, b.G.p, s);
    HIPC(hipMemcpyAsync(rr.data(), b.G.p, rr.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(theta.data(), b.theta.p, theta.size() * sizeof(double),
                        hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    worst = 0.0;
    for (int k = 0; k < nks; ++k)
      for (int n = 0; n < nb_out; ++n)
        worst = std::max(worst, std::sqrt(std::max(0.0, rr[((size_t)k * m + n) * m + n].x)));
    if (worst < tol || it >= max_iter) break;
    // Degree of this iteration's filter.  Normalised at the lowest Ritz value
    // a0, the filter scales the component along the highest wanted one (at
    // theta_t) down by T_d(x(a0)) / T_d(x(theta_t)), x mapping [a, ub] to
    // [-1, 1]; a column then keeps its own direction only against the
    // admixture of lower ones that it carries, and beyond about 1e8 that is
    // lost to rounding in the orthonormalisation (89 free-electron bands:
    // degree 40 would scale by 1e-15 and the upper eight directions were
    // dropped).  So d stays below ln(1e8) / (acosh|x(a0)| - acosh|x(theta_t)|).
    int deg = kChebDegree;
    for (int k = 0; k < nks; ++k) {
      const double a = theta[(size_t)k * m + m - 1], a0 = theta[(size_t)k * m];
      const double at = theta[(size_t)k * m + nb_out - 1];
      const double e = 0.5 * (ub[k] - a), c = 0.5 * (ub[k] + a);
      const double x0 = std::max(1.0, std::fabs((a0 - c) / e));
      const double xt = std::max(1.0, std::fabs((at - c) / e));
      const double gap = std::acosh(x0) - std::acosh(xt);
      if (gap > 0.0) deg = std::min(deg, std::max(kChebMinDegree, (int)(std::log(1e8) / gap)));
    }
    // coefficients of the filter steps per sphere
    for (int k = 0; k < nks; ++k) {
      const double a = theta[(size_t)k * m + m - 1], a0 = theta[(size_t)k * m];
      const double e = 0.5 * (ub[k] - a), c = 0.5 * (ub[k] + a);
      double sig = e / (a0 - c);
      const double sig1 = sig;
      for (int d = 0; d < deg; ++d) {
        double* cf = &coef[((size_t)d * nks + k) * 3];
        if (d == 0) {
          cf[0] = sig1 / e;
          cf[1] = -c * sig1 / e;
          cf[2] = 0.0;
        } else {
          const double sn = 1.0 / (2.0 / sig1 - sig);
          cf[0] = 2.0 * sn / e;
          cf[1] = -2.0 * sn * c / e;
          cf[2] = -sig * sn;
          sig = sn;
        }
      }
    }
    HIPC(hipMemcpyAsync(dcoef.p, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice,
                        s));
    // filter: Y_0 = X, Y_1 = c0 H X + c1 X, Y_d = c0 H Y_{d-1} + c1 Y_{d-1} + c2 Y_{d-2}
    void* prev = b.X.p;  // Y_{d-2}
    void* cur = b.W.p;   // Y_{d-1}
    launch_cheb_step(cur, b.HX.p, b.X.p, nullptr, dcoef.as<double>(), m, npwx, nks, s);
    for (int d = 1; d < deg; ++d) {
      apply_half<double>(I, cur, b.HW.p, false, s);
      launch_cheb_step(prev, b.HW.p, cur, prev, dcoef.as<double>() + (size_t)d * nks * 3, m, npwx,
                       nks, s);
      std::swap(prev, cur);
    }
    // cur = filtered block: orthonormalise it (columns scaled to unit norm
    // first; twice, the second pass removing what rounding leaves of the
    // first), through prev
    for (int pass = 0; pass < 2; ++pass) {
      gs_gram(I, b, cur, m, cur, m, b.G.p, s);
      launch_gram_unit(b.G.p, m, dscale.as<double>(), nks, s);
      launch_heev(b.G.p, m, m, b.wv.as<double>(), b.Ym.p, nks, s);
      launch_orth_coef(b.Ym.p, b.wv.as<double>(), m, 1e-13, b.Cm.p, b.keep.as<int>(), nks, s);
      launch_row_scale(b.Cm.p, m, dscale.as<double>(), nks, s);
      gs_comb(I, prev, cur, m, b.Cm.p, m, false, s);
      std::swap(prev, cur);
    }
    std::swap(prev, cur);  // the orthonormal block in prev, cur free
    // Rayleigh-Ritz in its span: X = V Y, HX = HV Y
    apply_half<double>(I, prev, b.HW.p, false, s);
    gs_gram(I, b, prev, m, b.HW.p, m, b.Tm.p, s);
    launch_mask_dropped(b.Tm.p, m, 0, m, b.keep.as<int>(), nks, s);
    launch_heev(b.Tm.p, m, m, b.theta.as<double>(), b.Ym.p, nks, s);
    gs_comb(I, cur, prev, m, b.Ym.p, m, false, s);
    gs_comb(I, b.HX.p, b.HW.p, m, b.Ym.p, m, false, s);
    // the new block is in cur: make it b.X (the buffers of b.X and b.W hold
    // prev and cur in some order)
    if (cur != b.X.p) std::swap(b.X.p, b.W.p);
  }
}

}  // namespace

extern "C" {

lz_status lz_ground_state(const lz_system* sys, int32_t n_extra, double tol, int32_t max_iter,
                          int32_t device, void* hip_stream, double* evc_out, double* et_out,
                          int32_t* iterations, double* max_residual) {
  return guarded([&] {
    if (!sys || !evc_out || !et_out) fail(LZ_ERR_ARG, "null argument");
    if (n_extra < 0 || !(tol > 0) || max_iter < 1) fail(LZ_ERR_ARG, "bad solver parameters");
    const int nb_out = sys->nbnd;
    const int m = nb_out + n_extra;
    if (nb_out < 1 || 3 * m > kSmallOrderMax) fail(LZ_ERR_ARG, "3 (nbnd + n_extra) must lie in [3, 512]");
    if (!sys->vloc_r || !sys->wk || !sys->xk || !sys->npw_kq || !sys->nl_kq || !sys->npw_k ||
        !sys->nl_k)
      fail(LZ_ERR_ARG, "null array in the system");
    int ndev = 0;
    HIPC(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(LZ_ERR_ARG, "no such device");
    HIPC(hipSetDevice(device));
    HIPC(enable_large_lds_fft<double>());
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    HIPC(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct Guard {
      hipStream_t& s;
      hipEvent_t& e;
      ~Guard() {
        if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
        if (e) (void)hipEventDestroy(e);
      }
    } guard{s, ev};
    HIPC(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPC(hipEventRecord(ev, (hipStream_t)hip_stream));
    HIPC(hipStreamWaitEvent(s, ev, 0));
    // the internal instance: m bands, no valence manifold, zero energies
    const int nks = sys->nks, npwx = sys->npwx;
    const int N = sys->nr[0] * sys->nr[1] * sys->nr[2];
    std::vector<double> zevc((size_t)nks * m * npwx * 2, 0.0), zet((size_t)nks * m, 0.0),
        zf((size_t)N, 0.0);
    lz_system g = *sys;
    g.nbnd = m;
    // no right-hand side is formed here: any nonzero Q passes the checks
    g.g0[0] = 1;
    g.g0[1] = 0;
    g.g0[2] = 0;
    g.evc_k = zevc.data();
    g.evc_kq = zevc.data();
    g.et_k = zet.data();
    g.fxc_r = zf.data();
    lz_options o{};
    o.prec = LZ_FP64;
    o.approx = LZ_IPA;
    o.max_steps = 1;
    o.projector_gemm = LZ_GEMM_VALU;
    std::unique_ptr<Instance> Ip = build_instance(g, o, s);
    Instance& I = *Ip;
    const size_t vb = (size_t)nks * m * npwx * sizeof(double2);
    const int n2 = 2 * m, n3 = 3 * m;
    GsBuffers b;
    for (DBuf* d : {&b.X, &b.HX, &b.R, &b.W, &b.HW, &b.P, &b.HP}) d->alloc(vb);
    for (DBuf* d : {&b.Z, &b.HZ, &b.Zc, &b.HZc}) d->alloc(2 * vb);
    b.V.alloc(3 * vb);
    b.HV.alloc(3 * vb);
    {
      size_t pe = 0;  // the largest partials of the Gram products below
      const int dims[4][2] = {{m, m}, {m, n2}, {n2, n2}, {n3, n3}};
      for (const auto& d : dims) pe = std::max(pe, gs_part_elems(I, d[0], d[1]));
      b.part.alloc(pe * sizeof(double2));
    }
    for (DBuf* d : {&b.G, &b.Tm, &b.Ym, &b.Cm}) d->alloc((size_t)nks * n3 * n3 * sizeof(double2));
    b.wv.alloc((size_t)nks * n3 * sizeof(double));
    b.keep.alloc((size_t)nks * n2 * sizeof(int));
    b.theta.alloc((size_t)nks * m * sizeof(double));
    // start: the m plane waves of lowest kinetic energy on each sphere, with a
    // small deterministic admixture of the others, orthonormalised
    std::vector<double> kin((size_t)nks * npwx);
    HIPC(hipMemcpyAsync(kin.data(), I.kin.p, kin.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::vector<double> x0((size_t)nks * m * npwx * 2, 0.0);
    uint64_t lcg = 0x9E3779B97F4A7C15ull;
    auto urand = [&] {
      lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
      return (double)(lcg >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    };
    for (int k = 0; k < nks; ++k) {
      const int np = sys->npw_kq[k];
      if (np < n3) fail(LZ_ERR_ARG, "a sphere holds fewer plane waves than 3 (nbnd + n_extra)");
      std::vector<int> ord(np);
      for (int i = 0; i < np; ++i) ord[i] = i;
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) {
        return kin[(size_t)k * npwx + a] < kin[(size_t)k * npwx + c];
      });
      for (int bnd = 0; bnd < m; ++bnd) {
        double* row = x0.data() + ((size_t)k * m + bnd) * npwx * 2;
        for (int i = 0; i < np; ++i) {
          row[2 * i] = 1e-3 * urand() / (1.0 + kin[(size_t)k * npwx + i]);
          row[2 * i + 1] = 1e-3 * urand() / (1.0 + kin[(size_t)k * npwx + i]);
        }
        row[2 * ord[bnd]] += 1.0;
      }
    }
    HIPC(hipMemcpyAsync(b.W.p, x0.data(), vb, hipMemcpyHostToDevice, s));
    // orthonormalise the start block: X = W Q lam^{-1/2}
    gs_gram(I, b, b.W.p, m, b.W.p, m, b.G.p, s);
    launch_heev(b.G.p, m, m, b.wv.as<double>(), b.Ym.p, nks, s);
    launch_orth_coef(b.Ym.p, b.wv.as<double>(), m, 1e-12, b.Cm.p, b.keep.as<int>(), nks, s);
    gs_comb(I, b.X.p, b.W.p, m, b.Cm.p, m, false, s);
    // Rayleigh-Ritz in span(X)
    apply_half<double>(I, b.X.p, b.HX.p, false, s);
    gs_gram(I, b, b.X.p, m, b.HX.p, m, b.G.p, s);
    launch_heev(b.G.p, m, m, b.theta.as<double>(), b.Ym.p, nks, s);
    gs_comb(I, b.W.p, b.X.p, m, b.Ym.p, m, false, s);
    gs_comb(I, b.HW.p, b.HX.p, m, b.Ym.p, m, false, s);
    std::swap(b.X.p, b.W.p);
    std::swap(b.HX.p, b.HW.p);
    std::vector<double2> rr((size_t)nks * m * m);
    int it = 0;
    double worst = 0.0;
    if (3 * m > kLobpcgOrderMax) {
      chebyshev_ground_state(*sys, I, b, m, nb_out, kin, tol, max_iter, it, worst, s);
    } else for (;; ++it) {
      // residuals, their norms, the preconditioned corrections and H W
      launch_gs_residual(b.X.p, b.HX.p, b.theta.as<double>(), I.kin.p, m, npwx, nks, 1.0, b.R.p,
                         b.W.p, s);
      gs_gram(I, b, b.R.p, m, b.R.p, m, b.G.p, s);
      HIPC(hipMemcpyAsync(rr.data(), b.G.p, rr.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      worst = 0.0;
      for (int k = 0; k < nks; ++k)
        for (int n = 0; n < nb_out; ++n)
          worst = std::max(worst, std::sqrt(std::max(0.0, rr[((size_t)k * m + n) * m + n].x)));
      if (worst < tol || it >= max_iter) break;
      // Z = [W, P] (P = 0 on the first iteration: its directions are dropped)
      gs_stack(I, b.Z.p, b.W.p, m, b.P.p, m, s);
      for (int pass = 0; pass < 2; ++pass) {
        gs_gram(I, b, b.X.p, m, b.Z.p, n2, b.G.p, s);
        launch_small_take(b.Cm.p, b.G.p, m, n2, n2, 0, m * n2, -1.0, nks, s);
        gs_comb(I, b.Z.p, b.X.p, m, b.Cm.p, n2, true, s);
      }
      // orthonormal directions of Z (the second pass removes what the first
      // leaves of non-orthogonality; its directions all survive)
      gs_gram(I, b, b.Z.p, n2, b.Z.p, n2, b.G.p, s);
      launch_heev(b.G.p, n2, n2, b.wv.as<double>(), b.Ym.p, nks, s);
      launch_orth_coef(b.Ym.p, b.wv.as<double>(), n2, 1e-10, b.Cm.p, b.HW.as<int>(), nks, s);
      gs_comb(I, b.Zc.p, b.Z.p, n2, b.Cm.p, n2, false, s);
      // (the kept columns of the second pass, in its own order, mark T)
      gs_gram(I, b, b.Zc.p, n2, b.Zc.p, n2, b.G.p, s);
      launch_heev(b.G.p, n2, n2, b.wv.as<double>(), b.Ym.p, nks, s);
      launch_orth_coef(b.Ym.p, b.wv.as<double>(), n2, 1e-3, b.Cm.p, b.keep.as<int>(), nks, s);
      gs_comb(I, b.Z.p, b.Zc.p, n2, b.Cm.p, n2, false, s);
      // H on the two halves of the orthonormal block
      {
        const size_t row = (size_t)npwx * sizeof(double2);
        HIPC(hipMemcpy2DAsync(b.W.p, m * row, b.Z.p, n2 * row, m * row, nks,
                              hipMemcpyDeviceToDevice, s));
        HIPC(hipMemcpy2DAsync(b.R.p, m * row, (const char*)b.Z.p + m * row, n2 * row, m * row,
                              nks, hipMemcpyDeviceToDevice, s));
      }
      apply_half<double>(I, b.W.p, b.HW.p, false, s);
      apply_half<double>(I, b.R.p, b.HP.p, false, s);
      std::swap(b.Zc.p, b.Z.p);
      gs_stack(I, b.HZc.p, b.HW.p, m, b.HP.p, m, s);
      // Rayleigh-Ritz in span(X, Z')
      gs_stack(I, b.V.p, b.X.p, m, b.Zc.p, n2, s);
      gs_stack(I, b.HV.p, b.HX.p, m, b.HZc.p, n2, s);
      gs_gram(I, b, b.V.p, n3, b.HV.p, n3, b.Tm.p, s);
      launch_mask_dropped(b.Tm.p, n3, m, n2, b.keep.as<int>(), nks, s);
      launch_heev(b.Tm.p, n3, n3, b.wv.as<double>(), b.Ym.p, nks, s);
      launch_small_take(b.Cm.p, b.Ym.p, n3, m, n3, 0, n3 * n3, 1.0, nks, s);
      gs_comb(I, b.X.p, b.V.p, n3, b.Cm.p, m, false, s);
      gs_comb(I, b.HX.p, b.HV.p, n3, b.Cm.p, m, false, s);
      // P = Z' Y[m:, :m]
      launch_small_take(b.Cm.p, (const double2*)b.Ym.p + (size_t)m * n3, n2, m, n3, 0, n3 * n3,
                        1.0, nks, s);
      gs_comb(I, b.P.p, b.Zc.p, n2, b.Cm.p, m, false, s);
      HIPC(hipMemcpy2DAsync(b.theta.p, m * sizeof(double), b.wv.p, n3 * sizeof(double),
                            m * sizeof(double), nks, hipMemcpyDeviceToDevice, s));
    }
    // eigenpairs 0..nbnd-1 in the caller's plane-wave order
    LaunchLin<double>::perm_out(b.X.p, b.W.p, I.perm.as<int>(), I.npw_kq.as<int>(), nks, m, npwx,
                                s);
    std::vector<double> xo((size_t)nks * m * npwx * 2), th((size_t)nks * m);
    HIPC(hipMemcpyAsync(xo.data(), b.W.p, vb, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(th.data(), b.theta.p, th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int k = 0; k < nks; ++k) {
      std::memcpy(evc_out + (size_t)k * nb_out * npwx * 2, xo.data() + (size_t)k * m * npwx * 2,
                  (size_t)nb_out * npwx * 2 * sizeof(double));
      std::memcpy(et_out + (size_t)k * nb_out, th.data() + (size_t)k * m, nb_out * sizeof(double));
    }
    if (iterations) *iterations = it;
    if (max_residual) *max_residual = worst;
  });
}

lz_status lz_ground_density(const lz_system* sys, int32_t xc, int32_t device, void* hip_stream,
                            double* n0_out, double* fxc_out) {
  return guarded([&] {
    if (!sys || (!n0_out && !fxc_out)) fail(LZ_ERR_ARG, "null argument");
    if (xc != LZ_XC_X && xc != LZ_XC_PZ) fail(LZ_ERR_ARG, "unknown xc kernel");
    if (!sys->evc_k || !sys->wk || !sys->xk || !sys->npw_k || !sys->nl_k || !sys->vloc_r)
      fail(LZ_ERR_ARG, "null array in the system");
    int ndev = 0;
    HIPC(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(LZ_ERR_ARG, "no such device");
    HIPC(hipSetDevice(device));
    HIPC(enable_large_lds_fft<double>());
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    HIPC(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct Guard {
      hipStream_t& s;
      hipEvent_t& e;
      ~Guard() {
        if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
        if (e) (void)hipEventDestroy(e);
      }
    } guard{s, ev};
    HIPC(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPC(hipEventRecord(ev, (hipStream_t)hip_stream));
    HIPC(hipStreamWaitEvent(s, ev, 0));
    // an internal instance whose valence orbitals are the orbitals at k (its
    // real-space orbitals are what the density needs; no projectors, no
    // Hartree kernel, and any nonzero Q passes the checks)
    const int nks = sys->nks, nbnd = sys->nbnd;
    const int N = sys->nr[0] * sys->nr[1] * sys->nr[2];
    std::vector<double> zet((size_t)nks * nbnd, 0.0), zf((size_t)N, 0.0);
    lz_system g = *sys;
    g.q[0] = g.q[1] = g.q[2] = 0.0;
    g.g0[0] = 1;
    g.g0[1] = 0;
    g.g0[2] = 0;
    g.npw_kq = sys->npw_k;
    g.nl_kq = sys->nl_k;
    g.evc_kq = sys->evc_k;
    g.et_k = zet.data();
    g.fxc_r = zf.data();
    g.nproj = 0;
    g.vkb_kq = nullptr;
    g.dkb = nullptr;
    lz_options o{};
    o.prec = LZ_FP64;
    o.approx = LZ_IPA;
    o.max_steps = 1;
    o.projector_gemm = LZ_GEMM_VALU;
    std::unique_ptr<Instance> Ip = build_instance(g, o, s);
    Instance& I = *Ip;
    std::vector<double> w((size_t)I.nb);
    for (int b = 0; b < I.nb; ++b) w[b] = 2.0 * sys->wk[b / nbnd] / I.omega;
    DBuf dw, dn, df;
    upload(dw, w);
    dn.alloc((size_t)N * sizeof(double));
    df.alloc((size_t)N * sizeof(double));
    launch_ground_density(I.ur.p, dw.as<double>(), I.nb, N, xc == LZ_XC_PZ ? 1 : 0,
                          dn.as<double>(), df.as<double>(), s);
    HIPC(hipGetLastError());
    std::vector<double> hn(N), hf(N);
    HIPC(hipMemcpyAsync(hn.data(), dn.p, N * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(hf.data(), df.p, N * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    // plane-major [i3][i1][i2] -> the caller's (i1 N2 + i2) N3 + i3
    for (int i1 = 0; i1 < I.n1; ++i1)
      for (int i2 = 0; i2 < I.n2; ++i2)
        for (int i3 = 0; i3 < I.n3; ++i3) {
          const size_t src = ((size_t)i3 * I.n1 + i1) * I.n2 + i2;
          const size_t dst = ((size_t)i1 * I.n2 + i2) * I.n3 + i3;
          if (n0_out) n0_out[dst] = hn[src];
          if (fxc_out) fxc_out[dst] = hf[src];
        }
  });
}

}  // extern "C"

extern "C" {

lz_status lz_free(lz_ctx* c) {
  return guarded([&] {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    delete c;
  });
}

const char* lz_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
