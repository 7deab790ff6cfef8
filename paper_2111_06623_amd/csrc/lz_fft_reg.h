// Register-resident FFTs of whole lines for the cubic grid lengths of the
// production workloads (24, 32, 48, 64; 96 as a lane pair of 48-point lines).  One thread holds one line of N
// complex values and transforms it without any data exchange: N = R1 * R2
// with R1 in {8, 16} and R2 in {3, 4} is split as a Cooley-Tukey pair,
//   X[k1 + R1 k2] = sum_n2 W_N^{n2 k1} W_R2^{n2 k2} sum_n1 x[R2 n1 + n2] W_R1^{n1 k1},
// every index and twiddle being a compile-time constant.  Twiddles are
// rotations by multiples of 2 pi / 192 (192 is the least common multiple of
// the four lengths), applied as an exact quarter-turn times a rotation by
// less than pi/2 taken from a table of cosines.
#pragma once
#include <type_traits>

#include "lz_fft_ct.h"

namespace lz {

// cos(2 pi j / 192), j = 0..48
constexpr double kCos192[49] = {
    1.000000000000000000000, 0.999464587476365644430, 0.997858923238603506738,
    0.995184726672196886245, 0.991444861373810411145, 0.986643332084879004747,
    0.980785280403230449126, 0.973876979277333648150, 0.965925826289068286750,
    0.956940335732208864936, 0.946930129495105664256, 0.935905926757325700292,
    0.923879532511286756128, 0.910863824921175818573, 0.896872741532688303894,
    0.881921264348355029713, 0.866025403784438646764, 0.849202181526578887649,
    0.831469612302545237079, 0.812846684591615216579, 0.793353340291235164580,
    0.773010453362736960811, 0.751839807478977396408, 0.729864072697835657350,
    0.707106781186547524401, 0.683592302022871280513, 0.659345815100068868425,
    0.634393284163645498215, 0.608761429008720639416, 0.582477696867802149197,
    0.555570233019602224743, 0.528067850650367995873, 0.500000000000000000000,
    0.471396736825997648556, 0.442288690219001281995, 0.412707029804394737048,
    0.382683432365089771728, 0.352250047921233506532, 0.321439465303161580701,
    0.290284677254462367636, 0.258819045102520762349, 0.227076263034373207586,
    0.195090322016128267848, 0.162895473394588739481, 0.130526192220051591548,
    0.098017140329560601994, 0.065403129230143066815, 0.032719082821776142064,
    0.0};

// cos(2 pi j / 576), j = 0..144 (for lengths that do not divide 192: 72, 36, 9)
constexpr double kCos576[145] = {
    1.0, 0.99994050500014975, 0.99976202707990913, 0.99946458747636568,
    0.9990482215818578, 0.9985129789397631, 0.99785892323860348, 0.99708613230446663,
    0.99619469809174555, 0.99518472667219693, 0.99405633822231965, 0.99280966700905504,
    0.99144486137381038, 0.98996208371480787, 0.98836151046776066, 0.98664333208487898,
    0.98480775301220802, 0.98285499166530121, 0.98078528040323043, 0.97859886550093833,
    0.97629600711993336, 0.97387697927733363, 0.97134206981326143, 0.96869158035659308,
    0.96592582628906831, 0.96304513670776271, 0.96004985438592871, 0.95694033573220882,
    0.95371695074822693, 0.95038008298456111, 0.94693012949510569, 0.94336750078982523,
    0.93969262078590843, 0.93590592675732565, 0.93200786928279855, 0.92799891219218456,
    0.92387953251128674, 0.91965022040509226, 0.91531147911944721, 0.91086382492117579,
    0.90630778703664994, 0.90164390758881607, 0.89687274153268826, 0.89199485658931421,
    0.88701083317822171, 0.88192126434835505, 0.87672675570750769, 0.87142792535026137,
    0.86602540378443871, 0.860519833856079, 0.85491187067294661, 0.84920218152657889,
    0.84339144581288572, 0.8374803549513079, 0.83146961230254524, 0.82535993308486377,
    0.8191520442889918, 0.81284668459161524, 0.80644460426748255, 0.79994656510012974,
    0.79335334029123528, 0.78666571436861699, 0.77988448309288183, 0.77301045336273699,
    0.76604444311897801, 0.75898728124716186, 0.75183980747897738, 0.74460287229232625,
    0.73727733681012397, 0.7298640726978356, 0.72236396205975562, 0.7147778973340464,
    0.70710678118654757, 0.69935152640336706, 0.6915130557822694, 0.68359230202287136,
    0.67559020761566035, 0.66750772472984743, 0.65934581510006895, 0.65110544991194907,
    0.64278760968653936, 0.63439328416364549, 0.62592347218405919, 0.61737918157070493,
    0.60876142900872066, 0.60007123992448097, 0.59130964836358246, 0.58247769686780226,
    0.57357643635104616, 0.56460692597430051, 0.55557023301960229, 0.54646743276304344,
    0.53729960834682389, 0.5280678506503681, 0.51877325816052133, 0.50941693684084188,
    0.5, 0.49052356815930809, 0.48098876891938774, 0.47139673682599759,
    0.46174861323503386, 0.45204554617671966, 0.44228869021900125, 0.4324792063301664,
    0.42261826174069944, 0.41270702980439472, 0.40274668985873724, 0.39273842708457413,
    0.38268343236508984, 0.372582902144103, 0.36243803828370169, 0.3522500479212336,
    0.34202014332566882, 0.3317495417533522, 0.3214394653031617, 0.31109114077109085,
    0.30070579950427306, 0.29028467725446233, 0.2798290140309922, 0.26934005395322619,
    0.25881904510252096, 0.24826723937371628, 0.2376858923261731, 0.22707626303437323,
    0.2164396139381029, 0.20577721069223492, 0.19509032201612833, 0.18438021954266345,
    0.17364817766693041, 0.16289547339458882, 0.1521233861899168, 0.1413331978235674,
    0.13052619222005149, 0.11970365530496267, 0.10886687485196474, 0.09801714032956077,
    0.087155742747658138, 0.076283974503952273, 0.065403129230143048, 0.054514501638006321,
    0.043619387365336007, 0.032719082821776387, 0.021814885034561159, 0.010908091494182422,
    0.0};

template <int N> struct RegSplit;
template <> struct RegSplit<9> { static constexpr int R1 = 3, R2 = 3; };
template <> struct RegSplit<12> { static constexpr int R1 = 4, R2 = 3; };
template <> struct RegSplit<16> { static constexpr int R1 = 16, R2 = 1; };
template <> struct RegSplit<24> { static constexpr int R1 = 8, R2 = 3; };
template <> struct RegSplit<36> { static constexpr int R1 = 4, R2 = 9; };
template <> struct RegSplit<32> { static constexpr int R1 = 8, R2 = 4; };
template <> struct RegSplit<48> { static constexpr int R1 = 16, R2 = 3; };
template <> struct RegSplit<64> { static constexpr int R1 = 16, R2 = 4; };

template <int N> constexpr bool reg_fft_supported() {
  return N == 24 || N == 32 || N == 48 || N == 64;
}

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// a * exp(DIR 2 pi i J / 192)
template <typename T, int J, int DIR>
__device__ __forceinline__ cplx<T> w192(cplx<T> a) {
  constexpr int j = ((J % 192) + 192) % 192;
  constexpr int quarter = j / 48, r = j % 48;
  if constexpr (r != 0) {
    const T c = T(kCos192[r]);
    const T s = T(DIR * kCos192[48 - r]);
    a = mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
  }
  if constexpr (quarter == 1) return mul_i<T>(a, DIR);
  if constexpr (quarter == 2) return mk<T>(-a.x, -a.y);
  if constexpr (quarter == 3) return mul_i<T>(a, -DIR);
  return a;
}

// a * exp(DIR 2 pi i J / 576)
template <typename T, int J, int DIR>
__device__ __forceinline__ cplx<T> w576(cplx<T> a) {
  constexpr int j = ((J % 576) + 576) % 576;
  constexpr int quarter = j / 144, r = j % 144;
  if constexpr (r != 0) {
    const T c = T(kCos576[r]);
    const T s = T(DIR * kCos576[144 - r]);
    a = mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
  }
  if constexpr (quarter == 1) return mul_i<T>(a, DIR);
  if constexpr (quarter == 2) return mk<T>(-a.x, -a.y);
  if constexpr (quarter == 3) return mul_i<T>(a, -DIR);
  return a;
}

// a * exp(DIR 2 pi i NUM / N) from the table that holds it
template <typename T, int N, int NUM, int DIR>
__device__ __forceinline__ cplx<T> wtw(cplx<T> a) {
  if constexpr (192 % N == 0) return w192<T, (192 / N) * NUM, DIR>(a);
  else return w576<T, (576 / N) * NUM, DIR>(a);
}

// In-place transform of x (natural order in and out); DIR = -1 forward
// (exp(-i ..)), +1 inverse, unnormalised.
template <typename T, int N, int DIR>
__device__ __forceinline__ void reg_fft(cplx<T> (&x)[N]) {
  constexpr int R1 = RegSplit<N>::R1, R2 = RegSplit<N>::R2;
  if constexpr (R2 == 1) {
    Dft<T, N, DIR>::run(x);
  } else {
    cplx<T> y[R2][R1];
    sfor<0, R2>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      cplx<T> a[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n1] = x[R2 * n1 + n2];
      Dft<T, R1, DIR>::run(a);
      sfor<0, R1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        y[n2][k1] = wtw<T, N, n2 * k1, DIR>(a[k1]);
      });
    });
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cplx<T> b[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) b[n2] = y[n2][k1];
      if constexpr (R2 == 9) reg_fft<T, 9, DIR>(b);
      else Dft<T, R2, DIR>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = b[k2];
    }
  }
}

// Value held by the partner lane (lane ^ 1) of a lane pair (DPP quad
// permutation [1, 0, 3, 2]; both lanes of a pair are active wherever it is
// used).
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
template <typename T>
__device__ __forceinline__ cplx<T> pair_swap(cplx<T> v) {
  return mk<T>(pair_swap(v.x), pair_swap(v.y));
}

// Length-N transform shared by a lane pair (h = lane & 1), each lane holding
// N/2 values: a radix-2 step across the pair and a register transform of
// length N/2 on each lane.  With E and O the transforms of the even and odd
// samples, V[k] = E[k] + W^k O[k] and V[k + N/2] = E[k] - W^k O[k].
//   pair_fft_dit: in x[j] = v[2 j + h], out x[k] = V[h N/2 + k]
//   pair_fft_dif: in x[k] = v[h N/2 + k], out x[j] = V[2 j + h]
// The radix-2 step runs in groups of 8 values between scheduling barriers:
// scheduled freely, all of its temporaries were live at once (228 registers
// for a forward and an inverse transform against 136).
template <typename T, int N, int DIR>
__device__ __forceinline__ void pair_fft_dit(cplx<T> (&x)[N / 2], int h) {
  constexpr int M = N / 2;
  reg_fft<T, M, DIR>(x);
  sfor<0, M>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    const cplx<T> t = wtw<T, N, k, DIR>(x[k]);
    const cplx<T> own = h ? t : x[k];
    const cplx<T> other = pair_swap<T>(own);
    x[k] = h ? csub<T>(other, own) : cadd<T>(own, other);
  });
  __builtin_amdgcn_sched_barrier(0);
}

template <typename T, int N, int DIR>
__device__ __forceinline__ void pair_fft_dif(cplx<T> (&x)[N / 2], int h) {
  constexpr int M = N / 2;
  __builtin_amdgcn_sched_barrier(0);
  sfor<0, M>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    const cplx<T> other = pair_swap<T>(x[k]);
    const cplx<T> b = wtw<T, N, k, DIR>(csub<T>(other, x[k]));
    x[k] = h ? b : cadd<T>(x[k], other);
  });
  reg_fft<T, M, DIR>(x);
}

}  // namespace lz
