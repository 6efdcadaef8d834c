// In-register FFT building blocks for one lane (gfx950, wave64).
//
// Every transform here runs inside a single lane on a register array with
// compile-time indices, so after unrolling the data never leaves VGPRs.
// Twiddle factors are compile-time constants: cos/sin of 2*pi*e/L are
// evaluated in double precision by a constexpr Taylor series after an exact
// octant reduction of the rational angle e/L, then rounded once to float.
//
// Direction convention: W_L^e = exp(DIR * 2*pi*i*e/L); DIR = -1 is the
// forward DFT sum_r x(r) exp(-2 pi i u r / L), DIR = +1 the unnormalised
// inverse sum_u X(u) exp(+2 pi i u r / L).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

// Per-lane code is host+device so that the same index logic can be run by a
// host emulation of one wave (test harness) as well as on the GPU.
#define MFBD_HDI __host__ __device__ __forceinline__

namespace mfbd {

// ----------------------------------------------------------------- complex
MFBD_HDI float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
MFBD_HDI float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
MFBD_HDI float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
MFBD_HDI float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
MFBD_HDI float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
MFBD_HDI float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }
MFBD_HDI float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
MFBD_HDI float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// --------------------------------------------------- compile-time loops
template <int I, int N, class F>
MFBD_HDI void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ------------------------------------------- constexpr trigonometry (FP64)
namespace detail {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double sin_series(double x) {  // |x| <= pi/4
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {  // |x| <= pi/4
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2*pi*e/L for integers, with exact reduction to [0, pi/4].
struct CS { double c, s; };
constexpr CS cossin_2pi(long e, long L) {
  long r = ((e % L) + L) % L;        // angle = 2 pi r / L in [0, 2 pi)
  long q = (4 * r) / L;              // quadrant
  long rr = 4 * r - q * L;           // angle within quadrant = (pi/2) rr / L
  bool swap = (2 * rr > L);          // past pi/4: use the complement
  long num = swap ? (L - rr) : rr;   // reduced angle = (pi/2) num / L <= pi/4
  double a = 0.5 * kPi * double(num) / double(L);
  double c0 = cos_series(a), s0 = sin_series(a);
  double c = swap ? s0 : c0, s = swap ? c0 : s0;  // cos/sin of (pi/2) rr/L
  switch (q) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}
}  // namespace detail

// x * W_L^E with W_L = exp(DIR * 2 pi i / L); trivial factors cost nothing.
template <int DIR, int L, int E>
MFBD_HDI float2 twmul(float2 a) {
  constexpr int e = ((E % L) + L) % L;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == L) {
    return cneg(a);
  } else if constexpr (4 * e == L) {           // W = DIR * i
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else if constexpr (4 * e == 3 * L) {       // W = -DIR * i
    return DIR > 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  } else {
    constexpr detail::CS cs = detail::cossin_2pi(e, L);
    constexpr float c = float(cs.c);
    constexpr float s = float(DIR * cs.s);
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// The constant W_L^E itself (float2), for code that needs it as a value.
template <int DIR, int L, int E>
MFBD_HDI float2 twval() {
  constexpr detail::CS cs = detail::cossin_2pi(E, L);
  return make_float2(float(cs.c), float(DIR * cs.s));
}

// --------------------------------------------------- factored twiddles
// A twiddle W = c + i s is written f u with f the larger-magnitude of its
// components (|f| >= 1/sqrt 2) and u = 1 + i s/c (f = c) or c/s + i (f = s),
// whose other component has magnitude <= 1.  x u takes two FMAs, and the
// butterfly y +- W x = y +- f (x u) two more per output, so the factor f of
// every twiddle is carried into the FMAs of the butterfly that follows it
// (Linzer and Feig's scaled-twiddle form of the radix-2^k butterfly): a
// twiddled butterfly costs 6 instructions instead of 8.
namespace detail {
struct TF {
  double f, t;
  int kind;   // 0: u = 1 + i t, 1: u = t + i
};
constexpr double dabs(double x) { return x < 0 ? -x : x; }
constexpr TF twfact(int dir, long e, long L) {
  const CS cs = cossin_2pi(e, L);
  const double c = cs.c, s = dir * cs.s;
  return dabs(c) >= dabs(s) ? TF{c, s / c, 0} : TF{s, c / s, 1};
}
}  // namespace detail

// the real factor f of W_L^E (DIR as for twmul)
template <int DIR, int L, int E>
MFBD_HDI constexpr float twf() {
  return float(detail::twfact(DIR, ((E % L) + L) % L, L).f);
}

// x u, u the unit factor of W_L^E (W_L^E = twf() u)
template <int DIR, int L, int E>
MFBD_HDI float2 twu(float2 x) {
  constexpr detail::TF tf = detail::twfact(DIR, ((E % L) + L) % L, L);
  constexpr float t = float(tf.t);
  if constexpr (tf.kind == 0) {
    if constexpr (tf.t == 0.0) return x;
    else return make_float2(x.x - t * x.y, x.y + t * x.x);
  } else {
    if constexpr (tf.t == 0.0) return make_float2(-x.y, x.x);
    else return make_float2(t * x.x - x.y, t * x.y + x.x);
  }
}

// ----------------------------------------------------------- small DFTs
template <int DIR>
MFBD_HDI void dft2(float2& a0, float2& a1) {
  float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <int DIR>
MFBD_HDI void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = twmul<DIR, 4, 1>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 4-point DFT of (a0, s1 a1, s2 a2, s3 a3) for real constants s1..s3 (the
// factors of twiddles already applied to a1..a3 as twu): every add is an
// FMA, so the scales cost nothing.  Natural order, results in a0..a3.
template <int DIR>
MFBD_HDI void dft4s(float2& a0, float2& a1, float2& a2, float2& a3, float s1, float s2,
                    float s3) {
  const float r = s3 / s1;
  const float2 t0 = make_float2(a0.x + s2 * a2.x, a0.y + s2 * a2.y);
  const float2 t1 = make_float2(a0.x - s2 * a2.x, a0.y - s2 * a2.y);
  const float2 p = make_float2(a1.x + r * a3.x, a1.y + r * a3.y);   // (a1 + s3/s1 a3)
  const float2 m = make_float2(a1.x - r * a3.x, a1.y - r * a3.y);
  const float d = DIR * s1;   // (DIR i) s1 m = (-d m.y, d m.x)
  a0 = make_float2(t0.x + s1 * p.x, t0.y + s1 * p.y);
  a2 = make_float2(t0.x - s1 * p.x, t0.y - s1 * p.y);
  a1 = make_float2(t1.x - d * m.y, t1.y + d * m.x);
  a3 = make_float2(t1.x + d * m.y, t1.y - d * m.x);
}

// 8-point DFT of (a0, s1 a1, ..., s7 a7) (s0 = 1), natural order: the even
// and odd halves as scaled 4-point DFTs (the odd one relative to s1), then
// the W8 butterflies with their factors carried into the FMAs.
template <int DIR>
MFBD_HDI void dft8s(float2& a0, float2& a1, float2& a2, float2& a3, float2& a4, float2& a5,
                    float2& a6, float2& a7, float s1, float s2, float s3, float s4, float s5,
                    float s6, float s7) {
  dft4s<DIR>(a0, a2, a4, a6, s2, s4, s6);                  // E[0..3] in a0,a2,a4,a6
  dft4s<DIR>(a1, a3, a5, a7, s3 / s1, s5 / s1, s7 / s1);   // O[0..3] / s1 in a1,a3,a5,a7
  const float2 o0 = a1, o1 = twu<DIR, 8, 1>(a3), o2 = twu<DIR, 8, 2>(a5), o3 = twu<DIR, 8, 3>(a7);
  const float f0 = s1, f1 = s1 * twf<DIR, 8, 1>(), f2 = s1 * twf<DIR, 8, 2>(),
              f3 = s1 * twf<DIR, 8, 3>();
  const float2 e0 = a0, e1 = a2, e2 = a4, e3 = a6;
  a0 = make_float2(e0.x + f0 * o0.x, e0.y + f0 * o0.y);
  a4 = make_float2(e0.x - f0 * o0.x, e0.y - f0 * o0.y);
  a1 = make_float2(e1.x + f1 * o1.x, e1.y + f1 * o1.y);
  a5 = make_float2(e1.x - f1 * o1.x, e1.y - f1 * o1.y);
  a2 = make_float2(e2.x + f2 * o2.x, e2.y + f2 * o2.y);
  a6 = make_float2(e2.x - f2 * o2.x, e2.y - f2 * o2.y);
  a3 = make_float2(e3.x + f3 * o3.x, e3.y + f3 * o3.y);
  a7 = make_float2(e3.x - f3 * o3.x, e3.y - f3 * o3.y);
}

// natural-order 8-point DFT on references
template <int DIR>
MFBD_HDI void dft8(float2& a0, float2& a1, float2& a2, float2& a3,
                                     float2& a4, float2& a5, float2& a6, float2& a7) {
  dft8s<DIR>(a0, a1, a2, a3, a4, a5, a6, a7, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f);
}

// 32-point DFT in natural order, 8 x 4 decomposition:
//   n = 4 n1 + n2, k = k1 + 8 k2;
//   X[k1 + 8 k2] = sum_n2 W32^{n2 k1} W4^{n2 k2} sum_n1 x[4 n1 + n2] W8^{n1 k1}.
// The twiddles W32^{n2 k1} enter the second-stage 4-point DFTs in factored
// form.
template <int DIR>
MFBD_HDI void fft32(float2 (&x)[32]) {
  static_for<0, 4>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    dft8<DIR>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2], x[16 + n2], x[20 + n2], x[24 + n2],
              x[28 + n2]);
  });
  float2 y[32];
  static_for<0, 8>([&](auto K1) {
    constexpr int k1 = decltype(K1)::value;
    float2 a0 = x[4 * k1 + 0], a1 = twu<DIR, 32, k1>(x[4 * k1 + 1]),
           a2 = twu<DIR, 32, 2 * k1>(x[4 * k1 + 2]), a3 = twu<DIR, 32, 3 * k1>(x[4 * k1 + 3]);
    dft4s<DIR>(a0, a1, a2, a3, twf<DIR, 32, k1>(), twf<DIR, 32, 2 * k1>(),
               twf<DIR, 32, 3 * k1>());
    y[k1 + 0] = a0;
    y[k1 + 8] = a1;
    y[k1 + 16] = a2;
    y[k1 + 24] = a3;
  });
  static_for<0, 32>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

// Input factors of a transform whose input x[n] is c[n] W_L^{E0 + n} (a
// phase ramp), passed as x[n] = twu(c[n]) with the factor f(n) left out.
template <int DIR, int L, int E0>
struct RampFactors {
  static MFBD_HDI constexpr float f(int n) {
    return float(detail::twfact(DIR, (((E0 + n) % L) + L) % L, L).f);
  }
};

// fft32 of (f(0) x[0], f(1) x[1], ..., f(31) x[31]) for the compile-time
// input factors SC::f, with f(0) = 1: the factors enter the FMAs of the
// first-stage 8-point DFTs (relative to the first input of each) and of the
// second stage, so they cost nothing.
template <int DIR, class SC>
MFBD_HDI void fft32s(float2 (&x)[32]) {
  static_assert(SC::f(0) == 1.0f, "the first input factor must be 1");
  static_for<0, 4>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    constexpr float s0 = SC::f(n2);
    dft8s<DIR>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2], x[16 + n2], x[20 + n2], x[24 + n2],
               x[28 + n2], SC::f(4 + n2) / s0, SC::f(8 + n2) / s0, SC::f(12 + n2) / s0,
               SC::f(16 + n2) / s0, SC::f(20 + n2) / s0, SC::f(24 + n2) / s0,
               SC::f(28 + n2) / s0);
  });
  // first-stage output k1 of column n2 carries the factor f(n2)
  float2 y[32];
  static_for<0, 8>([&](auto K1) {
    constexpr int k1 = decltype(K1)::value;
    float2 a0 = x[4 * k1 + 0], a1 = twu<DIR, 32, k1>(x[4 * k1 + 1]),
           a2 = twu<DIR, 32, 2 * k1>(x[4 * k1 + 2]), a3 = twu<DIR, 32, 3 * k1>(x[4 * k1 + 3]);
    dft4s<DIR>(a0, a1, a2, a3, twf<DIR, 32, k1>() * SC::f(1), twf<DIR, 32, 2 * k1>() * SC::f(2),
               twf<DIR, 32, 3 * k1>() * SC::f(3));
    y[k1 + 0] = a0;
    y[k1 + 8] = a1;
    y[k1 + 16] = a2;
    y[k1 + 24] = a3;
  });
  static_for<0, 32>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

// 64-point DFT in natural order, 8 x 8 decomposition (n = 8 n1 + n2), the
// twiddles W64^{n2 k1} in factored form in the second-stage 8-point DFTs.
template <int DIR>
MFBD_HDI void fft64(float2 (&x)[64]) {
  static_for<0, 8>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    dft8<DIR>(x[n2], x[8 + n2], x[16 + n2], x[24 + n2], x[32 + n2], x[40 + n2], x[48 + n2],
              x[56 + n2]);
  });
  float2 y[64];
  static_for<0, 8>([&](auto K1) {
    constexpr int k = decltype(K1)::value;
    float2 a0 = x[8 * k + 0], a1 = twu<DIR, 64, k>(x[8 * k + 1]),
           a2 = twu<DIR, 64, 2 * k>(x[8 * k + 2]), a3 = twu<DIR, 64, 3 * k>(x[8 * k + 3]),
           a4 = twu<DIR, 64, 4 * k>(x[8 * k + 4]), a5 = twu<DIR, 64, 5 * k>(x[8 * k + 5]),
           a6 = twu<DIR, 64, 6 * k>(x[8 * k + 6]), a7 = twu<DIR, 64, 7 * k>(x[8 * k + 7]);
    dft8s<DIR>(a0, a1, a2, a3, a4, a5, a6, a7, twf<DIR, 64, k>(), twf<DIR, 64, 2 * k>(),
               twf<DIR, 64, 3 * k>(), twf<DIR, 64, 4 * k>(), twf<DIR, 64, 5 * k>(),
               twf<DIR, 64, 6 * k>(), twf<DIR, 64, 7 * k>());
    y[k + 0] = a0;
    y[k + 8] = a1;
    y[k + 16] = a2;
    y[k + 24] = a3;
    y[k + 32] = a4;
    y[k + 40] = a5;
    y[k + 48] = a6;
    y[k + 56] = a7;
  });
  static_for<0, 64>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

}  // namespace mfbd
