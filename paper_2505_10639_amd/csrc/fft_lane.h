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

// natural-order 8-point DFT on references
template <int DIR>
MFBD_HDI void dft8(float2& a0, float2& a1, float2& a2, float2& a3,
                                     float2& a4, float2& a5, float2& a6, float2& a7) {
  dft4<DIR>(a0, a2, a4, a6);  // E[0..3] in a0,a2,a4,a6
  dft4<DIR>(a1, a3, a5, a7);  // O[0..3] in a1,a3,a5,a7
  float2 o1 = twmul<DIR, 8, 1>(a3);
  float2 o2 = twmul<DIR, 8, 2>(a5);
  float2 o3 = twmul<DIR, 8, 3>(a7);
  float2 e0 = a0, e1 = a2, e2 = a4, e3 = a6, o0 = a1;
  a0 = cadd(e0, o0);
  a4 = csub(e0, o0);
  a1 = cadd(e1, o1);
  a5 = csub(e1, o1);
  a2 = cadd(e2, o2);
  a6 = csub(e2, o2);
  a3 = cadd(e3, o3);
  a7 = csub(e3, o3);
}

// 32-point DFT in natural order, 8 x 4 decomposition:
//   n = 4 n1 + n2, k = k1 + 8 k2;
//   X[k1 + 8 k2] = sum_n2 W32^{n2 k1} W4^{n2 k2} sum_n1 x[4 n1 + n2] W8^{n1 k1}.
template <int DIR>
MFBD_HDI void fft32(float2 (&x)[32]) {
  static_for<0, 4>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    dft8<DIR>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2], x[16 + n2], x[20 + n2], x[24 + n2],
              x[28 + n2]);
    // x[4*k1 + n2] now holds inner DFT output k1 for column n2
    static_for<1, 8>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      x[4 * k1 + n2] = twmul<DIR, 32, n2 * k1>(x[4 * k1 + n2]);
    });
  });
  float2 y[32];
  static_for<0, 8>([&](auto K1) {
    constexpr int k1 = decltype(K1)::value;
    float2 a0 = x[4 * k1 + 0], a1 = x[4 * k1 + 1], a2 = x[4 * k1 + 2], a3 = x[4 * k1 + 3];
    dft4<DIR>(a0, a1, a2, a3);
    y[k1 + 0] = a0;
    y[k1 + 8] = a1;
    y[k1 + 16] = a2;
    y[k1 + 24] = a3;
  });
  static_for<0, 32>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

// 64-point DFT in natural order, 8 x 8 decomposition (n = 8 n1 + n2).
template <int DIR>
MFBD_HDI void fft64(float2 (&x)[64]) {
  static_for<0, 8>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    dft8<DIR>(x[n2], x[8 + n2], x[16 + n2], x[24 + n2], x[32 + n2], x[40 + n2], x[48 + n2],
              x[56 + n2]);
    static_for<1, 8>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      x[8 * k1 + n2] = twmul<DIR, 64, n2 * k1>(x[8 * k1 + n2]);
    });
  });
  float2 y[64];
  static_for<0, 8>([&](auto K1) {
    constexpr int k1 = decltype(K1)::value;
    float2 a0 = x[8 * k1 + 0], a1 = x[8 * k1 + 1], a2 = x[8 * k1 + 2], a3 = x[8 * k1 + 3];
    float2 a4 = x[8 * k1 + 4], a5 = x[8 * k1 + 5], a6 = x[8 * k1 + 6], a7 = x[8 * k1 + 7];
    dft8<DIR>(a0, a1, a2, a3, a4, a5, a6, a7);
    y[k1 + 0] = a0;
    y[k1 + 8] = a1;
    y[k1 + 16] = a2;
    y[k1 + 24] = a3;
    y[k1 + 32] = a4;
    y[k1 + 40] = a5;
    y[k1 + 48] = a6;
    y[k1 + 56] = a7;
  });
  static_for<0, 64>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

}  // namespace mfbd
