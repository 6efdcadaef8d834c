// Wave-level 2-D transforms of one 128x128 MOMFBD unit (one workgroup of
// four wavefronts = 256 lanes).
//
// Layouts (lane l in [0,256)):
//   band-column  lane (q = l>>2, r = l&3): pupil band column vx = 32 + q, output
//                rows of residue r mod 4 (first pass of op1);
//   row-parity   lane (y = l>>1, e = l&1): image row y, columns 2m + e, m in [0,64);
//   column-quad  lane (r = l>>6, the wave, q = l&63): spectral column q, rows of
//                residue r mod 4 (the column passes of op2, op3, op4);
//   spectral SL  every lane: X(ky = 4m + r, kx = q), m in [0,32) (kx = 0 for
//                q = 0), and lanes l < 128 also X(ky = l, kx = 64).
//
// The pupil support lies in the central band [32,96) of both axes (diameter
// below N/2).  64- and 128-point sums fold into in-lane 32- and 64-point FFTs:
// band-limited inputs fold by output residue (the modulation of the folded
// sequence is a phase ramp the caller adds before the exponential), the
// 128-point column transforms split into four residue classes, one per wave
// (forward: a radix-4 fold of the inputs before a 32-point FFT; inverse: a
// 32-point FFT per class, then the radix-4 butterfly across the four waves
// through LDS), and the real row transforms pack even/odd samples into one
// complex sequence, with the halves exchanged between the two lanes of a row
// through LDS.  Every phase is a per-lane function; phases are separated by a
// workgroup barrier.  The residue class r is the wave index, so its twiddles
// W128^{nr} come from a table at a wave-uniform index (scalar loads).
#pragma once

#include "fft_lane.h"

namespace mfbd {
namespace n128 {

constexpr int N = 128;
constexpr int HC = 65;          // N/2 + 1
constexpr int BAND0 = 32;
constexpr int BW = 64;

// LDS strides (float2 units)
constexpr int U1 = 132;         // [q][ky]      op1 column pass -> rows
constexpr int U2 = 66;          // [y][kx]      rows -> columns (op2, op4)
constexpr int U3 = 65;          // [y][kx]      op3 columns -> rows
constexpr int LDS_MAIN = 128 * U2;     // 8448 float2 (>= 64*U1, 128*U3)
constexpr int LDS_HALF = 128 * U2;     // 8448 floats: the forward's half-size buffer
constexpr int LDS_AUX = 128;

// Residue class of a lane in the column-quad layout: its wave, uniform
// across the wave (a scalar register on the device).
MFBD_HDI int wave_of(int lane) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_readfirstlane(lane >> 6);
#else
  return lane >> 6;
#endif
}

MFBD_HDI int sl_index(int lane, int m) { return (4 * m + (lane >> 6)) * HC + (lane & 63); }
MFBD_HDI int sl_index64(int lane) { return lane * HC + 64; }

// cos and sin of 2 pi n r / 128 for the residue classes r in [0,4) and
// n in [0,32), rounded once from the FP64 constexpr evaluation.
struct Tw4 {
  float c[4][32];
  float s[4][32];
};
constexpr Tw4 make_tw4() {
  Tw4 t{};
  for (int r = 0; r < 4; ++r)
    for (int n = 0; n < 32; ++n) {
      const detail::CS cs = detail::cossin_2pi(n * r, 128);
      t.c[r][n] = float(cs.c);
      t.s[r][n] = float(cs.s);
    }
  return t;
}
constexpr Tw4 kTw4 = make_tw4();

// a * W128^{n r} (DIR as in twmul) for a wave-uniform r.
template <int DIR, int n>
MFBD_HDI float2 twmul_r(float2 a, int r) {
  const float c = kTw4.c[r][n], s = DIR * kTw4.s[r][n];
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// Forward radix-4 fold of column q of rows stored at T[y * U + q] for the
// lane's residue class r:
//   z[n] = W128^{-n r} sum_t (-i)^{t r} x(n + 32 t),   n in [0,32),
// so that X(4m + r) = FFT32(z)[m].  With a = x0 + (-1)^r x2 and
// b = x1 + (-1)^r x3, the sum is a + (-i)^r b.
template <int U>
MFBD_HDI void fold4_fwd(const float2* T, int q, int r, float2 (&z)[32]) {
  const float s = (r & 1) ? -1.0f : 1.0f;
  const float sg = (r & 2) ? -1.0f : 1.0f;
  auto ab = [&](int n, float2& a, float2& b) {
    const float2 x0 = T[n * U + q], x1 = T[(n + 32) * U + q];
    const float2 x2 = T[(n + 64) * U + q], x3 = T[(n + 96) * U + q];
    a = make_float2(x0.x + s * x2.x, x0.y + s * x2.y);
    b = make_float2(x1.x + s * x3.x, x1.y + s * x3.y);
  };
  if (r & 1) {         // (-i)^r b = sg (b.y, -b.x)
    static_for<0, 32>([&](auto I) {
      float2 a, b;
      ab(decltype(I)::value, a, b);
      z[decltype(I)::value] = make_float2(a.x + sg * b.y, a.y - sg * b.x);
    });
  } else {             // (-i)^r b = sg b
    static_for<0, 32>([&](auto I) {
      float2 a, b;
      ab(decltype(I)::value, a, b);
      z[decltype(I)::value] = make_float2(a.x + sg * b.x, a.y + sg * b.y);
    });
  }
  static_for<1, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    z[n] = twmul_r<-1, n>(z[n], r);
  });
}

// ---------------------------------------------------------------------------
// Op 1: inverse DFT of the band-limited pupil field.
// Column pass input of lane (q, r): z[n] = y[n] + y[n+32], n in [0,32), with
// y[n] = P(32+n, 32+q) W128^{+(32+n) r}.  Output rows ky = 4m + r.
// ---------------------------------------------------------------------------
MFBD_HDI void op1_cols(float2 (&z)[32], float2* T, int lane) {
  const int q = lane >> 2, r = lane & 3;
  fft32<+1>(z);
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    T[q * U1 + 4 * m + r] = z[m];
  });
}

// Row pass: lane (y, e) -> p(y, 2m + e), m in [0,64), from the row's band
// values p[q] = column pass output at (y, q).
MFBD_HDI void op1_rows_fft(float2 (&p)[64], int lane) {
  const int e = lane & 1;
  if (e) {
    static_for<0, 64>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      p[q] = twmul<+1, 128, 32 + q>(p[q]);
    });
  }
  fft64<+1>(p);
  static_for<0, 64>([&](auto M) {
    constexpr int m = decltype(M)::value;
    if constexpr (m & 1) p[m] = cneg(p[m]);
  });
}

// (The same steps written out for the full buffer: the 128x128 adjoint's
// register allocation depends on this form.)
MFBD_HDI void op1_rows(const float2* T, int lane, float2 (&p)[64]) {
  const int y = lane >> 1, e = lane & 1;
  static_for<0, 64>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    p[q] = T[q * U1 + y];
  });
  if (e) {
    static_for<0, 64>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      p[q] = twmul<+1, 128, 32 + q>(p[q]);
    });
  }
  fft64<+1>(p);
  static_for<0, 64>([&](auto M) {
    constexpr int m = decltype(M)::value;
    if constexpr (m & 1) p[m] = cneg(p[m]);
  });
}

// Half-buffer form of the op 1 transpose (the forward kernel): the column
// results go through a buffer of floats, real parts (P = 0), then
// imaginary parts (P = 1); the caller has run fft32<+1> on z, and puts
// after the buffer's previous readers are done, gets after a barrier.
template <int P>
MFBD_HDI void op1_cols_put(const float2 (&z)[32], float* Tf, int lane) {
  const int q = lane >> 2, r = lane & 3;
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    Tf[q * U1 + 4 * m + r] = P ? z[m].y : z[m].x;
  });
}
template <int P>
MFBD_HDI void op1_rows_get(const float* Tf, int lane, float2 (&p)[64]) {
  const int y = lane >> 1;
  static_for<0, 64>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    if (P) p[q].y = Tf[q * U1 + y];
    else p[q].x = Tf[q * U1 + y];
  });
}

// ---------------------------------------------------------------------------
// Exchange of 32 values between the two lanes of a row (lane l and l^1),
// staged in LDS.  The staging area aliases the main buffer, so callers put
// after the buffer's previous readers are done (barrier), get after a
// barrier, and write the buffer again only after another barrier.
// ---------------------------------------------------------------------------
template <class V>
MFBD_HDI void xput(const V (&v)[32], V* X, int lane) {
  static_for<0, 32>([&](auto I) { X[lane * 33 + decltype(I)::value] = v[decltype(I)::value]; });
}
template <class V>
MFBD_HDI void xget(const V* X, int lane, V (&o)[32]) {
  const int partner = lane ^ 1;
  static_for<0, 32>([&](auto I) { o[decltype(I)::value] = X[partner * 33 + decltype(I)::value]; });
}

// ---------------------------------------------------------------------------
// Op 2: forward DFT of a real image in row-parity layout -> half spectrum.
//   s_e[m] = s(y, 2m + e).  Packed row sequence z[n] = s(y,2n) + i s(y,2n+1);
//   lane e computes Z[2k'+e] of its 64-point DFT from the folds
//   z[n'] +- z[n'+32]: lane 0 folds the even samples, lane 1 the odd ones,
//   and each sends the other the fold it needs.
// ---------------------------------------------------------------------------
MFBD_HDI void op2_rows_fold(const float (&s)[64], float (&keep)[32], float (&send)[32], int lane) {
  const int e = lane & 1;
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    const float plus = s[n] + s[n + 32], minus = s[n] - s[n + 32];
    // lane 0 keeps the + fold (real part for k even) and sends the - fold;
    // lane 1 keeps the - fold (imag part for k odd) and sends the + fold
    keep[n] = e ? minus : plus;
    send[n] = e ? plus : minus;
  });
}

// The row's half spectrum as the lane's 32 values: v[kp] = Sr(y, 2 kp + e)
// (lane e = 0, kp = 0: the packed (Sr0, Sr64)), from the folds of HALF the
// image row (s / 2): then Sr[k] = (Z[k] + conj Z[64-k]) + W128^{-k} (Z[k] -
// conj Z[64-k]) / i with no factor 1/2, the twiddle in factored form.
MFBD_HDI void op2_rows_values(const float (&keep)[32], const float (&other)[32], int lane,
                              float2 (&v)[32]) {
  const int e = lane & 1;
  float2 w[32];
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    w[n] = e ? make_float2(other[n], keep[n]) : make_float2(keep[n], other[n]);
  });
  if (e) {
    static_for<1, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      w[n] = twmul<-1, 64, n>(w[n]);
    });
  }
  fft32<-1>(w);   // w[k'] = Z[2k' + e]
  // (a + c) + W128^{-k} (a - c) / i with a = Z[k], c = conj Z[64-k], k = e mod 2
  auto val = [](auto K, float2 a, float2 c) {
    constexpr int k = decltype(K)::value;
    const float2 t = twu<-1, 128, k>(make_float2(a.y - c.y, c.x - a.x));
    constexpr float f = twf<-1, 128, k>();
    return make_float2((a.x + c.x) + f * t.x, (a.y + c.y) + f * t.y);
  };
  if (e == 0) {
    v[0] = make_float2(2.0f * (w[0].x + w[0].y), 2.0f * (w[0].x - w[0].y));    // (Sr0, Sr64)
    static_for<1, 32>([&](auto K) {
      constexpr int kp = decltype(K)::value;      // k = 2 kp
      v[kp] = val(std::integral_constant<int, 2 * kp>{}, w[kp], cconj(w[32 - kp]));
    });
  } else {
    static_for<0, 32>([&](auto K) {
      constexpr int kp = decltype(K)::value;      // k = 2 kp + 1, partner 63 - 2kp
      v[kp] = val(std::integral_constant<int, 2 * kp + 1>{}, w[kp], cconj(w[31 - kp]));
    });
  }
}

MFBD_HDI void op2_rows_finish(const float (&keep)[32], const float (&other)[32], float2* T,
                              int lane) {
  const int y = lane >> 1, e = lane & 1;
  float2 v[32];
  op2_rows_values(keep, other, lane, v);
  static_for<0, 32>([&](auto K) {
    constexpr int kp = decltype(K)::value;
    T[y * U2 + 2 * kp + e] = v[kp];
  });
}

// Half-buffer form of the op 2 transpose: real parts (P = 0), then
// imaginary parts (P = 1), of the row values; the column pass folds each
// part as it arrives (op2_cols_half_x, then op2_cols_half_y, which finishes
// the column transform).
template <int P>
MFBD_HDI void op2_rows_put(const float2 (&v)[32], float* Tf, int lane) {
  const int y = lane >> 1, e = lane & 1;
  static_for<0, 32>([&](auto K) {
    constexpr int kp = decltype(K)::value;
    Tf[y * U2 + 2 * kp + e] = P ? v[kp].y : v[kp].x;
  });
}

// Real parts of the radix-4 fold's a = x0 + (-1)^r x2 and b = x1 + (-1)^r x3.
MFBD_HDI void op2_cols_half_x(const float* Tf, int lane, float (&ax)[32], float (&bx)[32]) {
  const int r = wave_of(lane), q = lane & 63;
  const float s = (r & 1) ? -1.0f : 1.0f;
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    ax[n] = Tf[n * U2 + q] + s * Tf[(n + 64) * U2 + q];
    bx[n] = Tf[(n + 32) * U2 + q] + s * Tf[(n + 96) * U2 + q];
  });
}

// Imaginary parts, the fold z = a + (-i)^r b, its twiddle and the 32-point
// FFT: X[m] = S(4m + r, q); column 0 left in Taux as in op2_cols.
MFBD_HDI void op2_cols_half_y(const float* Tf, float2* Taux, int lane, const float (&ax)[32],
                              const float (&bx)[32], float2 (&X)[32]) {
  const int r = wave_of(lane), q = lane & 63;
  const float s = (r & 1) ? -1.0f : 1.0f;
  const float sg = (r & 2) ? -1.0f : 1.0f;
  auto ab_y = [&](int n, float& ay, float& by) {
    ay = Tf[n * U2 + q] + s * Tf[(n + 64) * U2 + q];
    by = Tf[(n + 32) * U2 + q] + s * Tf[(n + 96) * U2 + q];
  };
  if (r & 1) {         // (-i)^r b = sg (b.y, -b.x)
    static_for<0, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      float ay, by;
      ab_y(n, ay, by);
      X[n] = make_float2(ax[n] + sg * by, ay - sg * bx[n]);
    });
  } else {             // (-i)^r b = sg b
    static_for<0, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      float ay, by;
      ab_y(n, ay, by);
      X[n] = make_float2(ax[n] + sg * bx[n], ay + sg * by);
    });
  }
  static_for<1, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    X[n] = twmul_r<-1, n>(X[n], r);
  });
  fft32<-1>(X);
  if (q == 0) {
    static_for<0, 32>([&](auto I) { Taux[4 * decltype(I)::value + r] = X[decltype(I)::value]; });
  }
}

// Column pass (all lanes): X[m] = S(4m + r, q), m in [0,32), for q >= 1;
// q = 0 holds the packed real columns 0 and 64 (see op2_unpack).
MFBD_HDI void op2_cols(const float2* T, float2* Taux, int lane, float2 (&X)[32]) {
  const int r = wave_of(lane), q = lane & 63;
  fold4_fwd<U2>(T, q, r, X);
  fft32<-1>(X);
  // column 0 packs the real columns kx = 0 and 64 (F = S0 + i S64, both
  // Hermitian in ky): left in Taux[ky] for op2_unpack
  if (q == 0) {
    static_for<0, 32>([&](auto I) { Taux[4 * decltype(I)::value + r] = X[decltype(I)::value]; });
  }
}

// After a barrier, lane ky < 128 unpacks row ky: returns S(ky, 64) and leaves
// S(ky, 0) in T[ky] (the column pass has read T).
MFBD_HDI float2 op2_unpack(const float2* Taux, float2* T, int lane) {
  const float2 f = Taux[lane], c = cconj(Taux[(128 - lane) & 127]);
  const float2 d = csub(f, c);
  T[lane] = cscale(cadd(f, c), 0.5f);
  return make_float2(0.5f * d.y, -0.5f * d.x);
}

// After another barrier, the lanes of column 0 take X[m] = S(4m + r, 0).
MFBD_HDI void op2_collect(const float2* T, int lane, float2 (&X)[32]) {
  if ((lane & 63) == 0) {
    const int r = wave_of(lane);
    static_for<0, 32>([&](auto I) { X[decltype(I)::value] = T[4 * decltype(I)::value + r]; });
  }
}

// ---------------------------------------------------------------------------
// Op 3: inverse DFT of a Hermitian half spectrum (SL; X(ky, 64) in Taux[ky])
// -> real image in row-parity layout.
// Column pass in three steps separated by barriers.  First, the lane's
// residue class: Y_r[n] = W128^{+n r} sum_m X(4m + r, q) W32^{+n m} into
// T[(32 r + n) U3 + q] (column 0 packs X(ky, 64) as its imaginary part).
// Then the radix-4 butterfly across the column's four lanes,
// x(32 r + n, q) = sum_r' i^{r r'} Y_r'[n], held in registers, and after a
// barrier written over T[(32 r + n) U3 + q]: T then holds the column
// transforms in natural row order.
// ---------------------------------------------------------------------------
MFBD_HDI void op3_cols_put(const float2 (&X)[32], float2* T, int lane) {
  const int r = wave_of(lane), q = lane & 63;
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    T[(32 * r + n) * U3 + q] = X[n];
  });
}

MFBD_HDI void op3_cols(float2 (&X)[32], const float2* Taux, float2* T, int lane) {
  const int r = wave_of(lane), q = lane & 63;
  if (q == 0) {
    static_for<0, 32>([&](auto I) {
      constexpr int m = decltype(I)::value;
      const float2 g64 = Taux[4 * m + r];
      X[m] = make_float2(X[m].x - g64.y, X[m].y + g64.x);
    });
  }
  fft32<+1>(X);
  static_for<1, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    X[n] = twmul_r<+1, n>(X[n], r);
  });
  op3_cols_put(X, T, lane);
}

// With a = Y0 + (-1)^r Y2 and b = Y1 + (-1)^r Y3, the sum is a + i^r b.
MFBD_HDI void op3_cols_combine(const float2* T, int lane, float2 (&X)[32]) {
  const int r = wave_of(lane), q = lane & 63;
  const float s = (r & 1) ? -1.0f : 1.0f;
  const float sg = (r & 2) ? -1.0f : 1.0f;
  auto ab = [&](int n, float2& a, float2& b) {
    const float2 y0 = T[n * U3 + q], y1 = T[(32 + n) * U3 + q];
    const float2 y2 = T[(64 + n) * U3 + q], y3 = T[(96 + n) * U3 + q];
    a = make_float2(y0.x + s * y2.x, y0.y + s * y2.y);
    b = make_float2(y1.x + s * y3.x, y1.y + s * y3.y);
  };
  if (r & 1) {         // i^r b = sg (-b.y, b.x)
    static_for<0, 32>([&](auto I) {
      float2 a, b;
      ab(decltype(I)::value, a, b);
      X[decltype(I)::value] = make_float2(a.x - sg * b.y, a.y + sg * b.x);
    });
  } else {             // i^r b = sg b
    static_for<0, 32>([&](auto I) {
      float2 a, b;
      ab(decltype(I)::value, a, b);
      X[decltype(I)::value] = make_float2(a.x + sg * b.x, a.y + sg * b.y);
    });
  }
}

// Row pass (all lanes): lane (y, f) forms the row half spectrum, then the
// parity-f half of the packed inverse, z[2n'+f], n' in [0,32).  It keeps the
// part of z that belongs to its own column parity and sends the other part.
//   X[k] (k in [0,64]) from the column pass (row y of T; column 0 packs the
//   real columns 0 and 64);
//   Z[k] = (X[k] + X[k+64]) + i W128^{+k} (X[k] - X[k+64]), X[k+64] = conj X[64-k];
//   w[k'] = Z[k'] + (-1)^f Z[k'+32], k' in [0,32).
// The values are read from LDS in groups {k, 64-k, 32+k, 32-k}, which give
// Z at those four points and hence w[k] and w[32-k]; neither X nor Z is
// ever held whole (register pressure).
MFBD_HDI void op3_rows_compute(const float2* T, int lane, float (&keep)[32], float (&send)[32]) {
  const int y = lane >> 1, f = lane & 1;
  const float sf = f ? -1.0f : 1.0f;
  auto xr = [&](int q) { return T[y * U3 + q]; };
  // Z at k and 64 - k from X[k], X[64-k] (1 <= k <= 63)
  auto zpair = [&](auto K, float2 xa, float2 xb, float2& za, float2& zb) {
    constexpr int k = decltype(K)::value;
    {   // s + i W128^k (xa - c), the twiddle in factored form
      const float2 c = cconj(xb);
      const float2 s = cadd(xa, c);
      const float2 t = twu<+1, 128, k>(csub(xa, c));
      constexpr float f = twf<+1, 128, k>();
      za = make_float2(s.x - f * t.y, s.y + f * t.x);
    }
    {
      const float2 c = cconj(xa);
      const float2 s = cadd(xb, c);
      const float2 t = twu<+1, 128, 64 - k>(csub(xb, c));
      constexpr float f = twf<+1, 128, 64 - k>();
      zb = make_float2(s.x - f * t.y, s.y + f * t.x);
    }
  };
  auto wmix = [&](float2 za, float2 zb) {
    return make_float2(za.x + sf * zb.x, za.y + sf * zb.y);
  };
  float2 w[32];
  {
    // k = 0 (X[0] packs the real X(r,0), X(r,64)) and k = 32 (its own pair)
    const float2 x0 = xr(0), x32 = xr(32);
    const float2 z0 = make_float2(x0.x + x0.y, x0.x - x0.y);
    const float2 c = cconj(x32);
    const float2 s2 = cadd(x32, c);
    const float2 t = twmul<+1, 128, 32>(csub(x32, c));
    const float2 z32 = make_float2(s2.x - t.y, s2.y + t.x);
    w[0] = wmix(z0, z32);
  }
  {
    // k = 16: Z[16], Z[48] from X[16], X[48]
    float2 z16, z48;
    zpair(std::integral_constant<int, 16>{}, xr(16), xr(48), z16, z48);
    w[16] = wmix(z16, z48);
  }
  static_for<1, 16>([&](auto K) {
    constexpr int k = decltype(K)::value;
    float2 zk, z64k, z32k, z32mk;
    zpair(std::integral_constant<int, k>{}, xr(k), xr(64 - k), zk, z64k);
    zpair(std::integral_constant<int, 32 - k>{}, xr(32 - k), xr(32 + k), z32mk, z32k);
    w[k] = wmix(zk, z32k);             // Z[k] +- Z[k+32]
    w[32 - k] = wmix(z32mk, z64k);     // Z[32-k] +- Z[64-k]
  });
  if (f) {
    static_for<1, 32>([&](auto I) {
      constexpr int k = decltype(I)::value;
      w[k] = twmul<+1, 64, k>(w[k]);
    });
  }
  fft32<+1>(w);   // w[n'] = z[2n' + f] = g(4n'+2f) + i g(4n'+2f+1)
  // lane f = 0 owns even columns: keeps Re (x = 4n'), sends Im (x = 4n'+1);
  // lane f = 1 owns odd columns: keeps Im (x = 4n'+3), sends Re (x = 4n'+2)
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    keep[n] = f ? w[n].y : w[n].x;
    send[n] = f ? w[n].x : w[n].y;
  });
}

// g[m] = g(y, 2m + e), m in [0,64).
MFBD_HDI void op3_rows_finish(const float (&keep)[32], const float (&other)[32], int lane,
                              float (&g)[64]) {
  const int e = lane & 1;
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    // e = 0: m = 2n (x = 4n) own, m = 2n+1 (x = 4n+2) from the partner
    // e = 1: m = 2n (x = 4n+1) from the partner, m = 2n+1 (x = 4n+3) own
    g[2 * n] = e ? other[n] : keep[n];
    g[2 * n + 1] = e ? keep[n] : other[n];
  });
}

// ---------------------------------------------------------------------------
// Op 4: forward DFT of a complex image in row-parity layout, sampled on the
// band: G(vy, vx) for vx in [32,96) (rows), then vy in [32,96) (columns).
// Row pass: lane (y, e) transforms its parity half, F = DFT64((-1)^m H_e);
// G_r(32 + v') = F_0[v'] + W128^{-(32+v')} F_1[v'].  Lane 0 produces
// v' in [0,32), lane 1 v' in [32,64); each keeps the half it uses (lane 0:
// F_0[v], lane 1: F_1[32+v]) in keep and stages the other in X for its
// partner (same LDS rules as xput).  The 8 x 8 transform hands its outputs
// over group by group: output k1 + 8j of group k1 pairs with k1 + 8(j+4),
// so the 64 outputs are never held at once, and the halves are chosen value
// by value (selects, never a runtime index into an array).
MFBD_HDI void op4_rows_fft(float2 (&H)[64], float2 (&keep)[32], float2* X, int lane) {
  const bool odd = lane & 1;
  static_for<0, 64>([&](auto I) {
    constexpr int m = decltype(I)::value;
    if constexpr (m & 1) H[m] = cneg(H[m]);
  });
  static_for<0, 8>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    dft8<-1>(H[n2], H[8 + n2], H[16 + n2], H[24 + n2], H[32 + n2], H[40 + n2], H[48 + n2],
             H[56 + n2]);
  });
  // second stage: the twiddles W64^{n2 k1} in factored form (as fft64)
  static_for<0, 8>([&](auto K1) {
    constexpr int k = decltype(K1)::value;
    float2 a0 = H[8 * k + 0], a1 = twu<-1, 64, k>(H[8 * k + 1]),
           a2 = twu<-1, 64, 2 * k>(H[8 * k + 2]), a3 = twu<-1, 64, 3 * k>(H[8 * k + 3]),
           a4 = twu<-1, 64, 4 * k>(H[8 * k + 4]), a5 = twu<-1, 64, 5 * k>(H[8 * k + 5]),
           a6 = twu<-1, 64, 6 * k>(H[8 * k + 6]), a7 = twu<-1, 64, 7 * k>(H[8 * k + 7]);
    dft8s<-1>(a0, a1, a2, a3, a4, a5, a6, a7, twf<-1, 64, k>(), twf<-1, 64, 2 * k>(),
              twf<-1, 64, 3 * k>(), twf<-1, 64, 4 * k>(), twf<-1, 64, 5 * k>(),
              twf<-1, 64, 6 * k>(), twf<-1, 64, 7 * k>());
    constexpr int k1 = k;
    const float2 lo[4] = {a0, a1, a2, a3}, hi[4] = {a4, a5, a6, a7};   // F[v], F[32 + v]
    static_for<0, 4>([&](auto J) {
      constexpr int j = decltype(J)::value, v = k1 + 8 * j;
      keep[v] = odd ? hi[j] : lo[j];
      X[lane * 33 + v] = odd ? lo[j] : hi[j];
    });
  });
}

MFBD_HDI void op4_rows_finish(const float2 (&keep)[32], const float2 (&other)[32], float2* T,
                              int lane) {
  const int y = lane >> 1, e = lane & 1;
  // a + W128^-E b, the twiddle in factored form
  auto comb = [](auto E, float2 a, float2 b) {
    constexpr int E_ = decltype(E)::value;
    const float2 t = twu<-1, 128, E_>(b);
    constexpr float f = twf<-1, 128, E_>();
    return make_float2(a.x + f * t.x, a.y + f * t.y);
  };
  if (e == 0) {
    static_for<0, 32>([&](auto I) {
      constexpr int v = decltype(I)::value;       // keep = F_0[v], other = F_1[v]
      T[y * U2 + v] = comb(std::integral_constant<int, 32 + v>{}, keep[v], other[v]);
    });
  } else {
    static_for<0, 32>([&](auto I) {
      constexpr int v = decltype(I)::value;       // keep = F_1[32+v], other = F_0[32+v]
      T[y * U2 + 32 + v] = comb(std::integral_constant<int, 64 + v>{}, other[v], keep[v]);
    });
  }
}

// Column pass (all lanes): GP[i] = G(vy = 32 + 4i + r, vx = 32 + q), i in [0,16).
MFBD_HDI void op4_cols(const float2* T, int lane, float2 (&GP)[16]) {
  const int r = wave_of(lane), q = lane & 63;
  float2 X[32];
  fold4_fwd<U2>(T, q, r, X);
  fft32<-1>(X);
  static_for<0, 16>([&](auto I) { GP[decltype(I)::value] = X[8 + decltype(I)::value]; });
}

}  // namespace n128
}  // namespace mfbd
