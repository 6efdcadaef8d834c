// Wave-level 2-D transforms of one 64x64 MOMFBD unit (one wavefront = 64 lanes).
//
// Data layouts inside a wave (lane l, q = l >> 1, b = l & 1):
//   band-column layout  lane (q,b) holds the pupil band column vx = 16 + q,
//                       rows vy = 16 + n, n in [0,32);
//   row layout          lane l holds image row r = l, columns in two 32-element
//                       halves: even columns (2n) and odd columns (2n+1);
//   spectral layout SL  lane (q,b) holds X(ky = 2m + b, kx = q), m in [0,32)
//                       (kx = 0 for q = 0), plus one extra value X(ky = l, kx = 32).
//
// The pupil support is confined to the central band [16,48) of both axes
// (diameter < N/2, which also keeps the OTF free of aliasing), so the first
// inverse transform of the pupil and the last forward transform back to it
// only touch a 32-wide band.  Every 64-point transform is then assembled from
// in-lane 32-point FFTs:
//   * a 64-point sum whose input lives in a 32-wide band, or whose output is
//     wanted at one parity of frequency, folds into a 32-point DFT;
//   * lane pairs (q,0), (q,1) split the two output parities of a column.
// One transpose through LDS per 2-D transform.
//
// Each operator is split into phases separated by a wave barrier; phases are
// per-lane functions so that a host harness can run them lane by lane.
#pragma once

#include "fft_lane.h"

namespace mfbd {
namespace n64 {

constexpr int N = 64;
constexpr int HC = 33;       // N/2 + 1 columns of a half spectrum
constexpr int BAND0 = 16;    // first row/column of the pupil band
constexpr int BW = 32;       // band width

// LDS strides in float2 units, chosen so that both the writing and the
// reading pattern of each transpose hit distinct banks.
constexpr int T1 = 66;       // [q][ky]     band-column IFFT -> rows
constexpr int T2 = 33;       // [r][q]      rows -> columns
constexpr int T3 = 65;       // [r'][2q+b]  columns -> rows (c2r)
constexpr int LDS_MAIN = 64 * T2 + 32;   // float2 elements of the main buffer (>= 32*T1, 32*T3)
constexpr int LDS_AUX = 64;              // float2 elements of the side buffer

// Index of spectral-layout element m of lane l in a [N][N/2+1] array.
MFBD_HDI int sl_index(int lane, int m) { return (2 * m + (lane & 1)) * HC + (lane >> 1); }
MFBD_HDI int sl_index32(int lane) { return lane * HC + 32; }

// ---------------------------------------------------------------------------
// Op 1: inverse 2-D DFT of the band-limited pupil field -> complex PSF amplitude.
//   p(r) = sum_v P(v) exp(+2 pi i v.r / 64), P zero outside the band.
// Input of lane (q,b): y[n] = P(16+n, 16+q) * W64^{+b(16+n)}.
// ---------------------------------------------------------------------------
MFBD_HDI void op1_cols(float2 (&y)[32], float2* T, int lane) {
  const int q = lane >> 1, b = lane & 1;
  fft32<+1>(y);
  // column value at ky = 2m + b is (-1)^m y[m]
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    float2 v = (m & 1) ? cneg(y[m]) : y[m];
    T[q * T1 + 2 * m + b] = v;
  });
}

// Output: pe[m] = p(r, 2m), po[m] = p(r, 2m+1) for row r = lane.
// The odd half's input is c[q] W64^{16+q}: the ramp enters fft32s as
// factored twiddles (RampFactors).
using Ramp16 = RampFactors<+1, 64, 16>;

MFBD_HDI void op1_rows(const float2* T, int lane, float2 (&pe)[32], float2 (&po)[32]) {
  static_for<0, 32>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    float2 c = T[q * T1 + lane];
    pe[q] = c;
    po[q] = twu<+1, 64, 16 + q>(c);
  });
  fft32<+1>(pe);
  fft32s<+1, Ramp16>(po);
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    if constexpr (m & 1) {
      pe[m] = cneg(pe[m]);
      po[m] = cneg(po[m]);
    }
  });
}

// ---------------------------------------------------------------------------
// Op 2: forward 2-D DFT of a real image held in row layout -> half spectrum
// in spectral layout.  Input: se[n] = s(r, 2n), so[n] = s(r, 2n+1).
// ---------------------------------------------------------------------------
MFBD_HDI void op2_rows(const float (&se)[32], const float (&so)[32], float2* T, int lane) {
  float2 z[32];
  static_for<0, 32>([&](auto I) { z[decltype(I)::value] = make_float2(se[decltype(I)::value],
                                                                     so[decltype(I)::value]); });
  fft32<-1>(z);
  // packed real columns kx = 0 and kx = 32
  T[lane * T2 + 0] = make_float2(z[0].x + z[0].y, z[0].x - z[0].y);
  static_for<1, 32>([&](auto K) {
    constexpr int k = decltype(K)::value;
    float2 a = z[k], c = cconj(z[32 - k]);
    float2 se_k = cscale(cadd(a, c), 0.5f);
    float2 d = csub(a, c);
    float2 so_k = make_float2(0.5f * d.y, -0.5f * d.x);   // d / (2i)
    T[lane * T2 + k] = cadd(se_k, twmul<-1, 64, k>(so_k));
  });
}

// Column pass.  Output of lane (q,b): X[m] = S(2m+b, q) for q >= 1.  The
// lanes of q = 0 hold the packed column F = S0 + i S32 (S0, S32 the real
// columns kx = 0 and 32, each Hermitian in ky) and leave it in Taux[ky] for
// op2_unpack.
MFBD_HDI void op2_cols(const float2* T, float2* Taux, int lane, float2 (&X)[32]) {
  const int q = lane >> 1, b = lane & 1;
  const float sb = b ? -1.0f : 1.0f;
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    float2 lo = T[n * T2 + q], hi = T[(n + 32) * T2 + q];
    X[n] = make_float2(lo.x + sb * hi.x, lo.y + sb * hi.y);
  });
  if (b) {
    static_for<1, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 64, n>(X[n]);
    });
  }
  fft32<-1>(X);
  if (q == 0) {
    static_for<0, 32>([&](auto I) { Taux[2 * decltype(I)::value + b] = X[decltype(I)::value]; });
  }
}

// After a barrier, every lane unpacks one row, ky = lane:
//   S0(ky) = (F(ky) + conj F(-ky)) / 2,  S32(ky) = (F(ky) - conj F(-ky)) / (2i).
// Returns S(ky, 32) and leaves S(ky, 0) in T[ky] (the column pass has read T).
MFBD_HDI float2 op2_unpack(const float2* Taux, float2* T, int lane) {
  const float2 f = Taux[lane], c = cconj(Taux[(64 - lane) & 63]);
  const float2 d = csub(f, c);
  T[lane] = cscale(cadd(f, c), 0.5f);
  return make_float2(0.5f * d.y, -0.5f * d.x);
}

// After another barrier, the lanes of column 0 take X[m] = S(2m+b, 0).
MFBD_HDI void op2_collect(const float2* T, int lane, float2 (&X)[32]) {
  if ((lane >> 1) == 0) {
    static_for<0, 32>([&](auto I) { X[decltype(I)::value] = T[2 * decltype(I)::value + (lane & 1)]; });
  }
}

// ---------------------------------------------------------------------------
// Half-buffer form of ops 1 and 2 (the forward kernel).  The two transposes
// move the real parts, then the imaginary parts, through a float buffer of
// half the size, so that a CU's LDS holds the workgroups of all the waves
// its registers allow (12 instead of 9).  Same arithmetic as op1_cols /
// op1_rows / op2_rows / op2_cols; a barrier separates every put from the
// get that reads it, and every get from the next put.
// ---------------------------------------------------------------------------
constexpr int LDS_HALF = 64 * T2 + 64;   // floats (>= 32 * T1; its first 64 float2 serve op2_unpack)

// part P (0: real, 1: imaginary) of the op1 column output; y after fft32<+1>
template <int P>
MFBD_HDI void op1_cols_put(const float2 (&y)[32], float* Tf, int lane) {
  const int q = lane >> 1, b = lane & 1;
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    const float v = P ? y[m].y : y[m].x;
    Tf[q * T1 + 2 * m + b] = (m & 1) ? -v : v;
  });
}

MFBD_HDI void op1_rows_get0(const float* Tf, int lane, float2 (&pe)[32]) {
  static_for<0, 32>([&](auto Q) { pe[decltype(Q)::value].x = Tf[decltype(Q)::value * T1 + lane]; });
}

// imaginary parts, then as op1_rows: pe[m] = p(r, 2m), po[m] = p(r, 2m+1)
MFBD_HDI void op1_rows_get1(const float* Tf, int lane, float2 (&pe)[32], float2 (&po)[32]) {
  static_for<0, 32>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    pe[q].y = Tf[q * T1 + lane];
    po[q] = twu<+1, 64, 16 + q>(pe[q]);
  });
  fft32<+1>(pe);
  fft32s<+1, Ramp16>(po);
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    if constexpr (m & 1) {
      pe[m] = cneg(pe[m]);
      po[m] = cneg(po[m]);
    }
  });
}

// the values op2_rows writes for an image s, v[k] for k in [0,32) (v[0]
// packing columns 0 and 32), from HALF the image: se[n] = s(r, 2n) / 2,
// so[n] = s(r, 2n+1) / 2.  Then the even- and odd-sample spectra are a + c
// and (a - c) / i (a = z[k], c = conj z[32-k]), with no factor 1/2, and
// v[k] = (a + c) + W64^-k (a - c) / i takes the twiddle in factored form.
MFBD_HDI void op2_rows_values(const float (&se)[32], const float (&so)[32], float2 (&v)[32]) {
  float2 z[32];
  static_for<0, 32>([&](auto I) { z[decltype(I)::value] = make_float2(se[decltype(I)::value],
                                                                     so[decltype(I)::value]); });
  fft32<-1>(z);
  v[0] = make_float2(2.0f * (z[0].x + z[0].y), 2.0f * (z[0].x - z[0].y));
  static_for<1, 32>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const float2 a = z[k], c = cconj(z[32 - k]);
    const float2 e = twu<-1, 64, k>(make_float2(a.y - c.y, c.x - a.x));   // (a - c) / i, times u
    constexpr float f = twf<-1, 64, k>();
    v[k] = make_float2((a.x + c.x) + f * e.x, (a.y + c.y) + f * e.y);
  });
}

template <int P>
MFBD_HDI void op2_rows_put(const float2 (&v)[32], float* Tf, int lane) {
  static_for<0, 32>([&](auto K) {
    constexpr int k = decltype(K)::value;
    Tf[lane * T2 + k] = P ? v[k].y : v[k].x;
  });
}

template <int P>
MFBD_HDI void op2_cols_get(const float* Tf, int lane, float2 (&X)[32]) {
  const int q = lane >> 1;
  const float sb = (lane & 1) ? -1.0f : 1.0f;
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    const float v = Tf[n * T2 + q] + sb * Tf[(n + 32) * T2 + q];
    if (P) X[n].y = v; else X[n].x = v;
  });
}

// rest of op2_cols: odd-row twiddles, the column FFT, column 0 packed in Taux
MFBD_HDI void op2_cols_finish(float2 (&X)[32], float2* Taux, int lane) {
  const int q = lane >> 1, b = lane & 1;
  if (b) {
    static_for<1, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 64, n>(X[n]);
    });
  }
  fft32<-1>(X);
  if (q == 0) {
    static_for<0, 32>([&](auto I) { Taux[2 * decltype(I)::value + b] = X[decltype(I)::value]; });
  }
}

// ---------------------------------------------------------------------------
// Op 3: inverse 2-D DFT of a Hermitian half spectrum in spectral layout ->
// real image in row layout: g(r) = sum_{u in N x N} G(u) exp(+2 pi i u.r/64).
// ---------------------------------------------------------------------------
MFBD_HDI void op3_gather(float2 x32, float2* Taux, int lane) { Taux[lane] = x32; }

MFBD_HDI void op3_cols(float2 (&X)[32], const float2* Taux, float2* T, int lane) {
  const int q = lane >> 1, b = lane & 1;
  if (q == 0) {
    // pack column 0 with column 32: both inverse transforms are real
    static_for<0, 32>([&](auto I) {
      constexpr int m = decltype(I)::value;
      float2 g32 = Taux[2 * m + b];
      X[m] = make_float2(X[m].x - g32.y, X[m].y + g32.x);
    });
  }
  fft32<+1>(X);   // lane b: E (b=0) or O (b=1) of the even/odd split along ky
  if (b) {
    static_for<1, 32>([&](auto I) {
      constexpr int r = decltype(I)::value;
      X[r] = twmul<+1, 64, r>(X[r]);
    });
  }
  static_for<0, 32>([&](auto I) {
    constexpr int r = decltype(I)::value;
    T[r * T3 + lane] = X[r];     // lane = 2q + b
  });
}

// Output: ge[n] = g(r, 2n), go[n] = g(r, 2n+1) for r = lane.
MFBD_HDI void op3_rows(const float2* T, int lane, float (&ge)[32], float (&go)[32]) {
  const int rp = lane & 31;
  const float sg = (lane < 32) ? 1.0f : -1.0f;
  float2 Xr[32];
  static_for<0, 32>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    float2 e = T[rp * T3 + 2 * q], wo = T[rp * T3 + 2 * q + 1];
    Xr[q] = make_float2(e.x + sg * wo.x, e.y + sg * wo.y);
  });
  // Xr[0] = (X(r,0), X(r,32)), both real; Xr[k] = X(r,k) for k in [1,32)
  float2 Z[32];
  Z[0] = make_float2(Xr[0].x + Xr[0].y, Xr[0].x - Xr[0].y);
  static_for<1, 32>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const float2 a = Xr[k], c = cconj(Xr[32 - k]);
    const float2 s = cadd(a, c);
    const float2 t = twu<+1, 64, k>(csub(a, c));   // t f = W64^k (a - c)
    constexpr float f = twf<+1, 64, k>();
    Z[k] = make_float2(s.x - f * t.y, s.y + f * t.x);    // s + i W64^k (a - c)
  });
  fft32<+1>(Z);
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    ge[n] = Z[n].x;
    go[n] = Z[n].y;
  });
}

// ---------------------------------------------------------------------------
// Op 4: forward 2-D DFT of a complex image in row layout, evaluated only on
// the pupil band: G(v) = sum_r H(r) exp(-2 pi i v.r/64), v in [16,48)^2.
// Output of lane (q,b): GP[i] = G(vy = 16 + 2i + b, vx = 16 + q), i in [0,16).
// ---------------------------------------------------------------------------
MFBD_HDI void op4_rows(float2 (&he)[32], float2 (&ho)[32], float2* T, int lane) {
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    if constexpr (n & 1) {
      he[n] = cneg(he[n]);
      ho[n] = cneg(ho[n]);
    }
  });
  fft32<-1>(he);
  fft32<-1>(ho);
  static_for<0, 32>([&](auto V) {
    constexpr int v = decltype(V)::value;
    T[lane * T2 + v] = cadd(he[v], twmul<-1, 64, 16 + v>(ho[v]));
  });
}

MFBD_HDI void op4_cols(const float2* T, int lane, float2 (&GP)[16]) {
  const int q = lane >> 1, b = lane & 1;
  const float sb = b ? -1.0f : 1.0f;
  float2 X[32];
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    float2 lo = T[n * T2 + q], hi = T[(n + 32) * T2 + q];
    X[n] = make_float2(lo.x + sb * hi.x, lo.y + sb * hi.y);
  });
  if (b) {
    static_for<1, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 64, n>(X[n]);
    });
  }
  fft32<-1>(X);
  static_for<0, 16>([&](auto I) { GP[decltype(I)::value] = X[8 + decltype(I)::value]; });
}

// ---------------------------------------------------------------------------
// Op 1+4 fused for the adjoint: from the band-column transform of the pupil
// (left in LDS by op1_cols) and the real image g (row layout), form
//   H = kap2 * g * p  (p the complex PSF amplitude of op1_rows)
// and run the row pass of op4 on it, one parity half of the columns at a
// time, so that p never has to be held in full.  The (-1)^m factors of the
// op1 row output and of the op4 row input cancel.  Result, for row r = lane:
//   Gr[v'] = G_r(r, 16 + v'), v' in [0,32), to be written by op14_write
// after a barrier (it overwrites the buffer op1_cols filled).
// ---------------------------------------------------------------------------
template <int E>
MFBD_HDI void op14_half(const float2* T, int lane, const float (&g)[32], float kap2,
                        float2 (&A)[32]) {
  static_for<0, 32>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    float2 c = T[q * T1 + lane];
    A[q] = E ? twu<+1, 64, 16 + q>(c) : c;
  });
  if constexpr (E) fft32s<+1, Ramp16>(A);
  else fft32<+1>(A);
  static_for<0, 32>([&](auto M) {
    constexpr int m = decltype(M)::value;
    A[m] = cscale(A[m], kap2 * g[m]);
  });
  fft32<-1>(A);
}

MFBD_HDI void op14_rows(const float2* T, int lane, const float (&ge)[32], const float (&go)[32],
                        float kap2, float2 (&Gr)[32]) {
  op14_half<0>(T, lane, ge, kap2, Gr);
  float2 B[32];
  op14_half<1>(T, lane, go, kap2, B);
  static_for<0, 32>([&](auto V) {
    constexpr int v = decltype(V)::value;
    const float2 b = twu<-1, 64, 16 + v>(B[v]);
    constexpr float f = twf<-1, 64, 16 + v>();
    Gr[v] = make_float2(Gr[v].x + f * b.x, Gr[v].y + f * b.y);
  });
}

MFBD_HDI void op14_write(const float2 (&Gr)[32], float2* T, int lane) {
  static_for<0, 32>([&](auto V) {
    constexpr int v = decltype(V)::value;
    T[lane * T2 + v] = Gr[v];
  });
}

}  // namespace n64
}  // namespace mfbd
