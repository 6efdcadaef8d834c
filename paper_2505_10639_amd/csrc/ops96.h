// Workgroup-level 2-D transforms of one 96x96 MOMFBD unit: the 64x64 scheme
// with 96 active lanes of a two-wave workgroup and 48-point in-lane FFTs
// (radix 3 x 16).
//
// Data layouts (lane l < 96, q = l >> 1, b = l & 1):
//   band-column layout  lane (q,b) holds the pupil band column vx = 24 + q,
//                       rows vy = 24 + n, n in [0,48);
//   row layout          lane l holds image row r = l, columns in two
//                       48-element halves: even columns (2n), odd (2n+1);
//   spectral layout SL  lane (q,b) holds X(ky = 2m + b, kx = q), m in [0,48)
//                       (kx = 0 for q = 0), plus X(ky = l, kx = 48).
//
// The pupil support lies in the central band [24,72) of both axes, so each
// 96-point line transform with a band-limited input or a band-limited output
// folds into 48-point DFTs; lane pairs split the two output parities of a
// column.  One transpose through LDS per 2-D transform.  Phases are per-lane
// functions separated by workgroup barriers, so that a host harness can run
// them lane by lane.
#pragma once

#include "fft_lane.h"

namespace mfbd {
namespace n96 {

constexpr int N = 96;
constexpr int H = 48;        // half size = band width
constexpr int HC = 49;       // N/2 + 1 columns of a half spectrum
constexpr int BAND0 = 24;    // first row/column of the pupil band
constexpr int LANES = 96;    // active lanes of the 128-thread workgroup

constexpr int T1 = N + 2;    // [q][ky]     band-column IFFT -> rows
constexpr int T2 = HC;       // [r][q]      rows -> columns
constexpr int T3 = N + 1;    // [r'][2q+b]  columns -> rows (c2r)
constexpr int LDS_MAIN = N * T2 + 48;   // float2 elements (>= H*T1, H*T3)
constexpr int LDS_AUX = N;

MFBD_HDI int sl_index(int lane, int m) { return (2 * m + (lane & 1)) * HC + (lane >> 1); }
MFBD_HDI int sl_index48(int lane) { return lane * HC + 48; }

// ---------------------------------------------------------------- FFTs
// 3-point DFT of (a0, s1 a1, s2 a2) for real constants s1, s2 (factors of
// twiddles applied to a1, a2 as twu), every add an FMA:
//   X0 = a0 + s1 p, X1,2 = a0 - (s1/2) p +- DIR i h s1 m,
// with p = a1 + (s2/s1) a2, m = a1 - (s2/s1) a2.
template <int DIR>
MFBD_HDI void dft3s(float2& a0, float2& a1, float2& a2, float s1, float s2) {
  constexpr float h = 0.86602540378443864676f;   // sqrt(3)/2
  const float r = s2 / s1, hs = 0.5f * s1, d = DIR * h * s1;
  const float2 p = make_float2(a1.x + r * a2.x, a1.y + r * a2.y);
  const float2 m = make_float2(a1.x - r * a2.x, a1.y - r * a2.y);
  const float2 t = make_float2(a0.x - hs * p.x, a0.y - hs * p.y);
  a0 = make_float2(a0.x + s1 * p.x, a0.y + s1 * p.y);
  a1 = make_float2(t.x - d * m.y, t.y + d * m.x);
  a2 = make_float2(t.x + d * m.y, t.y - d * m.x);
}

// 16-point DFT in natural order, 4 x 4 (n = 4 a + b, k = c + 4 d), the
// twiddles W16^{bc} in factored form in the second-stage 4-point DFTs.
template <int DIR>
MFBD_HDI void fft16(float2 (&x)[16]) {
  static_for<0, 4>([&](auto B) {
    constexpr int b = decltype(B)::value;
    dft4<DIR>(x[b], x[4 + b], x[8 + b], x[12 + b]);
  });
  float2 y[16];
  static_for<0, 4>([&](auto Cc) {
    constexpr int c = decltype(Cc)::value;
    float2 a0 = x[4 * c], a1 = twu<DIR, 16, c>(x[4 * c + 1]), a2 = twu<DIR, 16, 2 * c>(x[4 * c + 2]),
           a3 = twu<DIR, 16, 3 * c>(x[4 * c + 3]);
    dft4s<DIR>(a0, a1, a2, a3, twf<DIR, 16, c>(), twf<DIR, 16, 2 * c>(), twf<DIR, 16, 3 * c>());
    y[c] = a0;
    y[c + 4] = a1;
    y[c + 8] = a2;
    y[c + 12] = a3;
  });
  static_for<0, 16>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

// 48-point DFT in natural order, 16 x 3:
//   n = 3 n1 + n2, k = k1 + 16 k2;
//   X[k1 + 16 k2] = sum_n2 W48^{n2 k1} W3^{n2 k2} sum_n1 x[3 n1 + n2] W16^{n1 k1},
// the twiddles W48^{n2 k1} in factored form in the 3-point DFTs.
template <int DIR>
MFBD_HDI void fft48(float2 (&x)[48]) {
  static_for<0, 3>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    float2 t[16];
    static_for<0, 16>([&](auto I) { t[decltype(I)::value] = x[3 * decltype(I)::value + n2]; });
    fft16<DIR>(t);
    static_for<0, 16>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      x[3 * k1 + n2] = twu<DIR, 48, n2 * k1>(t[k1]);
    });
  });
  float2 y[48];
  static_for<0, 16>([&](auto K1) {
    constexpr int k1 = decltype(K1)::value;
    float2 a0 = x[3 * k1], a1 = x[3 * k1 + 1], a2 = x[3 * k1 + 2];
    dft3s<DIR>(a0, a1, a2, twf<DIR, 48, k1>(), twf<DIR, 48, 2 * k1>());
    y[k1] = a0;
    y[k1 + 16] = a1;
    y[k1 + 32] = a2;
  });
  static_for<0, 48>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
}

// ---------------------------------------------------------------------------
// Op 1: inverse 2-D DFT of the band-limited pupil field -> PSF amplitude.
// Input of lane (q,b): y[n] = P(24+n, 24+q) * W96^{+b(24+n)}.
// ---------------------------------------------------------------------------
MFBD_HDI void op1_cols(float2 (&y)[48], float2* T, int lane) {
  const int q = lane >> 1, b = lane & 1;
  fft48<+1>(y);
  // column value at ky = 2m + b is (-1)^m y[m]
  static_for<0, 48>([&](auto M) {
    constexpr int m = decltype(M)::value;
    T[q * T1 + 2 * m + b] = (m & 1) ? cneg(y[m]) : y[m];
  });
}

// Output: pe[m] = p(r, 2m), po[m] = p(r, 2m+1) for row r = lane.
MFBD_HDI void op1_rows(const float2* T, int lane, float2 (&pe)[48], float2 (&po)[48]) {
  static_for<0, 48>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    const float2 c = T[q * T1 + lane];
    pe[q] = c;
    po[q] = twmul<+1, 96, 24 + q>(c);
  });
  fft48<+1>(pe);
  fft48<+1>(po);
  static_for<0, 48>([&](auto M) {
    constexpr int m = decltype(M)::value;
    if constexpr (m & 1) {
      pe[m] = cneg(pe[m]);
      po[m] = cneg(po[m]);
    }
  });
}

// ---------------------------------------------------------------------------
// Op 2: forward 2-D DFT of a real image in row layout -> half spectrum (SL).
// ---------------------------------------------------------------------------
MFBD_HDI void op2_rows(const float (&se)[48], const float (&so)[48], float2* T, int lane) {
  float2 z[48];
  static_for<0, 48>([&](auto I) {
    constexpr int i = decltype(I)::value;
    z[i] = make_float2(se[i], so[i]);
  });
  fft48<-1>(z);
  T[lane * T2 + 0] = make_float2(z[0].x + z[0].y, z[0].x - z[0].y);   // kx = 0 and 48, packed
  static_for<1, 48>([&](auto K) {
    constexpr int k = decltype(K)::value;
    // (a + c) / 2 + W96^-k (a - c) / (2i), the twiddle in factored form
    const float2 a = z[k], c = cconj(z[48 - k]);
    const float2 e = twu<-1, 96, k>(make_float2(a.y - c.y, c.x - a.x));
    constexpr float f = 0.5f * twf<-1, 96, k>();
    T[lane * T2 + k] = make_float2(0.5f * (a.x + c.x) + f * e.x, 0.5f * (a.y + c.y) + f * e.y);
  });
}

// Column pass.  Output of lane (q,b): X[m] = S(2m+b, q) for q >= 1; q = 0
// holds the packed real columns 0 and 48 (see op2_unpack).
MFBD_HDI void op2_cols(const float2* T, float2* Taux, int lane, float2 (&X)[48]) {
  const int q = lane >> 1, b = lane & 1;
  const float sb = b ? -1.0f : 1.0f;
  static_for<0, 48>([&](auto I) {
    constexpr int n = decltype(I)::value;
    const float2 lo = T[n * T2 + q], hi = T[(n + 48) * T2 + q];
    X[n] = make_float2(lo.x + sb * hi.x, lo.y + sb * hi.y);
  });
  if (b) {
    static_for<1, 48>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 96, n>(X[n]);
    });
  }
  fft48<-1>(X);
  // column 0 packs the real columns kx = 0 and 48 (F = S0 + i S48, both
  // Hermitian in ky): left in Taux[ky] for op2_unpack
  if (q == 0) {
    static_for<0, 48>([&](auto I) { Taux[2 * decltype(I)::value + b] = X[decltype(I)::value]; });
  }
}

// After a barrier, lane ky < 96 unpacks row ky: returns S(ky, 48) and leaves
// S(ky, 0) in T[ky] (the column pass has read T).
MFBD_HDI float2 op2_unpack(const float2* Taux, float2* T, int lane) {
  const float2 f = Taux[lane], c = cconj(Taux[(96 - lane) % 96]);
  const float2 d = csub(f, c);
  T[lane] = cscale(cadd(f, c), 0.5f);
  return make_float2(0.5f * d.y, -0.5f * d.x);
}

// After another barrier, the lanes of column 0 take X[m] = S(2m+b, 0).
MFBD_HDI void op2_collect(const float2* T, int lane, float2 (&X)[48]) {
  if ((lane >> 1) == 0) {
    static_for<0, 48>([&](auto I) { X[decltype(I)::value] = T[2 * decltype(I)::value + (lane & 1)]; });
  }
}

// ---------------------------------------------------------------------------
// Op 3: inverse 2-D DFT of a Hermitian half spectrum (SL) -> real image rows.
// ---------------------------------------------------------------------------
MFBD_HDI void op3_gather(float2 x48, float2* Taux, int lane) { Taux[lane] = x48; }

MFBD_HDI void op3_cols(float2 (&X)[48], const float2* Taux, float2* T, int lane) {
  const int q = lane >> 1, b = lane & 1;
  if (q == 0) {
    static_for<0, 48>([&](auto I) {
      constexpr int m = decltype(I)::value;
      const float2 g = Taux[2 * m + b];
      X[m] = make_float2(X[m].x - g.y, X[m].y + g.x);   // column 0 + i column 48
    });
  }
  fft48<+1>(X);
  if (b) {
    static_for<1, 48>([&](auto I) {
      constexpr int r = decltype(I)::value;
      X[r] = twmul<+1, 96, r>(X[r]);
    });
  }
  static_for<0, 48>([&](auto I) {
    constexpr int r = decltype(I)::value;
    T[r * T3 + lane] = X[r];
  });
}

// Output: ge[n] = g(r, 2n), go[n] = g(r, 2n+1) for r = lane.
MFBD_HDI void op3_rows(const float2* T, int lane, float (&ge)[48], float (&go)[48]) {
  const int rp = lane < 48 ? lane : lane - 48;
  const float sg = lane < 48 ? 1.0f : -1.0f;
  float2 Xr[48];
  static_for<0, 48>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    const float2 e = T[rp * T3 + 2 * q], wo = T[rp * T3 + 2 * q + 1];
    Xr[q] = make_float2(e.x + sg * wo.x, e.y + sg * wo.y);
  });
  float2 Z[48];
  Z[0] = make_float2(Xr[0].x + Xr[0].y, Xr[0].x - Xr[0].y);
  static_for<1, 48>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const float2 a = Xr[k], c = cconj(Xr[48 - k]);
    const float2 s = cadd(a, c);
    const float2 t = twu<+1, 96, k>(csub(a, c));   // t f = W96^k (a - c)
    constexpr float f = twf<+1, 96, k>();
    Z[k] = make_float2(s.x - f * t.y, s.y + f * t.x);   // s + i W96^k (a - c)
  });
  fft48<+1>(Z);
  static_for<0, 48>([&](auto I) {
    constexpr int n = decltype(I)::value;
    ge[n] = Z[n].x;
    go[n] = Z[n].y;
  });
}

// ---------------------------------------------------------------------------
// Op 4: forward 2-D DFT of a complex image (row layout) on the pupil band only.
// Output of lane (q,b): GP[i] = G(vy = 24 + 2i + b, vx = 24 + q), i in [0,24).
// ---------------------------------------------------------------------------
MFBD_HDI void op4_cols(const float2* T, int lane, float2 (&GP)[24]) {
  const int q = lane >> 1, b = lane & 1;
  const float sb = b ? -1.0f : 1.0f;
  float2 X[48];
  static_for<0, 48>([&](auto I) {
    constexpr int n = decltype(I)::value;
    const float2 lo = T[n * T2 + q], hi = T[(n + 48) * T2 + q];
    X[n] = make_float2(lo.x + sb * hi.x, lo.y + sb * hi.y);
  });
  if (b) {
    static_for<1, 48>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 96, n>(X[n]);
    });
  }
  fft48<-1>(X);
  static_for<0, 24>([&](auto I) { GP[decltype(I)::value] = X[12 + decltype(I)::value]; });
}

// ---------------------------------------------------------------------------
// Op 1+4 fused for the adjoint (as for 64x64): from op1_cols' band-column
// transform of the pupil in LDS and the real image g (row layout), form
// H = kap2 g p and its row transform to the band, one parity half of the
// columns at a time.  Gr[v'] = G_r(r, 24 + v'), v' in [0,48), r = lane.
// ---------------------------------------------------------------------------
template <int E>
MFBD_HDI void op14_half(const float2* T, int lane, const float (&g)[48], float kap2,
                        float2 (&A)[48]) {
  static_for<0, 48>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    const float2 c = T[q * T1 + lane];
    A[q] = E ? twmul<+1, 96, 24 + q>(c) : c;
  });
  fft48<+1>(A);
  static_for<0, 48>([&](auto M) {
    constexpr int m = decltype(M)::value;
    A[m] = cscale(A[m], kap2 * g[m]);
  });
  fft48<-1>(A);
}

MFBD_HDI void op14_rows(float2* T, int lane, const float (&ge)[48], const float (&go)[48],
                        float kap2, float2 (&Gr)[48]) {
  op14_half<0>(T, lane, ge, kap2, Gr);
  // Odd half.  The band-transform values this lane reads, T[q T1 + lane],
  // are read by no other lane: each is loaded (twiddled) into B and the
  // even-half result parked in its slot, so one 48-element array is live
  // at a time; the last radix-3 stage of B's forward transform adds each
  // output, twiddled, to the parked value (register pressure).
  float2 B[48];
  static_for<0, 48>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    const float2 c = T[q * T1 + lane];
    T[q * T1 + lane] = Gr[q];
    B[q] = twmul<+1, 96, 24 + q>(c);
  });
  fft48<+1>(B);
  static_for<0, 48>([&](auto M) {
    constexpr int m = decltype(M)::value;
    B[m] = cscale(B[m], kap2 * go[m]);
  });
  static_for<0, 3>([&](auto N2) {
    constexpr int n2 = decltype(N2)::value;
    float2 t[16];
    static_for<0, 16>([&](auto I) { t[decltype(I)::value] = B[3 * decltype(I)::value + n2]; });
    fft16<-1>(t);
    static_for<0, 16>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      B[3 * k1 + n2] = twu<-1, 48, n2 * k1>(t[k1]);
    });
  });
  // y + W96^-E x with the twiddle in factored form
  auto comb = [](auto E, float2 y, float2 x) {
    constexpr int e = decltype(E)::value;
    const float2 u = twu<-1, 96, e>(x);
    constexpr float f = twf<-1, 96, e>();
    return make_float2(y.x + f * u.x, y.y + f * u.y);
  };
  static_for<0, 16>([&](auto K1) {
    constexpr int k1 = decltype(K1)::value;
    float2 a0 = B[3 * k1], a1 = B[3 * k1 + 1], a2 = B[3 * k1 + 2];
    dft3s<-1>(a0, a1, a2, twf<-1, 48, k1>(), twf<-1, 48, 2 * k1>());   // outputs k1, k1 + 16, k1 + 32
    Gr[k1] = comb(std::integral_constant<int, 24 + k1>{}, T[k1 * T1 + lane], a0);
    Gr[k1 + 16] = comb(std::integral_constant<int, 40 + k1>{}, T[(k1 + 16) * T1 + lane], a1);
    Gr[k1 + 32] = comb(std::integral_constant<int, 56 + k1>{}, T[(k1 + 32) * T1 + lane], a2);
  });
}

MFBD_HDI void op14_write(const float2 (&Gr)[48], float2* T, int lane) {
  static_for<0, 48>([&](auto V) {
    constexpr int v = decltype(V)::value;
    T[lane * T2 + v] = Gr[v];
  });
}

}  // namespace n96
}  // namespace mfbd
