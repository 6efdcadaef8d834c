// Wave-level 2-D transforms of one 128x128 MOMFBD unit (one workgroup of
// four wavefronts = 256 lanes).
//
// Layouts (lane l in [0,256)):
//   band-column  lane (q = l>>2, r = l&3): pupil band column vx = 32 + q, output
//                rows of residue r mod 4 (first pass of op1);
//   row-parity   lane (y = l>>1, e = l&1): image row y, columns 2m + e, m in [0,64);
//   column-pair  lane (q = l>>1, b = l&1), l < 128: spectral column q, rows of
//                parity b (the column passes of op2, op3, op4; lanes 128..255
//                idle there);
//   spectral SL  lanes l < 128: X(ky = 2m + b, kx = q), m in [0,64) (kx = 0 for
//                q = 0) plus X(ky = l, kx = 64).
//
// The pupil support lies in the central band [32,96) of both axes (diameter
// below N/2).  64- and 128-point sums fold into in-lane 32- and 64-point FFTs:
// band-limited inputs fold by output residue (the modulation of the folded
// sequence is a phase ramp the caller adds before the exponential), columns
// split by output parity over a lane pair, and the real row transforms pack
// even/odd samples into one complex sequence, with the halves exchanged
// between the two lanes of a row through LDS.  Every phase is a per-lane
// function; phases are separated by a workgroup barrier.
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
constexpr int U3 = 129;         // [r'][2q+b]   op3 columns -> rows
constexpr int LDS_MAIN = 128 * U2;     // 8448 float2 (>= 64*U1, 64*U3)
constexpr int LDS_AUX = 128;

MFBD_HDI int sl_index(int lane, int m) { return (2 * m + (lane & 1)) * HC + (lane >> 1); }
MFBD_HDI int sl_index64(int lane) { return lane * HC + 64; }

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

// Row pass: lane (y, e) -> p(y, 2m + e), m in [0,64).
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

MFBD_HDI void op2_rows_finish(const float (&keep)[32], const float (&other)[32], float2* T,
                              int lane) {
  const int y = lane >> 1, e = lane & 1;
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
  // Sr[k] = (Z[k] + conj Z[64-k])/2 + W128^{-k} (Z[k] - conj Z[64-k])/(2i), k = e mod 2
  if (e == 0) {
    T[y * U2 + 0] = make_float2(w[0].x + w[0].y, w[0].x - w[0].y);    // (Sr0, Sr64)
    static_for<1, 32>([&](auto K) {
      constexpr int kp = decltype(K)::value;      // k = 2 kp
      float2 a = w[kp], c = cconj(w[32 - kp]);
      float2 se = cscale(cadd(a, c), 0.5f);
      float2 d = csub(a, c);
      float2 so = make_float2(0.5f * d.y, -0.5f * d.x);
      T[y * U2 + 2 * kp] = cadd(se, twmul<-1, 128, 2 * kp>(so));
    });
  } else {
    static_for<0, 32>([&](auto K) {
      constexpr int kp = decltype(K)::value;      // k = 2 kp + 1, partner 63 - 2kp
      float2 a = w[kp], c = cconj(w[31 - kp]);
      float2 se = cscale(cadd(a, c), 0.5f);
      float2 d = csub(a, c);
      float2 so = make_float2(0.5f * d.y, -0.5f * d.x);
      T[y * U2 + 2 * kp + 1] = cadd(se, twmul<-1, 128, 2 * kp + 1>(so));
    });
  }
}

// Column pass (lanes < 128): X[m] = S(2m + b, q), m in [0,64); q = 0 unpacks
// the real columns 0 and 64 and leaves column 64 in Taux[ky].
MFBD_HDI void op2_cols(const float2* T, float2* Taux, int lane, float2 (&X)[64]) {
  const int q = lane >> 1, b = lane & 1;
  const float sb = b ? -1.0f : 1.0f;
  static_for<0, 64>([&](auto I) {
    constexpr int n = decltype(I)::value;
    float2 lo = T[n * U2 + q], hi = T[(n + 64) * U2 + q];
    X[n] = make_float2(lo.x + sb * hi.x, lo.y + sb * hi.y);
  });
  if (b) {
    static_for<1, 64>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 128, n>(X[n]);
    });
  }
  fft64<-1>(X);
  if (q == 0) {
    // F = S0 + i S64 with S0, S64 Hermitian in ky; -ky has the same parity,
    // element m pairs with (64 - m) mod 64 (b = 0) or 63 - m (b = 1).  Each
    // pair is unpacked in place.
    auto unpack = [&](auto MA, auto MB) {
      constexpr int ma = decltype(MA)::value, mb = decltype(MB)::value;
      const float2 fa = X[ma], fb = X[mb];
      const float2 ca = cconj(fb), cb = cconj(fa);
      const float2 da = csub(fa, ca), db = csub(fb, cb);
      X[ma] = cscale(cadd(fa, ca), 0.5f);
      Taux[2 * ma + b] = make_float2(0.5f * da.y, -0.5f * da.x);
      if constexpr (ma != mb) {
        X[mb] = cscale(cadd(fb, cb), 0.5f);
        Taux[2 * mb + b] = make_float2(0.5f * db.y, -0.5f * db.x);
      }
    };
    if (b == 0) {
      static_for<0, 33>([&](auto I) {
        constexpr int m = decltype(I)::value;
        unpack(std::integral_constant<int, m>{}, std::integral_constant<int, (64 - m) & 63>{});
      });
    } else {
      static_for<0, 32>([&](auto I) {
        constexpr int m = decltype(I)::value;
        unpack(std::integral_constant<int, m>{}, std::integral_constant<int, 63 - m>{});
      });
    }
  }
}

// ---------------------------------------------------------------------------
// Op 3: inverse DFT of a Hermitian half spectrum (SL, lanes < 128) -> real
// image in row-parity layout.
// ---------------------------------------------------------------------------
MFBD_HDI void op3_cols(float2 (&X)[64], const float2* Taux, float2* T, int lane) {
  const int q = lane >> 1, b = lane & 1;
  if (q == 0) {
    static_for<0, 64>([&](auto I) {
      constexpr int m = decltype(I)::value;
      float2 g64 = Taux[2 * m + b];
      X[m] = make_float2(X[m].x - g64.y, X[m].y + g64.x);
    });
  }
  fft64<+1>(X);
  if (b) {
    static_for<1, 64>([&](auto I) {
      constexpr int r = decltype(I)::value;
      X[r] = twmul<+1, 128, r>(X[r]);
    });
  }
  static_for<0, 64>([&](auto I) {
    constexpr int r = decltype(I)::value;
    T[r * U3 + lane] = X[r];
  });
}

// Row pass (all lanes): lane (y, f) forms the row half spectrum, then the
// parity-f half of the packed inverse, z[2n'+f], n' in [0,32).  It keeps the
// part of z that belongs to its own column parity and sends the other part.
MFBD_HDI void op3_rows_compute(const float2* T, int lane, float (&keep)[32], float (&send)[32]) {
  const int y = lane >> 1, f = lane & 1;
  const int rp = y & 63;
  const float sg = (y < 64) ? 1.0f : -1.0f;
  float2 Xr[64];
  static_for<0, 64>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    float2 ev = T[rp * U3 + 2 * q], wo = T[rp * U3 + 2 * q + 1];
    Xr[q] = make_float2(ev.x + sg * wo.x, ev.y + sg * wo.y);
  });
  // Z[k] = (X[k] + X[k+64]) + i W128^{+k} (X[k] - X[k+64]), X[k+64] = conj X[64-k]
  float2 Z[64];
  Z[0] = make_float2(Xr[0].x + Xr[0].y, Xr[0].x - Xr[0].y);
  static_for<1, 64>([&](auto K) {
    constexpr int k = decltype(K)::value;
    float2 a = Xr[k], c = cconj(Xr[64 - k]);
    float2 s = cadd(a, c);
    float2 t = twmul<+1, 128, k>(csub(a, c));
    Z[k] = make_float2(s.x - t.y, s.y + t.x);
  });
  // z[2n'+f] = sum_k' (Z[k'] + (-1)^f Z[k'+32]) W64^{k' f} W32^{k' n'}
  const float sf = f ? -1.0f : 1.0f;
  float2 w[32];
  static_for<0, 32>([&](auto I) {
    constexpr int k = decltype(I)::value;
    w[k] = make_float2(Z[k].x + sf * Z[k + 32].x, Z[k].y + sf * Z[k + 32].y);
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
// v' in [0,32), lane 1 v' in [32,64); each sends the other half it holds.
// ---------------------------------------------------------------------------
MFBD_HDI void op4_rows_fft(float2 (&H)[64], float2 (&keep)[32], float2 (&send)[32], int lane) {
  const int e = lane & 1;
  static_for<0, 64>([&](auto I) {
    constexpr int m = decltype(I)::value;
    if constexpr (m & 1) H[m] = cneg(H[m]);
  });
  fft64<-1>(H);
  static_for<0, 32>([&](auto I) {
    constexpr int v = decltype(I)::value;
    // lane 0 keeps F_0[v] (v < 32) and sends F_0[32+v]; lane 1 keeps F_1[32+v], sends F_1[v]
    keep[v] = e ? H[32 + v] : H[v];
    send[v] = e ? H[v] : H[32 + v];
  });
}

MFBD_HDI void op4_rows_finish(const float2 (&keep)[32], const float2 (&other)[32], float2* T,
                              int lane) {
  const int y = lane >> 1, e = lane & 1;
  if (e == 0) {
    static_for<0, 32>([&](auto I) {
      constexpr int v = decltype(I)::value;       // other = F_1[v]
      T[y * U2 + v] = cadd(keep[v], twmul<-1, 128, 32 + v>(other[v]));
    });
  } else {
    static_for<0, 32>([&](auto I) {
      constexpr int v = decltype(I)::value;       // other = F_0[32+v]
      T[y * U2 + 32 + v] = cadd(other[v], twmul<-1, 128, 64 + v>(keep[v]));
    });
  }
}

// Column pass (lanes < 128): GP[i] = G(vy = 32 + 2i + b, vx = 32 + q), i in [0,32).
MFBD_HDI void op4_cols(const float2* T, int lane, float2 (&GP)[32]) {
  const int q = lane >> 1, b = lane & 1;
  const float sb = b ? -1.0f : 1.0f;
  float2 X[64];
  static_for<0, 64>([&](auto I) {
    constexpr int n = decltype(I)::value;
    float2 lo = T[n * U2 + q], hi = T[(n + 64) * U2 + q];
    X[n] = make_float2(lo.x + sb * hi.x, lo.y + sb * hi.y);
  });
  if (b) {
    static_for<1, 64>([&](auto I) {
      constexpr int n = decltype(I)::value;
      X[n] = twmul<-1, 128, n>(X[n]);
    });
  }
  fft64<-1>(X);
  static_for<0, 32>([&](auto I) { GP[decltype(I)::value] = X[16 + decltype(I)::value]; });
}

}  // namespace n128
}  // namespace mfbd
