// Host emulation of the 64x64, 96x96 and 128x128 unit operators -- test
// infrastructure.
//
// Runs the per-lane phases of ops64.h lane by lane on the CPU with an
// ordinary array standing in for LDS, so that the index logic of the GPU
// transforms can be checked without a GPU.  The GPU library never loads
// this file's library.
#include <cmath>
#include <cstring>

#include "bf16split.h"
#include "ops128.h"
#include "ops64.h"
#include "ops96.h"

using namespace mfbd;
using namespace mfbd::n64;

namespace {

struct Wave {
  float2 T[LDS_MAIN];
  float2 Taux[LDS_AUX];
};

// half spectrum [64][33] <-> spectral layout
void load_sl(const float* half, float2 (&X)[64][32], float2 (&x32)[64]) {
  const float2* h = reinterpret_cast<const float2*>(half);
  for (int l = 0; l < 64; ++l) {
    for (int m = 0; m < 32; ++m) X[l][m] = h[sl_index(l, m)];
    x32[l] = h[sl_index32(l)];
  }
}

void store_sl(float* half, const float2 (&X)[64][32], const float2 (&x32)[64]) {
  float2* h = reinterpret_cast<float2*>(half);
  for (int l = 0; l < 64; ++l) {
    for (int m = 0; m < 32; ++m) h[sl_index(l, m)] = X[l][m];
    h[sl_index32(l)] = x32[l];
  }
}

void r2c(Wave& w, const float* img, float2 (&X)[64][32], float2 (&x32)[64]) {
  for (int l = 0; l < 64; ++l) {
    float se[32], so[32];
    for (int n = 0; n < 32; ++n) {
      se[n] = img[l * 64 + 2 * n];
      so[n] = img[l * 64 + 2 * n + 1];
    }
    op2_rows(se, so, w.T, l);
  }
  for (int l = 0; l < 64; ++l) op2_cols(w.T, w.Taux, l, X[l]);
  for (int l = 0; l < 64; ++l) x32[l] = op2_unpack(w.Taux, w.T, l);
  for (int l = 0; l < 64; ++l) op2_collect(w.T, l, X[l]);
}

// the same transform through the half-size buffer (the forward kernel's form)
void r2c_half(Wave& w, const float* img, float2 (&X)[64][32], float2 (&x32)[64]) {
  static float2 v[64][32];
  float* Tf = reinterpret_cast<float*>(w.T);
  for (int l = 0; l < 64; ++l) {
    float se[32], so[32];   // half the image (op2_rows_values' input)
    for (int n = 0; n < 32; ++n) {
      se[n] = 0.5f * img[l * 64 + 2 * n];
      so[n] = 0.5f * img[l * 64 + 2 * n + 1];
    }
    op2_rows_values(se, so, v[l]);
  }
  for (int l = 0; l < 64; ++l) op2_rows_put<0>(v[l], Tf, l);
  for (int l = 0; l < 64; ++l) op2_cols_get<0>(Tf, l, X[l]);
  for (int l = 0; l < 64; ++l) op2_rows_put<1>(v[l], Tf, l);
  for (int l = 0; l < 64; ++l) op2_cols_get<1>(Tf, l, X[l]);
  for (int l = 0; l < 64; ++l) op2_cols_finish(X[l], w.Taux, l);
  for (int l = 0; l < 64; ++l) x32[l] = op2_unpack(w.Taux, w.T, l);
  for (int l = 0; l < 64; ++l) op2_collect(w.T, l, X[l]);
}

void c2r(Wave& w, float2 (&X)[64][32], const float2 (&x32)[64], float* img) {
  for (int l = 0; l < 64; ++l) op3_gather(x32[l], w.Taux, l);
  for (int l = 0; l < 64; ++l) op3_cols(X[l], w.Taux, w.T, l);
  for (int l = 0; l < 64; ++l) {
    float ge[32], go[32];
    op3_rows(w.T, l, ge, go);
    for (int n = 0; n < 32; ++n) {
      img[l * 64 + 2 * n] = ge[n];
      img[l * 64 + 2 * n + 1] = go[n];
    }
  }
}

// pupil band (A, phase in turns) -> complex amplitude p, row layout
void pupil_to_p(Wave& w, const float* A, const float* ph, float2 (&pe)[64][32],
                float2 (&po)[64][32], float2 (&Pk)[64][16]) {
  for (int l = 0; l < 64; ++l) {
    const int q = l >> 1, b = l & 1;
    float2 P[32], y[32];
    for (int n = 0; n < 32; ++n) {
      const double ang = 2.0 * M_PI * (double)ph[n * 32 + q];
      const float a = A[n * 32 + q];
      P[n] = make_float2(a * (float)std::cos(ang), a * (float)std::sin(ang));
    }
    static_for<0, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      y[n] = b ? twmul<+1, 64, 16 + n>(P[n]) : P[n];
    });
    for (int i = 0; i < 16; ++i) Pk[l][i] = P[2 * i + b];
    op1_cols(y, w.T, l);
  }
  for (int l = 0; l < 64; ++l) op1_rows(w.T, l, pe[l], po[l]);
}

// the same through the half-size buffer (the forward kernel's form)
void pupil_to_p_half(Wave& w, const float* A, const float* ph, float2 (&pe)[64][32],
                     float2 (&po)[64][32]) {
  static float2 y[64][32];
  float* Tf = reinterpret_cast<float*>(w.T);
  for (int l = 0; l < 64; ++l) {
    const int q = l >> 1, b = l & 1;
    for (int n = 0; n < 32; ++n) {
      const double ang = 2.0 * M_PI * ((double)ph[n * 32 + q] + (b ? (16 + n) / 64.0 : 0.0));
      const float a = A[n * 32 + q];
      y[l][n] = make_float2(a * (float)std::cos(ang), a * (float)std::sin(ang));
    }
    fft32<+1>(y[l]);
  }
  for (int l = 0; l < 64; ++l) op1_cols_put<0>(y[l], Tf, l);
  for (int l = 0; l < 64; ++l) op1_rows_get0(Tf, l, pe[l]);
  for (int l = 0; l < 64; ++l) op1_cols_put<1>(y[l], Tf, l);
  for (int l = 0; l < 64; ++l) op1_rows_get1(Tf, l, pe[l], po[l]);
}

}  // namespace

extern "C" {

// The exact three-way bf16 split of n values (bf16split.h): parts as FP32
// words, [n][3].
void emu_split3(const float* x, int n, float* parts) {
  for (int i = 0; i < n; ++i) {
    uint32_t h, m, l;
    mfbd::split3_words(x[i], h, m, l);
    parts[3 * i] = mfbd::u2f(h);
    parts[3 * i + 1] = mfbd::u2f(m);
    parts[3 * i + 2] = mfbd::u2f(l);
  }
}

// The packed form of eight values (one MFMA operand per part): [3][4] words.
void emu_split8(const float* x, uint32_t* words) {
  float v[8];
  for (int e = 0; e < 8; ++e) v[e] = x[e];
  const mfbd::Split8 s = mfbd::split8(v);
  for (int w = 0; w < 4; ++w) {
    words[w] = s.h[w];
    words[4 + w] = s.m[w];
    words[8 + w] = s.l[w];
  }
}

// fft32 in place on 32 interleaved complex values; dir = -1 or +1
void emu_fft32(float* x, int dir) {
  float2 v[32];
  std::memcpy(v, x, sizeof(v));
  if (dir < 0) fft32<-1>(v); else fft32<+1>(v);
  std::memcpy(x, v, sizeof(v));
}

void emu_fft64(float* x, int dir) {
  float2 v[64];
  std::memcpy(v, x, sizeof(v));
  if (dir < 0) fft64<-1>(v); else fft64<+1>(v);
  std::memcpy(x, v, sizeof(v));
}

// real 64x64 image -> half spectrum [64][33] complex
void emu_r2c(const float* img, float* half) {
  static Wave w;
  static float2 X[64][32], x32[64];
  r2c(w, img, X, x32);
  store_sl(half, X, x32);
}

// the same through the half-size buffer
void emu_r2c_half(const float* img, float* half) {
  static Wave w;
  static float2 X[64][32], x32[64];
  r2c_half(w, img, X, x32);
  store_sl(half, X, x32);
}

// band pupil -> complex amplitude p through the half-size buffer
void emu_pupil_ifft_half(const float* A, const float* ph, float* p) {
  static Wave w;
  static float2 pe[64][32], po[64][32];
  pupil_to_p_half(w, A, ph, pe, po);
  float2* o = reinterpret_cast<float2*>(p);
  for (int l = 0; l < 64; ++l)
    for (int n = 0; n < 32; ++n) {
      o[l * 64 + 2 * n] = pe[l][n];
      o[l * 64 + 2 * n + 1] = po[l][n];
    }
}

// Hermitian half spectrum [64][33] -> real image (unnormalised inverse)
void emu_c2r(const float* half, float* img) {
  static Wave w;
  static float2 X[64][32], x32[64];
  load_sl(half, X, x32);
  c2r(w, X, x32, img);
}

// band pupil -> complex amplitude p [64][64] (interleaved complex)
void emu_pupil_ifft(const float* A, const float* ph, float* p) {
  static Wave w;
  static float2 pe[64][32], po[64][32], Pk[64][16];
  pupil_to_p(w, A, ph, pe, po, Pk);
  float2* o = reinterpret_cast<float2*>(p);
  for (int l = 0; l < 64; ++l)
    for (int n = 0; n < 32; ++n) {
      o[l * 64 + 2 * n] = pe[l][n];
      o[l * 64 + 2 * n + 1] = po[l][n];
    }
}

// complex image [64][64] -> forward DFT sampled on the band [32][32]
void emu_fft_to_band(const float* h, float* band) {
  static Wave w;
  const float2* H = reinterpret_cast<const float2*>(h);
  for (int l = 0; l < 64; ++l) {
    float2 he[32], ho[32];
    for (int n = 0; n < 32; ++n) {
      he[n] = H[l * 64 + 2 * n];
      ho[n] = H[l * 64 + 2 * n + 1];
    }
    op4_rows(he, ho, w.T, l);
  }
  float2* o = reinterpret_cast<float2*>(band);
  for (int l = 0; l < 64; ++l) {
    float2 GP[16];
    op4_cols(w.T, l, GP);
    const int q = l >> 1, b = l & 1;
    for (int i = 0; i < 16; ++i) o[(2 * i + b) * 32 + q] = GP[i];
  }
}

// Whole unit: forward PSF/OTF, then the adjoint for a given G half spectrum.
void emu_unit(const float* A, const float* ph, float kappa, const float* G_half, float* psf,
              float* S_half, float* gphi) {
  static Wave w;
  static float2 pe[64][32], po[64][32], Pk[64][16], X[64][32], x32[64];
  static float img[64 * 64], g[64 * 64];
  pupil_to_p(w, A, ph, pe, po, Pk);
  for (int l = 0; l < 64; ++l)
    for (int n = 0; n < 32; ++n) {
      img[l * 64 + 2 * n] = kappa * cabs2(pe[l][n]);
      img[l * 64 + 2 * n + 1] = kappa * cabs2(po[l][n]);
    }
  std::memcpy(psf, img, sizeof(img));
  r2c(w, img, X, x32);
  store_sl(S_half, X, x32);
  load_sl(G_half, X, x32);
  c2r(w, X, x32, g);
  for (int l = 0; l < 64; ++l) {
    float2 he[32], ho[32];
    for (int n = 0; n < 32; ++n) {
      he[n] = cscale(pe[l][n], 2.0f * kappa * g[l * 64 + 2 * n]);
      ho[n] = cscale(po[l][n], 2.0f * kappa * g[l * 64 + 2 * n + 1]);
    }
    op4_rows(he, ho, w.T, l);
  }
  for (int l = 0; l < 64; ++l) {
    float2 GP[16];
    op4_cols(w.T, l, GP);
    const int q = l >> 1, b = l & 1;
    for (int i = 0; i < 16; ++i) {
      const float2 pk = Pk[l][i], gp = GP[i];
      gphi[(2 * i + b) * 32 + q] = pk.x * gp.y - pk.y * gp.x;
    }
  }
}

// Same as emu_unit's adjoint half, through the fused op14 path.
void emu_unit_fused(const float* A, const float* ph, float kappa, const float* G_half,
                    float* gphi) {
  static Wave w;
  static float2 pe[64][32], po[64][32], Pk[64][16], X[64][32], x32[64], Gr[64][32];
  static float g[64 * 64];
  load_sl(G_half, X, x32);
  c2r(w, X, x32, g);
  pupil_to_p(w, A, ph, pe, po, Pk);   // leaves op1_cols output in w.T
  // pupil_to_p ran op1_rows as well, which only reads T: redo op1_cols so T holds it
  for (int l = 0; l < 64; ++l) {
    const int q = l >> 1, b = l & 1;
    float2 P[32], y[32];
    for (int n = 0; n < 32; ++n) {
      const double ang = 2.0 * M_PI * (double)ph[n * 32 + q];
      const float a = A[n * 32 + q];
      P[n] = make_float2(a * (float)std::cos(ang), a * (float)std::sin(ang));
    }
    static_for<0, 32>([&](auto I) {
      constexpr int n = decltype(I)::value;
      y[n] = b ? twmul<+1, 64, 16 + n>(P[n]) : P[n];
    });
    op1_cols(y, w.T, l);
  }
  for (int l = 0; l < 64; ++l) {
    float ge[32], go[32];
    for (int n = 0; n < 32; ++n) {
      ge[n] = g[l * 64 + 2 * n];
      go[n] = g[l * 64 + 2 * n + 1];
    }
    op14_rows(w.T, l, ge, go, 2.0f * kappa, Gr[l]);
  }
  for (int l = 0; l < 64; ++l) op14_write(Gr[l], w.T, l);
  for (int l = 0; l < 64; ++l) {
    float2 GP[16];
    op4_cols(w.T, l, GP);
    const int q = l >> 1, b = l & 1;
    for (int i = 0; i < 16; ++i) {
      const float2 pk = Pk[l][i], gp = GP[i];
      gphi[(2 * i + b) * 32 + q] = pk.x * gp.y - pk.y * gp.x;
    }
  }
}

// ------------------------------------------------------------- N = 128
namespace e128 {
using namespace mfbd::n128;
struct WG {
  float2 T[n128::LDS_MAIN];
  float2 Taux[n128::LDS_AUX];
};
constexpr int L = 256;

// band pupil [64][64] (A, turns) -> p in row-parity layout; Pk = P at the band
// rows of the column-pair lanes' parity (for dL/dphi)
void pupil_to_p(WG& w, const float* A, const float* ph, float2 (&p)[L][64]) {
  for (int l = 0; l < L; ++l) {
    const int q = l >> 2, r = l & 3;
    float2 z[32];
    for (int n = 0; n < 32; ++n) {
      float2 acc = make_float2(0.f, 0.f);
      for (int h = 0; h < 2; ++h) {
        const int nn = n + 32 * h;
        const double ang = 2.0 * M_PI * ((double)ph[nn * 64 + q] + (32.0 + nn) * r / 128.0);
        const float a = A[nn * 64 + q];
        acc = cadd(acc, make_float2(a * (float)std::cos(ang), a * (float)std::sin(ang)));
      }
      z[n] = acc;
    }
    n128::op1_cols(z, w.T, l);
  }
  for (int l = 0; l < L; ++l) n128::op1_rows(w.T, l, p[l]);
}

// (the row values are formed from half the image, as in the kernels)
void r2c(WG& w, const float (&s)[L][64], float2 (&X)[L][32], float2 (&x64)[128]) {
  static float keep[L][32], send[L][32], other[L][32], hs[L][64];
  for (int l = 0; l < L; ++l)
    for (int m = 0; m < 64; ++m) hs[l][m] = 0.5f * s[l][m];
  for (int l = 0; l < L; ++l) n128::op2_rows_fold(hs[l], keep[l], send[l], l);
  float* Xf = reinterpret_cast<float*>(w.T);
  for (int l = 0; l < L; ++l) n128::xput(send[l], Xf, l);
  for (int l = 0; l < L; ++l) n128::xget(Xf, l, other[l]);
  for (int l = 0; l < L; ++l) n128::op2_rows_finish(keep[l], other[l], w.T, l);
  for (int l = 0; l < L; ++l) n128::op2_cols(w.T, w.Taux, l, X[l]);
  for (int l = 0; l < 128; ++l) x64[l] = n128::op2_unpack(w.Taux, w.T, l);
  for (int l = 0; l < L; ++l) n128::op2_collect(w.T, l, X[l]);
}

// the forward kernel's form: both transposes through the half-size buffer
struct WGH {
  float Th[n128::LDS_HALF];
  float2 Taux[n128::LDS_AUX];
};

void pupil_to_p_half(WGH& w, const float* A, const float* ph, float2 (&p)[L][64]) {
  static float2 z[L][32];
  for (int l = 0; l < L; ++l) {
    const int q = l >> 2, r = l & 3;
    for (int n = 0; n < 32; ++n) {
      float2 acc = make_float2(0.f, 0.f);
      for (int h = 0; h < 2; ++h) {
        const int nn = n + 32 * h;
        const double ang = 2.0 * M_PI * ((double)ph[nn * 64 + q] + (32.0 + nn) * r / 128.0);
        const float a = A[nn * 64 + q];
        acc = cadd(acc, make_float2(a * (float)std::cos(ang), a * (float)std::sin(ang)));
      }
      z[l][n] = acc;
    }
    fft32<+1>(z[l]);
  }
  for (int l = 0; l < L; ++l) n128::op1_cols_put<0>(z[l], w.Th, l);
  for (int l = 0; l < L; ++l) n128::op1_rows_get<0>(w.Th, l, p[l]);
  for (int l = 0; l < L; ++l) n128::op1_cols_put<1>(z[l], w.Th, l);
  for (int l = 0; l < L; ++l) n128::op1_rows_get<1>(w.Th, l, p[l]);
  for (int l = 0; l < L; ++l) n128::op1_rows_fft(p[l], l);
}

void r2c_half(WGH& w, const float (&s)[L][64], float2 (&X)[L][32], float2 (&x64)[128]) {
  static float keep[L][32], send[L][32], other[L][32], ax[L][32], bx[L][32], hs[L][64];
  static float2 v[L][32];
  for (int l = 0; l < L; ++l)
    for (int m = 0; m < 64; ++m) hs[l][m] = 0.5f * s[l][m];
  for (int l = 0; l < L; ++l) n128::op2_rows_fold(hs[l], keep[l], send[l], l);
  for (int l = 0; l < L; ++l) n128::xput(send[l], w.Th, l);
  for (int l = 0; l < L; ++l) n128::xget(w.Th, l, other[l]);
  for (int l = 0; l < L; ++l) n128::op2_rows_values(keep[l], other[l], l, v[l]);
  for (int l = 0; l < L; ++l) n128::op2_rows_put<0>(v[l], w.Th, l);
  for (int l = 0; l < L; ++l) n128::op2_cols_half_x(w.Th, l, ax[l], bx[l]);
  for (int l = 0; l < L; ++l) n128::op2_rows_put<1>(v[l], w.Th, l);
  for (int l = 0; l < L; ++l) n128::op2_cols_half_y(w.Th, w.Taux, l, ax[l], bx[l], X[l]);
  float2* T2 = reinterpret_cast<float2*>(w.Th);
  for (int l = 0; l < 128; ++l) x64[l] = n128::op2_unpack(w.Taux, T2, l);
  for (int l = 0; l < L; ++l) n128::op2_collect(T2, l, X[l]);
}

void c2r(WG& w, float2 (&X)[L][32], const float2 (&x64)[128], float (&g)[L][64]) {
  static float keep[L][32], send[L][32], other[L][32];
  for (int l = 0; l < 128; ++l) w.Taux[l] = x64[l];
  for (int l = 0; l < L; ++l) n128::op3_cols(X[l], w.Taux, w.T, l);
  for (int l = 0; l < L; ++l) n128::op3_cols_combine(w.T, l, X[l]);
  for (int l = 0; l < L; ++l) n128::op3_cols_put(X[l], w.T, l);
  for (int l = 0; l < L; ++l) n128::op3_rows_compute(w.T, l, keep[l], send[l]);
  float* Xf = reinterpret_cast<float*>(w.T);
  for (int l = 0; l < L; ++l) n128::xput(send[l], Xf, l);
  for (int l = 0; l < L; ++l) n128::xget(Xf, l, other[l]);
  for (int l = 0; l < L; ++l) n128::op3_rows_finish(keep[l], other[l], l, g[l]);
}

void to_band(WG& w, float2 (&H)[L][64], float2 (&GP)[L][16]) {
  static float2 keep[L][32], other[L][32];
  for (int l = 0; l < L; ++l) n128::op4_rows_fft(H[l], keep[l], w.T, l);
  for (int l = 0; l < L; ++l) n128::xget(w.T, l, other[l]);
  for (int l = 0; l < L; ++l) n128::op4_rows_finish(keep[l], other[l], w.T, l);
  for (int l = 0; l < L; ++l) n128::op4_cols(w.T, l, GP[l]);
}
}  // namespace e128

void emu128_pupil_ifft(const float* A, const float* ph, float* p) {
  static e128::WG w;
  static float2 pp[256][64];
  e128::pupil_to_p(w, A, ph, pp);
  float2* o = reinterpret_cast<float2*>(p);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 64; ++m) o[(l >> 1) * 128 + 2 * m + (l & 1)] = pp[l][m];
}

void emu128_pupil_ifft_half(const float* A, const float* ph, float* p) {
  static e128::WGH w;
  static float2 pp[256][64];
  e128::pupil_to_p_half(w, A, ph, pp);
  float2* o = reinterpret_cast<float2*>(p);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 64; ++m) o[(l >> 1) * 128 + 2 * m + (l & 1)] = pp[l][m];
}

void emu128_r2c_half(const float* img, float* half) {
  static e128::WGH w;
  static float s[256][64];
  static float2 X[256][32], x64[128];
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 64; ++m) s[l][m] = img[(l >> 1) * 128 + 2 * m + (l & 1)];
  e128::r2c_half(w, s, X, x64);
  float2* h = reinterpret_cast<float2*>(half);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 32; ++m) h[n128::sl_index(l, m)] = X[l][m];
  for (int l = 0; l < 128; ++l) h[n128::sl_index64(l)] = x64[l];
}

void emu128_r2c(const float* img, float* half) {
  static e128::WG w;
  static float s[256][64];
  static float2 X[256][32], x64[128];
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 64; ++m) s[l][m] = img[(l >> 1) * 128 + 2 * m + (l & 1)];
  e128::r2c(w, s, X, x64);
  float2* h = reinterpret_cast<float2*>(half);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 32; ++m) h[n128::sl_index(l, m)] = X[l][m];
  for (int l = 0; l < 128; ++l) h[n128::sl_index64(l)] = x64[l];
}

void emu128_c2r(const float* half, float* img) {
  static e128::WG w;
  static float g[256][64];
  static float2 X[256][32], x64[128];
  const float2* h = reinterpret_cast<const float2*>(half);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 32; ++m) X[l][m] = h[n128::sl_index(l, m)];
  for (int l = 0; l < 128; ++l) x64[l] = h[n128::sl_index64(l)];
  e128::c2r(w, X, x64, g);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 64; ++m) img[(l >> 1) * 128 + 2 * m + (l & 1)] = g[l][m];
}

void emu128_fft_to_band(const float* hc, float* band) {
  static e128::WG w;
  static float2 H[256][64], GP[256][16];
  const float2* h = reinterpret_cast<const float2*>(hc);
  for (int l = 0; l < 256; ++l)
    for (int m = 0; m < 64; ++m) H[l][m] = h[(l >> 1) * 128 + 2 * m + (l & 1)];
  e128::to_band(w, H, GP);
  float2* o = reinterpret_cast<float2*>(band);
  for (int l = 0; l < 256; ++l)
    for (int i = 0; i < 16; ++i) o[(4 * i + (l >> 6)) * 64 + (l & 63)] = GP[l][i];
}

}  // extern "C"

// ------------------------------------------------------------- N = 96
namespace e96 {
using namespace mfbd::n96;
struct WG {
  float2 T[n96::LDS_MAIN];
  float2 Taux[n96::LDS_AUX];
};
constexpr int L = n96::LANES;

void pupil_cols(WG& w, const float* A, const float* ph, float2 (&Pk)[L][24]) {
  for (int l = 0; l < L; ++l) {
    const int q = l >> 1, b = l & 1;
    float2 P[48], y[48];
    for (int n = 0; n < 48; ++n) {
      const double ang = 2.0 * M_PI * (double)ph[n * 48 + q];
      const float a = A[n * 48 + q];
      P[n] = make_float2(a * (float)std::cos(ang), a * (float)std::sin(ang));
    }
    static_for<0, 48>([&](auto I) {
      constexpr int n = decltype(I)::value;
      y[n] = b ? twmul<+1, 96, 24 + n>(P[n]) : P[n];
    });
    for (int i = 0; i < 24; ++i) Pk[l][i] = P[2 * i + b];
    n96::op1_cols(y, w.T, l);
  }
}

void r2c(WG& w, const float* img, float2 (&X)[L][48], float2 (&x48)[L]) {
  for (int l = 0; l < L; ++l) {
    float se[48], so[48];
    for (int n = 0; n < 48; ++n) {
      se[n] = img[l * 96 + 2 * n];
      so[n] = img[l * 96 + 2 * n + 1];
    }
    n96::op2_rows(se, so, w.T, l);
  }
  for (int l = 0; l < L; ++l) n96::op2_cols(w.T, w.Taux, l, X[l]);
  for (int l = 0; l < L; ++l) x48[l] = n96::op2_unpack(w.Taux, w.T, l);
  for (int l = 0; l < L; ++l) n96::op2_collect(w.T, l, X[l]);
}

void c2r(WG& w, float2 (&X)[L][48], const float2 (&x48)[L], float* img) {
  for (int l = 0; l < L; ++l) n96::op3_gather(x48[l], w.Taux, l);
  for (int l = 0; l < L; ++l) n96::op3_cols(X[l], w.Taux, w.T, l);
  for (int l = 0; l < L; ++l) {
    float ge[48], go[48];
    n96::op3_rows(w.T, l, ge, go);
    for (int n = 0; n < 48; ++n) {
      img[l * 96 + 2 * n] = ge[n];
      img[l * 96 + 2 * n + 1] = go[n];
    }
  }
}
}  // namespace e96

extern "C" {

void emu96_fft48(float* x, int dir) {
  float2 v[48];
  std::memcpy(v, x, sizeof(v));
  if (dir < 0) n96::fft48<-1>(v); else n96::fft48<+1>(v);
  std::memcpy(x, v, sizeof(v));
}

// band pupil [48][48] -> complex amplitude p [96][96]
void emu96_pupil_ifft(const float* A, const float* ph, float* p) {
  static e96::WG w;
  static float2 Pk[e96::L][24];
  e96::pupil_cols(w, A, ph, Pk);
  float2* o = reinterpret_cast<float2*>(p);
  for (int l = 0; l < e96::L; ++l) {
    float2 pe[48], po[48];
    n96::op1_rows(w.T, l, pe, po);
    for (int n = 0; n < 48; ++n) {
      o[l * 96 + 2 * n] = pe[n];
      o[l * 96 + 2 * n + 1] = po[n];
    }
  }
}

void emu96_r2c(const float* img, float* half) {
  static e96::WG w;
  static float2 X[e96::L][48], x48[e96::L];
  e96::r2c(w, img, X, x48);
  float2* h = reinterpret_cast<float2*>(half);
  for (int l = 0; l < e96::L; ++l) {
    for (int m = 0; m < 48; ++m) h[n96::sl_index(l, m)] = X[l][m];
    h[n96::sl_index48(l)] = x48[l];
  }
}

void emu96_c2r(const float* half, float* img) {
  static e96::WG w;
  static float2 X[e96::L][48], x48[e96::L];
  const float2* h = reinterpret_cast<const float2*>(half);
  for (int l = 0; l < e96::L; ++l) {
    for (int m = 0; m < 48; ++m) X[l][m] = h[n96::sl_index(l, m)];
    x48[l] = h[n96::sl_index48(l)];
  }
  e96::c2r(w, X, x48, img);
}

// Whole unit through the kernels' sequence: PSF, OTF, and the fused adjoint
// (op14) for a given G half spectrum.
void emu96_unit(const float* A, const float* ph, float kappa, const float* G_half, float* psf,
                float* S_half, float* gphi) {
  static e96::WG w;
  static float2 Pk[e96::L][24], X[e96::L][48], x48[e96::L], Gr[e96::L][48];
  static float img[96 * 96], g[96 * 96];
  e96::pupil_cols(w, A, ph, Pk);
  for (int l = 0; l < e96::L; ++l) {
    float2 pe[48], po[48];
    n96::op1_rows(w.T, l, pe, po);
    for (int n = 0; n < 48; ++n) {
      img[l * 96 + 2 * n] = kappa * cabs2(pe[n]);
      img[l * 96 + 2 * n + 1] = kappa * cabs2(po[n]);
    }
  }
  std::memcpy(psf, img, sizeof(img));
  e96::r2c(w, img, X, x48);
  float2* sh = reinterpret_cast<float2*>(S_half);
  for (int l = 0; l < e96::L; ++l) {
    for (int m = 0; m < 48; ++m) sh[n96::sl_index(l, m)] = X[l][m];
    sh[n96::sl_index48(l)] = x48[l];
  }
  const float2* gh = reinterpret_cast<const float2*>(G_half);
  for (int l = 0; l < e96::L; ++l) {
    for (int m = 0; m < 48; ++m) X[l][m] = gh[n96::sl_index(l, m)];
    x48[l] = gh[n96::sl_index48(l)];
  }
  e96::c2r(w, X, x48, g);
  e96::pupil_cols(w, A, ph, Pk);
  for (int l = 0; l < e96::L; ++l) {
    float ge[48], go[48];
    for (int n = 0; n < 48; ++n) {
      ge[n] = g[l * 96 + 2 * n];
      go[n] = g[l * 96 + 2 * n + 1];
    }
    n96::op14_rows(w.T, l, ge, go, 2.0f * kappa, Gr[l]);
  }
  for (int l = 0; l < e96::L; ++l) n96::op14_write(Gr[l], w.T, l);
  for (int l = 0; l < e96::L; ++l) {
    float2 GP[24];
    n96::op4_cols(w.T, l, GP);
    const int q = l >> 1, b = l & 1;
    for (int i = 0; i < 24; ++i) {
      const float2 pk = Pk[l][i], gp = GP[i];
      gphi[(2 * i + b) * 48 + q] = pk.x * gp.y - pk.y * gp.x;
    }
  }
}

}  // extern "C"
