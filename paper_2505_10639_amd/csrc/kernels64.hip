// Unit kernels of the MOMFBD hot path for 64x64 patches (gfx950).
//
// One workgroup = one wavefront = one unit (patch p, channel c, frame j).
//   forward : phase -> pupil -> inverse 2-D DFT -> |.|^2 (unit-sum PSF)
//             -> forward 2-D DFT (OTF half spectrum)
//   object  : Wiener object O_k = N_k / Q_k and the residual-form loss of the
//             patch, accumulated in FP64
//   adjoint : G = -2 w conj(O)(D - O S) -> inverse DFT -> H = 2 kappa g p
//             -> forward DFT on the pupil band -> dL/dphi = Im(conj(P) G_P)
//   prepare : patch cut, mean removal, apodization, mean restore, 2-D DFT
//   objimg  : object spectrum -> real image / N^2
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ops64.h"

#ifndef MFBD_HW_SINCOS
#define MFBD_HW_SINCOS 1
#endif

namespace mfbd {
using namespace n64;

namespace {

constexpr int kUnitF2 = N * HC;   // float2 elements per half spectrum (2112)

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// exp(2 pi i t) for a phase t in turns.  The hardware sine/cosine take
// turns directly; the argument is first reduced to [0,1).
__device__ __forceinline__ float2 expi_turns(float t) {
#if MFBD_HW_SINCOS
  const float f = __builtin_amdgcn_fractf(t);
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
#else
  float s, c;
  sincospif(2.0f * t, &s, &c);
  return make_float2(c, s);
#endif
}

// Input of op1_cols for lane (q,b): y[n] = P(16+n, 16+q) W64^{+b(16+n)} with
// P = A exp(2 pi i t) on the band; the modulation is a phase ramp of
// b (16+n)/64 turns added before the exponential.
__device__ __forceinline__ void build_pupil(const float* __restrict__ A, const float* __restrict__ ph,
                                            int lane, float2 (&y)[32]) {
  const int q = lane >> 1, b = lane & 1;
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    const float a = A[n * kBand + q];
    const float t = ph[n * kBand + q] + (b ? (16 + n) * (1.0f / 64.0f) : 0.0f);
    y[n] = cscale(expi_turns(t), a);
  }
}

template <bool WANT_PSF>
__global__ __launch_bounds__(64) void k_forward64(int units, ChanTab ct, int C, int J,
                                                  const int* __restrict__ active,
                                                  const float* __restrict__ Ab,
                                                  const float* __restrict__ phi,
                                                  float* __restrict__ psf,
                                                  float2* __restrict__ S) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int u = blockIdx.x;
  if (u >= units) return;
  if (active && !active[u / (J * C)]) return;
  const int lane = threadIdx.x;
  const int c = (u / J) % C;
  float2 y[32];
  build_pupil(Ab + c * kBandPix, phi + (size_t)u * kBandPix, lane, y);
  op1_cols(y, T, lane);
  wave_sync();
  float2 pe[32], po[32];
  op1_rows(T, lane, pe, po);
  wave_sync();
  const float kap = ct.kappa[c];
  float se[32], so[32];
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    se[n] = kap * cabs2(pe[n]);
    so[n] = kap * cabs2(po[n]);
  }
  if (WANT_PSF) {
    float* row = psf + (size_t)u * N * N + lane * N;
#pragma unroll
    for (int n = 0; n < 32; ++n) {
      row[2 * n] = se[n];
      row[2 * n + 1] = so[n];
    }
  }
  op2_rows(se, so, T, lane);
  wave_sync();
  float2 X[32];
  op2_cols(T, Taux, lane, X);
  wave_sync();
  float2 x32 = op2_spread(Taux, lane);
  float2* out = S + (size_t)u * kUnitF2;
#pragma unroll
  for (int m = 0; m < 32; ++m) out[sl_index(lane, m)] = X[m];
  out[sl_index32(lane)] = x32;
}

// One block per patch; loops over objects and pairs of adjacent half-spectrum
// frequencies (16-byte loads).  One pass over D and S: N = sum w D conj(S),
// Q = gamma + sum w |S|^2 and E = sum w |D|^2 are accumulated in FP64, where
// the products of FP32 inputs are exact, so the loss term E - |N|^2/Q
// (Eq. loss_momfbd at the Wiener object, equal to the residual form) keeps
// full accuracy.  Units are read four at a time so that loads overlap.
struct Acc2 {
  double nr[2], ni[2], q[2], e[2];
};

__device__ __forceinline__ void acc_unit(Acc2& a, double w, float4 d, float4 s) {
  const double dx0 = d.x, dy0 = d.y, sx0 = s.x, sy0 = s.y;
  const double dx1 = d.z, dy1 = d.w, sx1 = s.z, sy1 = s.w;
  a.nr[0] += w * (dx0 * sx0 + dy0 * sy0);
  a.ni[0] += w * (dy0 * sx0 - dx0 * sy0);
  a.q[0] += w * (sx0 * sx0 + sy0 * sy0);
  a.e[0] += w * (dx0 * dx0 + dy0 * dy0);
  a.nr[1] += w * (dx1 * sx1 + dy1 * sy1);
  a.ni[1] += w * (dy1 * sx1 - dx1 * sy1);
  a.q[1] += w * (sx1 * sx1 + sy1 * sy1);
  a.e[1] += w * (dx1 * dx1 + dy1 * dy1);
}

__global__ __launch_bounds__(256) void k_object64(int P, int C, int J, int K, ChanTab ct,
                                                  LossArgs la, const int* __restrict__ active,
                                                  const float2* __restrict__ S,
                                                  float2* __restrict__ O,
                                                  double* __restrict__ loss) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  if (active && !active[p]) return;
  const int tid = threadIdx.x;
  double acc = 0.0;
  constexpr int kPairs = kUnitF2 / 2;
  for (int k = 0; k < K; ++k) {
    const int c0 = ct.obj_first[k], c1 = ct.obj_first[k + 1];
    for (int f2 = tid; f2 < kPairs; f2 += 256) {
      const int f = 2 * f2;
      Acc2 a;
      for (int i = 0; i < 2; ++i) {
        a.nr[i] = a.ni[i] = a.e[i] = 0.0;
        a.q[i] = la.gamma ? (double)la.gamma[(size_t)k * kUnitF2 + f + i] : (double)la.gamma_scalar;
      }
      for (int ci = c0; ci < c1; ++ci) {
        const int c = ct.obj_chans[ci];
        const float4* Dc = reinterpret_cast<const float4*>(la.D + ((size_t)(p * C + c) * J) * kUnitF2 + f);
        const float4* Sc = reinterpret_cast<const float4*>(S + ((size_t)(p * C + c) * J) * kUnitF2 + f);
        const float* wc = la.weights ? la.weights + c * J : nullptr;
        int j = 0;
        for (; j + 4 <= J; j += 4) {
          float4 d[4], s[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            d[u] = Dc[(size_t)(j + u) * (kUnitF2 / 2)];
            s[u] = Sc[(size_t)(j + u) * (kUnitF2 / 2)];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc_unit(a, wc ? (double)wc[j + u] : 1.0, d[u], s[u]);
        }
        for (; j < J; ++j)
          acc_unit(a, wc ? (double)wc[j] : 1.0, Dc[(size_t)j * (kUnitF2 / 2)],
                   Sc[(size_t)j * (kUnitF2 / 2)]);
      }
      float4 o;
      double part = 0.0;
      {
        const double inv0 = 1.0 / a.q[0], inv1 = 1.0 / a.q[1];
        o = make_float4((float)(a.nr[0] * inv0), (float)(a.ni[0] * inv0),
                        (float)(a.nr[1] * inv1), (float)(a.ni[1] * inv1));
        const int kx0 = f % HC, kx1 = (f + 1) % HC;
        const double h0 = (kx0 == 0 || kx0 == HC - 1) ? 1.0 : 2.0;
        const double h1 = (kx1 == 0 || kx1 == HC - 1) ? 1.0 : 2.0;
        part = h0 * (a.e[0] - (a.nr[0] * a.nr[0] + a.ni[0] * a.ni[0]) * inv0) +
               h1 * (a.e[1] - (a.nr[1] * a.nr[1] + a.ni[1] * a.ni[1]) * inv1);
      }
      reinterpret_cast<float4*>(O + ((size_t)p * K + k) * kUnitF2)[f2] = o;
      acc += part;
    }
  }
  red[tid] = acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (tid < s2) red[tid] += red[tid + s2];
    __syncthreads();
  }
  if (tid == 0) loss[p] = red[0];
}

__global__ __launch_bounds__(64) void k_adjoint64(int units, ChanTab ct, int C, int J, int K,
                                                  LossArgs la, const int* __restrict__ active,
                                                  const float* __restrict__ Ab,
                                                  const float* __restrict__ phi,
                                                  const float2* __restrict__ S,
                                                  const float2* __restrict__ O,
                                                  float* __restrict__ gphi) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int u = blockIdx.x;
  if (u >= units) return;
  const int lane = threadIdx.x;
  const int j = u % J;
  const int c = (u / J) % C;
  const int p = u / (J * C);
  if (active && !active[p]) return;
  const int k = ct.chan_obj[c];
  const float w2 = -2.0f * (la.weights ? la.weights[c * J + j] : 1.0f);
  const float2* Su = S + (size_t)u * kUnitF2;
  const float2* Du = la.D + (size_t)u * kUnitF2;
  const float2* Ok = O + ((size_t)p * K + k) * kUnitF2;

  // G = -2 w conj(O) (D - O S) in spectral layout
  float2 G[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) {
    const int idx = sl_index(lane, m);
    const float2 o = Ok[idx];
    const float2 r = csub(Du[idx], cmul(o, Su[idx]));
    G[m] = cscale(cmul(cconj(o), r), w2);
  }
  float2 g32;
  {
    const int idx = sl_index32(lane);
    const float2 o = Ok[idx];
    const float2 r = csub(Du[idx], cmul(o, Su[idx]));
    g32 = cscale(cmul(cconj(o), r), w2);
  }
  op3_gather(g32, Taux, lane);
  wave_sync();
  op3_cols(G, Taux, T, lane);
  wave_sync();
  float ge[32], go[32];
  op3_rows(T, lane, ge, go);
  wave_sync();

  // recompute the pupil band transform, then H = 2 kappa g p and its
  // forward transform to the band, half a row spectrum at a time
  const float* Ac = Ab + c * kBandPix;
  const float* phu = phi + (size_t)u * kBandPix;
  {
    float2 y[32];
    build_pupil(Ac, phu, lane, y);
    op1_cols(y, T, lane);
  }
  wave_sync();
  float2 Gr[32];
  op14_rows(T, lane, ge, go, 2.0f * ct.kappa[c], Gr);
  wave_sync();
  op14_write(Gr, T, lane);
  wave_sync();
  float2 GP[16];
  op4_cols(T, lane, GP);
  const int b = lane & 1, q = lane >> 1;
  float* gout = gphi + (size_t)u * kBandPix;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int n = 2 * i + b;
    const float2 pk = cscale(expi_turns(phu[n * kBand + q]), Ac[n * kBand + q]);
    const float2 gp = GP[i];
    gout[n * kBand + q] = pk.x * gp.y - pk.y * gp.x;   // Im(conj(P) G_P)
  }
}

__global__ __launch_bounds__(64) void k_prepare64(int units, int C, int J, int H, int W,
                                                  int stride, int nx,
                                                  const float* __restrict__ frames,
                                                  const float* __restrict__ apod,
                                                  float2* __restrict__ D) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int u = blockIdx.x;
  if (u >= units) return;
  const int lane = threadIdx.x;
  const int j = u % J;
  const int c = (u / J) % C;
  const int p = u / (J * C);
  const int y0 = (p / nx) * stride, x0 = (p % nx) * stride;
  float* Tf = reinterpret_cast<float*>(T);
  const float* src = frames + ((size_t)(c * J + j) * H + y0) * W + x0;
  for (int r = 0; r < N; ++r) Tf[r * 65 + lane] = src[(size_t)r * W + lane];
  wave_sync();
  float se[32], so[32];
  float sum = 0.f;
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    se[n] = Tf[lane * 65 + 2 * n];
    so[n] = Tf[lane * 65 + 2 * n + 1];
    sum += se[n] + so[n];
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  const float mean = sum * (1.0f / (N * N));
  const float* wr = apod + lane * N;
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    se[n] = wr[2 * n] * (se[n] - mean) + mean;
    so[n] = wr[2 * n + 1] * (so[n] - mean) + mean;
  }
  wave_sync();
  op2_rows(se, so, T, lane);
  wave_sync();
  float2 X[32];
  op2_cols(T, Taux, lane, X);
  wave_sync();
  float2 x32 = op2_spread(Taux, lane);
  float2* out = D + (size_t)u * kUnitF2;
#pragma unroll
  for (int m = 0; m < 32; ++m) out[sl_index(lane, m)] = X[m];
  out[sl_index32(lane)] = x32;
}

__global__ __launch_bounds__(64) void k_objimg64(int items, const float2* __restrict__ O,
                                                 float* __restrict__ obj) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int it = blockIdx.x;
  if (it >= items) return;
  const int lane = threadIdx.x;
  const float2* Oi = O + (size_t)it * kUnitF2;
  float2 X[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) X[m] = Oi[sl_index(lane, m)];
  op3_gather(Oi[sl_index32(lane)], Taux, lane);
  wave_sync();
  op3_cols(X, Taux, T, lane);
  wave_sync();
  float ge[32], go[32];
  op3_rows(T, lane, ge, go);
  float* row = obj + (size_t)it * N * N + lane * N;
  const float inv = 1.0f / (N * N);
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    row[2 * n] = ge[n] * inv;
    row[2 * n + 1] = go[n] * inv;
  }
}

}  // namespace

hipError_t launch_forward64(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                            const float* phi, float* psf, float2* S, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  if (psf)
    hipLaunchKernelGGL(k_forward64<true>, dim3(units), dim3(64), 0, s, units, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  else
    hipLaunchKernelGGL(k_forward64<false>, dim3(units), dim3(64), 0, s, units, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  return hipGetLastError();
}

hipError_t launch_object64(const Dims& d, const ChanTab& ct, const LossArgs& la, const int* active,
                           const float2* S, float2* O, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_object64, dim3(d.P), dim3(256), 0, s, d.P, d.C, d.J, d.K, ct, la, active,
                     S, O, loss);
  return hipGetLastError();
}

hipError_t launch_adjoint64(const Dims& d, const ChanTab& ct, const LossArgs& la,
                            const int* active, const float* Ab, const float* phi, const float2* S,
                            const float2* O, float* gphi, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  hipLaunchKernelGGL(k_adjoint64, dim3(units), dim3(64), 0, s, units, ct, d.C, d.J, d.K, la,
                     active, Ab, phi, S, O, gphi);
  return hipGetLastError();
}

hipError_t launch_prepare64(const Dims& d, const float* frames, int H, int W, int stride,
                            const float* apod, float2* D, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const int nx = (W - N) / stride + 1;
  hipLaunchKernelGGL(k_prepare64, dim3(units), dim3(64), 0, s, units, d.C, d.J, H, W, stride, nx,
                     frames, apod, D);
  return hipGetLastError();
}

hipError_t launch_objimg64(const Dims& d, const float2* O, float* obj, hipStream_t s) {
  const int items = d.P * d.K;
  hipLaunchKernelGGL(k_objimg64, dim3(items), dim3(64), 0, s, items, O, obj);
  return hipGetLastError();
}

}  // namespace mfbd
