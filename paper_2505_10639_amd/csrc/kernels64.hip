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

namespace mfbd {
using namespace n64;

namespace {

constexpr int kUnitF2 = N * HC;   // float2 elements per half spectrum (2112)

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// Pupil field on the band for lane (q,b): P[n] = A exp(2 pi i t), t in turns.
// y[n] = P[n] * W64^{+b (16+n)}, the input of op1_cols.
__device__ __forceinline__ void build_pupil(const float* __restrict__ A, const float* __restrict__ ph,
                                            int lane, float2 (&P)[32], float2 (&y)[32]) {
  const int q = lane >> 1, b = lane & 1;
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    float a = A[n * kBand + q];
    float t = ph[n * kBand + q];
    float s, c;
    sincospif(2.0f * t, &s, &c);
    P[n] = make_float2(a * c, a * s);
  }
  static_for<0, 32>([&](auto I) {
    constexpr int n = decltype(I)::value;
    y[n] = b ? twmul<+1, 64, 16 + n>(P[n]) : P[n];
  });
}

template <bool WANT_PSF>
__global__ __launch_bounds__(64) void k_forward64(int units, ChanTab ct, int C, int J,
                                                  const float* __restrict__ Ab,
                                                  const float* __restrict__ phi,
                                                  float* __restrict__ psf,
                                                  float2* __restrict__ S) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int u = blockIdx.x;
  if (u >= units) return;
  const int lane = threadIdx.x;
  const int c = (u / J) % C;
  float2 P[32], y[32];
  build_pupil(Ab + c * kBandPix, phi + (size_t)u * kBandPix, lane, P, y);
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

// One block per patch; loops over objects and the half-spectrum frequencies.
__global__ __launch_bounds__(256) void k_object64(int P, int C, int J, int K, ChanTab ct,
                                                  LossArgs la, const float2* __restrict__ S,
                                                  float2* __restrict__ O,
                                                  double* __restrict__ loss) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    const int c0 = ct.obj_first[k], c1 = ct.obj_first[k + 1];
    for (int f = tid; f < kUnitF2; f += 256) {
      const int kx = f % HC;
      const float h = (kx == 0 || kx == HC - 1) ? 1.0f : 2.0f;
      const float g = la.gamma ? la.gamma[(size_t)k * kUnitF2 + f] : la.gamma_scalar;
      float nr = 0.f, ni = 0.f, qq = g;
      for (int ci = c0; ci < c1; ++ci) {
        const int c = ct.obj_chans[ci];
        for (int j = 0; j < J; ++j) {
          const size_t idx = ((size_t)(p * C + c) * J + j) * kUnitF2 + f;
          const float w = la.weights ? la.weights[c * J + j] : 1.0f;
          const float2 d = la.D[idx], s = S[idx];
          nr += w * (d.x * s.x + d.y * s.y);
          ni += w * (d.y * s.x - d.x * s.y);
          qq += w * (s.x * s.x + s.y * s.y);
        }
      }
      const float2 o = make_float2(nr / qq, ni / qq);
      O[((size_t)p * K + k) * kUnitF2 + f] = o;
      double part = (double)(g * cabs2(o));
      for (int ci = c0; ci < c1; ++ci) {
        const int c = ct.obj_chans[ci];
        for (int j = 0; j < J; ++j) {
          const size_t idx = ((size_t)(p * C + c) * J + j) * kUnitF2 + f;
          const float w = la.weights ? la.weights[c * J + j] : 1.0f;
          const float2 d = la.D[idx], s = S[idx];
          const float2 r = csub(d, cmul(o, s));
          part += (double)(w * cabs2(r));
        }
      }
      acc += (double)h * part;
    }
  }
  red[tid] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) loss[p] = red[0];
}

__global__ __launch_bounds__(64) void k_adjoint64(int units, ChanTab ct, int C, int J, int K,
                                                  LossArgs la, const float* __restrict__ Ab,
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

  // recompute the complex PSF amplitude p
  float2 Pp[32], y[32];
  build_pupil(Ab + c * kBandPix, phi + (size_t)u * kBandPix, lane, Pp, y);
  const int b = lane & 1, q = lane >> 1;
  float2 Pk[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) Pk[i] = b ? Pp[2 * i + 1] : Pp[2 * i];
  op1_cols(y, T, lane);
  wave_sync();
  float2 pe[32], po[32];
  op1_rows(T, lane, pe, po);
  wave_sync();
  const float k2 = 2.0f * ct.kappa[c];
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    pe[n] = cscale(pe[n], k2 * ge[n]);
    po[n] = cscale(po[n], k2 * go[n]);
  }
  op4_rows(pe, po, T, lane);
  wave_sync();
  float2 GP[16];
  op4_cols(T, lane, GP);
  float* gout = gphi + (size_t)u * kBandPix;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float2 pk = Pk[i], gp = GP[i];
    gout[(2 * i + b) * kBand + q] = pk.x * gp.y - pk.y * gp.x;   // Im(conj(P) G_P)
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

// ---------------------------------------------------------------------------
// Tiled FP32 GEMM on the vector ALUs: out[r][col] = sum_k A(r,k) B(k,col).
// 64 x 64 output tile per 256-thread block, 4 x 4 per thread, k chunks of 16.
// ---------------------------------------------------------------------------
template <class Prob>
__global__ __launch_bounds__(256) void k_gemm(Prob pb) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < pb.Kdim; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e / 64, xx = e % 64;
      As[kk][xx] = pb.a(r0 + xx, k0 + kk);
      Bs[kk][xx] = pb.b(k0 + kk, c0 + xx);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][tr + 16 * i];
#pragma unroll
      for (int i = 0; i < 4; ++i) bv[i] = Bs[kk][tc + 16 * i];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] += av[i] * bv[jj];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) pb.store(r0 + tr + 16 * i, c0 + tc + 16 * jj, acc[i][jj]);
}

// phi[p][c][j][px] = theta[c][px] + sum_m alpha[p][j][m] Z[c][m][px]
// rows r = p*J + j, columns col = c*1024 + px, k = m
struct PhaseProb {
  int Rows, Cols, Kdim, J, C, M;
  const float* alpha;
  const float* Z;
  const float* theta;
  float* phi;
  __device__ float a(int r, int k) const {
    return (r < Rows && k < M) ? alpha[(size_t)r * M + k] : 0.f;
  }
  __device__ float b(int k, int col) const {
    if (k >= M || col >= Cols) return 0.f;
    const int c = col / kBandPix, px = col % kBandPix;
    return Z[((size_t)c * M + k) * kBandPix + px];
  }
  __device__ void store(int r, int col, float v) const {
    if (r >= Rows || col >= Cols) return;
    const int p = r / J, j = r % J, c = col / kBandPix, px = col % kBandPix;
    phi[(((size_t)p * C + c) * J + j) * kBandPix + px] = v + theta[c * kBandPix + px];
  }
};

// grad[p][j][m] = 2 pi sum_c sum_px Z[c][m][px] gphi[p][c][j][px]
// rows r = p*J + j, columns m, k = c*1024 + px
struct GradProb {
  int Rows, Cols, Kdim, J, C, M;
  const float* Z;
  const float* gphi;
  float* grad;
  __device__ float a(int r, int k) const {
    if (r >= Rows || k >= Kdim) return 0.f;
    const int p = r / J, j = r % J, c = k / kBandPix, px = k % kBandPix;
    return gphi[(((size_t)p * C + c) * J + j) * kBandPix + px];
  }
  __device__ float b(int k, int col) const {
    if (k >= Kdim || col >= Cols) return 0.f;
    const int c = k / kBandPix, px = k % kBandPix;
    return Z[((size_t)c * M + col) * kBandPix + px];
  }
  __device__ void store(int r, int col, float v) const {
    if (r >= Rows || col >= Cols) return;
    grad[(size_t)r * M + col] = 6.283185307179586f * v;
  }
};

}  // namespace

hipError_t launch_phase(const Dims& d, const float* alpha, const float* Zt, const float* thetat,
                        float* phi, hipStream_t s) {
  PhaseProb pb{d.P * d.J, d.C * kBandPix, d.M, d.J, d.C, d.M, alpha, Zt, thetat, phi};
  dim3 grid((pb.Cols + 63) / 64, (pb.Rows + 63) / 64);
  hipLaunchKernelGGL(k_gemm<PhaseProb>, grid, dim3(256), 0, s, pb);
  return hipGetLastError();
}

hipError_t launch_grad(const Dims& d, const float* Zt, const float* gphi, float* grad,
                       hipStream_t s) {
  GradProb pb{d.P * d.J, d.M, d.C * kBandPix, d.J, d.C, d.M, Zt, gphi, grad};
  dim3 grid((pb.Cols + 63) / 64, (pb.Rows + 63) / 64);
  hipLaunchKernelGGL(k_gemm<GradProb>, grid, dim3(256), 0, s, pb);
  return hipGetLastError();
}

hipError_t launch_forward64(const Dims& d, const ChanTab& ct, const float* Ab, const float* phi,
                            float* psf, float2* S, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  if (psf)
    hipLaunchKernelGGL(k_forward64<true>, dim3(units), dim3(64), 0, s, units, ct, d.C, d.J, Ab,
                       phi, psf, S);
  else
    hipLaunchKernelGGL(k_forward64<false>, dim3(units), dim3(64), 0, s, units, ct, d.C, d.J, Ab,
                       phi, psf, S);
  return hipGetLastError();
}

hipError_t launch_object64(const Dims& d, const ChanTab& ct, const LossArgs& la, const float2* S,
                           float2* O, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_object64, dim3(d.P), dim3(256), 0, s, d.P, d.C, d.J, d.K, ct, la, S, O,
                     loss);
  return hipGetLastError();
}

hipError_t launch_adjoint64(const Dims& d, const ChanTab& ct, const LossArgs& la, const float* Ab,
                            const float* phi, const float2* S, const float2* O, float* gphi,
                            hipStream_t s) {
  const int units = d.P * d.C * d.J;
  hipLaunchKernelGGL(k_adjoint64, dim3(units), dim3(64), 0, s, units, ct, d.C, d.J, d.K, la, Ab,
                     phi, S, O, gphi);
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
