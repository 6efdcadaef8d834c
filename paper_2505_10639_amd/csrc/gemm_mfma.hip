// Dense modal contractions on the matrix cores (FP32 MFMA, gfx950).
//
//   phase : phi[p][c][j][px] = theta_c[px] + sum_m Z_c[m][px] alpha[p][j][m]
//           (Eq. wavefront on the 32x32 pupil band, in turns)
//   grad  : dL/dalpha[p][j][m] = 2 pi sum_c sum_px Z_c[m][px] gphi[p][c][j][px]
//
// When every channel has the same band basis (zc = 1) the phase product is
// formed once and written for each channel with its own theta_c, and the
// gradient contracts Z with sum_c gphi[p][c][j][px] (channels summed first,
// in channel order): half the matrix-core work at two channels.
//
// Both use v_mfma_f32_16x16x4f32.  Operand layout of that instruction: lane l
// supplies A[i = l%16][k = l/16] and B[k = l/16][j = l%16]; the 16x16 result
// sits in 4 registers per lane, D[4 (l/16) + e][l%16], e = 0..3.
// The k order is free, so lane group g = l/16 takes k = k0 + 4g + s at step s:
// every lane then loads its four operands of a 16-wide k chunk as one float4.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mfbd {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(const floatx4& a, const floatx4& b, floatx4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
  return acc;
}

// One block = W waves = 16 rows (p,j) x all mode columns; wave w sums the
// slice [w K/W, (w+1) K/W) of k = c*bp + px; the partial sums are added in
// fixed order (wave 0 + 1 + ... + W-1) through LDS.  W (4 or 8) is a launch
// schedule the autotuner picks.
template <int MT, int W>
__global__ __launch_bounds__(64 * W) void k_grad_mfma(int R, int J, int C, int zc, int M, int bp,
                                                      const float* __restrict__ Zt,
                                                      const float* __restrict__ gphi,
                                                      float* __restrict__ grad) {
  __shared__ floatx4 red[W - 1][MT][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * 16;
  const int r = r0 + i16;
  const bool rok = r < R;
  const int p = rok ? r / J : 0, j = rok ? r % J : 0;
  floatx4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int Kq = zc * bp / W;
  const int k_begin = wave * Kq, k_end = (wave + 1) * Kq;
  // operands of chunk kk: a from gphi row r, b[t] from mode rows t*16 + i16;
  // the next chunk's operands are loaded before the current chunk's MFMAs
  auto load = [&](int kk, floatx4& a4, floatx4 (&b4)[MT]) {
    const int c = kk / bp, px = kk % bp + 4 * g;
    a4 = floatx4{0.f, 0.f, 0.f, 0.f};
    if (rok) {
      if (zc == C) {
        a4 = *reinterpret_cast<const floatx4*>(gphi + (((size_t)p * C + c) * J + j) * bp + px);
      } else {
        for (int ch = 0; ch < C; ++ch)
          a4 += *reinterpret_cast<const floatx4*>(gphi + (((size_t)p * C + ch) * J + j) * bp + px);
      }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int m = t * 16 + i16;
      b4[t] = (m < M) ? *reinterpret_cast<const floatx4*>(Zt + ((size_t)c * M + m) * bp + px)
                      : floatx4{0.f, 0.f, 0.f, 0.f};
    }
  };
  floatx4 a_cur, b_cur[MT];
  load(k_begin, a_cur, b_cur);
  for (int kk = k_begin; kk < k_end; kk += 16) {
    floatx4 a_nxt, b_nxt[MT];
    if (kk + 16 < k_end) load(kk + 16, a_nxt, b_nxt);
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = mfma4(a_cur, b_cur[t], acc[t]);
    if (kk + 16 < k_end) {
      a_cur = a_nxt;
#pragma unroll
      for (int t = 0; t < MT; ++t) b_cur[t] = b_nxt[t];
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < MT; ++t) red[wave - 1][t][lane] = acc[t];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    floatx4 v = acc[t];
#pragma unroll
    for (int w = 0; w < W - 1; ++w) v += red[w][t][lane];
    const int m = t * 16 + i16;
    if (m >= M) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + 4 * g + e;
      if (row < R) grad[(size_t)row * M + m] = 6.283185307179586f * v[e];
    }
  }
}

// phi^T per channel: D[px][col] = sum_m ZtT[c][px][m] alpha[col][m], col = p*J + j.
// Block = 4 waves, (basis, 64 columns, a quarter of the band pixels); with
// one shared basis the block writes every channel's phi from one product:
// the block's 64 coefficient rows (contiguous in alpha) are staged once in
// LDS with the mode index padded to Mp; each wave then walks 4 tiles of 16
// pixels x 64 columns, taking its B operands as float4 LDS reads.
__global__ __launch_bounds__(256) void k_phase_mfma(int R, int J, int C, int zc, int M, int Mp,
                                                    int bp,
                                                    const float* __restrict__ ZtT,
                                                    const float* __restrict__ theta,
                                                    const float* __restrict__ alpha,
                                                    float* __restrict__ phi) {
  extern __shared__ float al[];    // [64][Mp + 4]
  const int ldm = Mp + 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int c = blockIdx.x >> 2, quarter = blockIdx.x & 3;
  const int col0 = blockIdx.y * 64;
  const int ncol = min(64, R - col0);
  const float* src = alpha + (size_t)col0 * M;
  for (int r = wave; r < 64; r += 4)
    for (int m = lane; m < Mp; m += 64)
      al[r * ldm + m] = (r < ncol && m < M) ? src[(size_t)r * M + m] : 0.f;
  __syncthreads();
  const int ntile = bp / 256;        // 16-pixel tiles per wave in a quarter
  for (int tile = 0; tile < ntile; ++tile) {
    const int px0 = quarter * (bp / 4) + (tile * 4 + wave) * 16;
    floatx4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* arow = ZtT + ((size_t)c * bp + px0 + i16) * Mp;
    for (int kk = 0; kk < Mp; kk += 16) {
      const floatx4 a4 = *reinterpret_cast<const floatx4*>(arow + kk + 4 * g);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const floatx4 b4 =
            *reinterpret_cast<const floatx4*>(al + (t * 16 + i16) * ldm + kk + 4 * g);
        acc[t] = mfma4(a4, b4, acc[t]);
      }
    }
    const int c_lo = zc == C ? c : 0, c_hi = zc == C ? c + 1 : C;
    for (int ch = c_lo; ch < c_hi; ++ch) {
      const floatx4 th =
          *reinterpret_cast<const floatx4*>(theta + (size_t)ch * bp + px0 + 4 * g);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = col0 + t * 16 + i16;
        if (col >= R) continue;
        const int p = col / J, j = col % J;
        *reinterpret_cast<floatx4*>(phi + (((size_t)p * C + ch) * J + j) * bp + px0 + 4 * g) =
            acc[t] + th;
      }
    }
  }
}

template <int MT>
void launch_grad_t(const Dims& d, const float* Zt, const float* gphi, float* grad,
                   hipStream_t s) {
  const int R = d.P * d.J, zc = d.zc > 0 ? d.zc : d.C;
  // eight waves only while the partial sums fit in 64 KB of LDS
  if (MT <= 8 && d.grad_waves == 8)
    hipLaunchKernelGGL((k_grad_mfma<MT, (MT <= 8 ? 8 : 4)>), dim3((R + 15) / 16), dim3(512), 0, s,
                       R, d.J, d.C, zc, d.M, d.bandpix(), Zt, gphi, grad);
  else
    hipLaunchKernelGGL((k_grad_mfma<MT, 4>), dim3((R + 15) / 16), dim3(256), 0, s, R, d.J, d.C,
                       zc, d.M, d.bandpix(), Zt, gphi, grad);
}

}  // namespace

hipError_t launch_grad(const Dims& d, const float* Zt, const float* gphi, float* grad,
                       hipStream_t s) {
  const int mt = (d.M + 15) / 16;
  switch (mt) {
#define MFBD_CASE(n) \
  case n: launch_grad_t<n>(d, Zt, gphi, grad, s); break;
    MFBD_CASE(1) MFBD_CASE(2) MFBD_CASE(3) MFBD_CASE(4) MFBD_CASE(5) MFBD_CASE(6)
    MFBD_CASE(7) MFBD_CASE(8) MFBD_CASE(9) MFBD_CASE(10) MFBD_CASE(11) MFBD_CASE(12)
    MFBD_CASE(13) MFBD_CASE(14) MFBD_CASE(15) MFBD_CASE(16)
#undef MFBD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_phase(const Dims& d, const float* alpha, const float* ZtT, int Mp,
                        const float* thetat, float* phi, hipStream_t s) {
  const int R = d.P * d.J, zc = d.zc > 0 ? d.zc : d.C;
  dim3 grid(zc * 4, (R + 63) / 64);
  const size_t lds = (size_t)64 * (Mp + 4) * sizeof(float);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_phase_mfma),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_phase_mfma, grid, dim3(256), lds, s, R, d.J, d.C, zc, d.M, Mp, d.bandpix(),
                     ZtT, thetat, alpha, phi);
  return hipGetLastError();
}

}  // namespace mfbd
