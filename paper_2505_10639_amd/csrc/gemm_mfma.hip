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

// One block = W waves x RT row tiles (16 RT rows (p,j)) x all mode columns.
// Each wave sums the slice [w K/W, (w+1) K/W) of k = c*bp + px for all RT
// row tiles, so every basis chunk it loads serves RT x 16 rows (the basis
// reads through L2 are what bound this contraction).  Operands are loaded
// DEPTH chunks ahead.  The partial sums are added in wave order (wave 0,
// then 1, ..., W-1) in one LDS buffer.  The basis rows are zero-padded to
// MT*16 per basis, so no mode test is needed inside the loop; rows past R
// read row R-1 and are not written.  Schedules: W = 4 with RT = 4 and
// DEPTH = 2, or W = 8 with RT = 2 and DEPTH = 1.  CS is the number of
// channels summed per load when they share one basis (0: the run-time C),
// fixed at compile time where it can be so that the loads of a chunk issue
// together.
template <int MT, int RT, int W, int DEPTH, int CS>
__global__ __launch_bounds__(64 * W) void k_grad_mfma(int R, int J, int C, int zc, int M, int bp,
                                                      const float* __restrict__ Ztp,
                                                      const float* __restrict__ gphi,
                                                      float* __restrict__ grad) {
  __shared__ floatx4 red[RT * MT][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * 16 * RT;
  const size_t cstride = (size_t)J * bp;   // between the channels of one (p, j)
  const float* grow[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int r = min(r0 + q * 16 + i16, R - 1);
    grow[q] = gphi + ((size_t)(r / J) * C * J + r % J) * bp + 4 * g;
  }
  floatx4 acc[RT][MT];
#pragma unroll
  for (int q = 0; q < RT; ++q)
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[q][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int Kq = zc * bp / W;
  const int k_begin = wave * Kq, k_end = (wave + 1) * Kq;
  const float* zrow = Ztp + (size_t)i16 * bp + 4 * g;
  // operands of chunk kk: a[q] from gphi row q*16 + i16 (with one shared
  // basis, the sum over channels in channel order), b[t] from mode row
  // t*16 + i16
  auto load = [&](int kk, floatx4 (&a4)[RT], floatx4 (&b4)[MT]) {
    const int c = kk / bp, px = kk % bp;
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      if (CS == 1) {
        a4[q] = *reinterpret_cast<const floatx4*>(grow[q] + c * cstride + px);
      } else if (CS > 1) {
        a4[q] = *reinterpret_cast<const floatx4*>(grow[q] + px);
#pragma unroll
        for (int ch = 1; ch < CS; ++ch)
          a4[q] += *reinterpret_cast<const floatx4*>(grow[q] + ch * cstride + px);
      } else {
        a4[q] = *reinterpret_cast<const floatx4*>(grow[q] + px);
        for (int ch = 1; ch < C; ++ch)
          a4[q] += *reinterpret_cast<const floatx4*>(grow[q] + ch * cstride + px);
      }
    }
    const float* zb = zrow + (size_t)c * MT * 16 * bp + px;
#pragma unroll
    for (int t = 0; t < MT; ++t) b4[t] = *reinterpret_cast<const floatx4*>(zb + (size_t)t * 16 * bp);
  };
  auto compute = [&](const floatx4 (&a4)[RT], const floatx4 (&b4)[MT]) {
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[q][t] = mfma4(a4[q], b4[t], acc[q][t]);
  };
  if constexpr (DEPTH == 1) {
    floatx4 a_cur[RT], b_cur[MT];
    load(k_begin, a_cur, b_cur);
    for (int kk = k_begin; kk < k_end; kk += 16) {
      floatx4 a_nxt[RT], b_nxt[MT];
      if (kk + 16 < k_end) load(kk + 16, a_nxt, b_nxt);
      compute(a_cur, b_cur);
      if (kk + 16 < k_end) {
#pragma unroll
        for (int q = 0; q < RT; ++q) a_cur[q] = a_nxt[q];
#pragma unroll
        for (int t = 0; t < MT; ++t) b_cur[t] = b_nxt[t];
      }
    }
  } else {
    // two stages; the chunk count per wave, zc*bp/(16 W), is even for
    // bp in {1024, 2304, 4096} and W in {4, 8}
    floatx4 a0[RT], b0[MT], a1[RT], b1[MT];
    load(k_begin, a0, b0);
    load(k_begin + 16, a1, b1);
    for (int kk = k_begin; kk < k_end; kk += 32) {
      compute(a0, b0);
      if (kk + 32 < k_end) load(kk + 32, a0, b0);
      compute(a1, b1);
      if (kk + 48 < k_end) load(kk + 48, a1, b1);
    }
  }
  for (int w = 0; w < W; ++w) {
    if (wave == w) {
#pragma unroll
      for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (w == 0)
            red[q * MT + t][lane] = acc[q][t];
          else
            red[q * MT + t][lane] += acc[q][t];
        }
    }
    __syncthreads();
  }
  for (int qt = wave; qt < RT * MT; qt += W) {
    const int q = qt / MT, t = qt % MT;
    const floatx4 v = red[qt][lane];
    const int m = t * 16 + i16;
    if (m >= M) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + q * 16 + 4 * g + e;
      if (row < R) grad[(size_t)row * M + m] = 6.283185307179586f * v[e];
    }
  }
}

// phi^T per channel: D[px][col] = sum_m ZtT[c][px][m] alpha[col][m], col = p*J + j.
// Block = 4 waves, (basis, kCols columns, a quarter of the band pixels);
// with one shared basis the block writes every channel's phi from one
// product: the block's kCols coefficient rows (contiguous in alpha) are
// staged once in LDS with the mode index padded to Mp; each wave then walks
// tiles of 16 pixels x kCols columns, taking its B operands as float4 LDS
// reads.  32 columns per block (twice the blocks of 64) measured 7% faster.
constexpr int kCols = 32, kColTiles = kCols / 16;
__global__ __launch_bounds__(256) void k_phase_mfma(int R, int J, int C, int zc, int M, int Mp,
                                                    int bp,
                                                    const float* __restrict__ ZtT,
                                                    const float* __restrict__ theta,
                                                    const float* __restrict__ alpha,
                                                    float* __restrict__ phi) {
  extern __shared__ float al[];    // [kCols][Mp + 4]
  const int ldm = Mp + 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int c = blockIdx.x >> 2, quarter = blockIdx.x & 3;
  const int col0 = blockIdx.y * kCols;
  const int ncol = min(kCols, R - col0);
  const float* src = alpha + (size_t)col0 * M;
  for (int r = wave; r < kCols; r += 4)
    for (int m = lane; m < Mp; m += 64)
      al[r * ldm + m] = (r < ncol && m < M) ? src[(size_t)r * M + m] : 0.f;
  __syncthreads();
  const int ntile = bp / 256;        // 16-pixel tiles per wave in a quarter
  for (int tile = 0; tile < ntile; ++tile) {
    const int px0 = quarter * (bp / 4) + (tile * 4 + wave) * 16;
    floatx4 acc[kColTiles];
#pragma unroll
    for (int t = 0; t < kColTiles; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* arow = ZtT + ((size_t)c * bp + px0 + i16) * Mp;
    for (int kk = 0; kk < Mp; kk += 16) {
      const floatx4 a4 = *reinterpret_cast<const floatx4*>(arow + kk + 4 * g);
#pragma unroll
      for (int t = 0; t < kColTiles; ++t) {
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
      for (int t = 0; t < kColTiles; ++t) {
        const int col = col0 + t * 16 + i16;
        if (col >= R) continue;
        const int p = col / J, j = col % J;
        *reinterpret_cast<floatx4*>(phi + (((size_t)p * C + ch) * J + j) * bp + px0 + 4 * g) =
            acc[t] + th;
      }
    }
  }
}

template <int MT, int CS>
void launch_grad_cs(const Dims& d, int zc, const float* Ztp, const float* gphi, float* grad,
                    hipStream_t s) {
  const int R = d.P * d.J;
  if (d.grad_waves == 8)
    hipLaunchKernelGGL((k_grad_mfma<MT, 2, 8, 1, CS>), dim3((R + 31) / 32), dim3(512), 0, s, R,
                       d.J, d.C, zc, d.M, d.bandpix(), Ztp, gphi, grad);
  else
    hipLaunchKernelGGL((k_grad_mfma<MT, 4, 4, 2, CS>), dim3((R + 63) / 64), dim3(256), 0, s, R,
                       d.J, d.C, zc, d.M, d.bandpix(), Ztp, gphi, grad);
}

template <int MT>
void launch_grad_t(const Dims& d, const float* Ztp, const float* gphi, float* grad,
                   hipStream_t s) {
  const int zc = d.zc > 0 ? d.zc : d.C;
  if (zc == d.C)
    launch_grad_cs<MT, 1>(d, zc, Ztp, gphi, grad, s);
  else if (d.C == 2)
    launch_grad_cs<MT, 2>(d, zc, Ztp, gphi, grad, s);
  else
    launch_grad_cs<MT, 0>(d, zc, Ztp, gphi, grad, s);
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
  dim3 grid(zc * 4, (R + kCols - 1) / kCols);
  const size_t lds = (size_t)kCols * (Mp + 4) * sizeof(float);
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
