// Bodies of the dense modal contractions on the matrix cores (FP32 MFMA,
// gfx950), shared by the kernels of one plan (gemm_mfma.hip) and of a group
// of fields (gemm_group.hip).
//
//   phase : phi[p][c][j][px] = theta_c[px] + sum_m Z_c[m][px] alpha[p][j][m]
//           (Eq. wavefront on the (N/2)^2 pupil band, in turns)
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
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mfbd {
namespace contract {


typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(const floatx4& a, const floatx4& b, floatx4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
  return acc;
}

// One block = W waves x RT row tiles (16 RT rows (p,j)) x all mode columns
// x one of `splits` parts of the k range (blockIdx.y).  The k = c*bp + px
// range, in 16-wide chunks, is cut into W*splits nearly equal slices; wave w
// of split s sums slice s*W + w for all RT row tiles, so every basis chunk it
// loads serves RT x 16 rows (the basis reads through L2 are what bound this
// contraction).  Splitting k over blocks fills the chip when there are few
// row tiles.  Operands are loaded DEPTH chunks ahead.  The partial sums of a
// block are added in wave order (wave 0, then 1, ..., W-1) in one LDS buffer;
// with one split the block writes 2 pi times its sum to grad, otherwise its
// sum to part[s][R][M], which k_grad_combine adds in split order.  The
// basis rows are zero-padded to a multiple of 16 per basis, so no mode test
// is needed inside the loop; rows past R read row R-1 and are not written.
// Schedules: W = 4 with RT = 4 and DEPTH = 2, or W = 8 with RT = 2 and
// DEPTH = 1.  CS is the number of channels summed per load when they share
// one basis (0: the run-time C), fixed at compile time where it can be so
// that the loads of a chunk issue together.
//
// Row tile block `bx`, part `split` of `splits` of the k range.  `mt` (at
// most MT) is the number of 16-mode tiles the basis table holds; tiles
// beyond it are neither loaded nor multiplied.  CS < 0 selects at run time
// between separate bases per channel (zc == C) and one shared basis.
template <int MT, int RT, int W, int DEPTH, int CS>
__device__ __forceinline__ void grad_block(int bx, int split, int splits, int mt, int R, int J,
                                           int C, int zc, int M, int bp,
                                           const float* __restrict__ Ztp,
                                           const float* __restrict__ gphi,
                                           float* __restrict__ grad,
                                           float* __restrict__ part) {
  __shared__ floatx4 red[RT * MT][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int r0 = bx * 16 * RT;
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
  const int nchunk = zc * bp / 16, slices = W * splits, slice = split * W + wave;
  const int c_begin = (int)((long)slice * nchunk / slices);
  const int n = (int)((long)(slice + 1) * nchunk / slices) - c_begin;   // chunks of this wave
  const int k_begin = 16 * c_begin;
  const float* zrow = Ztp + (size_t)i16 * bp + 4 * g;
  // operands of chunk kk: a[q] from gphi row q*16 + i16 (with one shared
  // basis, the sum over channels in channel order), b[t] from mode row
  // t*16 + i16
  auto load = [&](int kk, floatx4 (&a4)[RT], floatx4 (&b4)[MT]) {
    const int c = kk / bp, px = kk % bp;
    const bool separate = CS == 1 || (CS < 0 && zc == C);
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      if (separate) {
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
    const float* zb = zrow + (size_t)c * mt * 16 * bp + px;   // bases of mt * 16 rows
#pragma unroll
    for (int t = 0; t < MT; ++t)
      b4[t] = t < mt ? *reinterpret_cast<const floatx4*>(zb + (size_t)t * 16 * bp)
                     : floatx4{0.f, 0.f, 0.f, 0.f};
  };
  auto compute = [&](const floatx4 (&a4)[RT], const floatx4 (&b4)[MT]) {
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
      for (int t = 0; t < MT; ++t)
        if (t < mt) acc[q][t] = mfma4(a4[q], b4[t], acc[q][t]);
  };
  if constexpr (DEPTH == 1) {
    floatx4 a_cur[RT], b_cur[MT];
    if (n > 0) load(k_begin, a_cur, b_cur);
    for (int i = 0; i < n; ++i) {
      floatx4 a_nxt[RT], b_nxt[MT];
      if (i + 1 < n) load(k_begin + 16 * (i + 1), a_nxt, b_nxt);
      compute(a_cur, b_cur);
      if (i + 1 < n) {
#pragma unroll
        for (int q = 0; q < RT; ++q) a_cur[q] = a_nxt[q];
#pragma unroll
        for (int t = 0; t < MT; ++t) b_cur[t] = b_nxt[t];
      }
    }
  } else {
    // two stages: chunks i and i + 1 in flight; an odd last chunk is in
    // stage 0
    floatx4 a0[RT], b0[MT], a1[RT], b1[MT];
    if (n > 0) load(k_begin, a0, b0);
    if (n > 1) load(k_begin + 16, a1, b1);
    int i = 0;
    for (; i + 2 <= n; i += 2) {
      compute(a0, b0);
      if (i + 2 < n) load(k_begin + 16 * (i + 2), a0, b0);
      compute(a1, b1);
      if (i + 3 < n) load(k_begin + 16 * (i + 3), a1, b1);
    }
    if (i < n) compute(a0, b0);
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
  float* out = splits == 1 ? grad : part + (size_t)split * R * M;
  const float scale = splits == 1 ? 6.283185307179586f : 1.0f;
  for (int qt = wave; qt < RT * MT; qt += W) {
    const int q = qt / MT, t = qt % MT;
    const floatx4 v = red[qt][lane];
    const int m = t * 16 + i16;
    if (m >= M) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + q * 16 + 4 * g + e;
      if (row < R) out[(size_t)row * M + m] = scale * v[e];
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
constexpr int kCols = kPhaseCols, kColTiles = kCols / 16;
__device__ __forceinline__ void phase_block(int bx, int by, int R, int J, int C, int zc, int M,
                                            int Mp, int bp, const float* __restrict__ ZtT,
                                            const float* __restrict__ theta,
                                            const float* __restrict__ alpha,
                                            float* __restrict__ phi) {
  // The coefficient tile is stored mode-major, al[m][col] with row stride
  // ldc = kCols + 4: a B operand element (k, j) of lane (i16 = j, g) is
  // al[(kk + 4g + s) ldc + 16t + i16], and with 4 ldc = 16 (mod 64) the 64
  // lanes of each read fall on distinct banks.  (Column-major rows of
  // Mp + 4 floats, read as float4, gave 4-way conflicts.)
  extern __shared__ float al[];    // [Mp][kCols + 4]
  constexpr int ldc = kCols + 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int c = bx >> 2, quarter = bx & 3;
  const int col0 = by * kCols;
  const int ncol = min(kCols, R - col0);
  const float* src = alpha + (size_t)col0 * M;
  for (int r = wave; r < kCols; r += 4)
    for (int m = lane; m < Mp; m += 64)
      al[m * ldc + r] = (r < ncol && m < M) ? src[(size_t)r * M + m] : 0.f;
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
        const float* bp4 = al + (kk + 4 * g) * ldc + t * 16 + i16;
        const floatx4 b4 = {bp4[0], bp4[ldc], bp4[2 * ldc], bp4[3 * ldc]};
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

}  // namespace contract
}  // namespace mfbd
