// Bodies of the dense modal contractions on the matrix cores (gfx950),
// shared by the kernels of one plan (gemm_mfma.hip) and of a group of fields
// (gemm_group.hip).
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
// FP32 operands on the bf16 matrix cores: every operand is split exactly
// into three bf16 parts (bf16split.h), and each 16x16x32 product is the sum
// of the six partial products hh, hm, mh, hl, lh, mm (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation).  The basis tables are split once, at plan creation;
// alpha is split as it is staged, gphi as it is loaded.  Operand layout of
// the instruction: lane l supplies A[i = l%16][k] and B[k][j = l%16] for the
// eight k of its lane group g = l/16, as eight packed bf16 (a uint4); the
// 16x16 result sits in 4 registers per lane, D[4g + e][l%16], e = 0..3.
// The k order is free as long as A and B agree, so lane group g takes the
// eight consecutive k = k0 + 8g .. k0 + 8g + 7 of a 32-wide chunk: one 16-byte
// load per part.
#pragma once

#include <hip/hip_runtime.h>

#include "bf16split.h"
#include "internal.h"

namespace mfbd {
namespace contract {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// The three parts of eight k values of one operand row or column.
struct Op3 {
  uint4 h, m, l;
};

__device__ __forceinline__ floatx4 mfma_bf16(const uint4& a, const uint4& b, floatx4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}

// acc + A B over one 32-wide k chunk, from the six partial products.
__device__ __forceinline__ floatx4 mfma6(const Op3& a, const Op3& b, floatx4 acc) {
  acc = mfma_bf16(a.m, b.m, acc);
  acc = mfma_bf16(a.l, b.h, acc);
  acc = mfma_bf16(a.h, b.l, acc);
  acc = mfma_bf16(a.m, b.h, acc);
  acc = mfma_bf16(a.h, b.m, acc);
  return mfma_bf16(a.h, b.h, acc);
}

__device__ __forceinline__ Op3 load_op3(const uint4* p) { return Op3{p[0], p[1], p[2]}; }

__device__ __forceinline__ Op3 split_op3(const float4& lo, const float4& hi) {
  const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  const Split8 s = split8(v);
  return Op3{make_uint4(s.h[0], s.h[1], s.h[2], s.h[3]), make_uint4(s.m[0], s.m[1], s.m[2], s.m[3]),
             make_uint4(s.l[0], s.l[1], s.l[2], s.l[3])};
}

// Gradient.  One block = W waves; wave w owns RT row tiles (16 RT rows
// (p, j)), so a block covers 16 W RT rows, for all mode columns and one of
// `splits` parts of the k = c*bp + px range (blockIdx.y), in 32-wide
// chunks.  The basis parts of a chunk (16 mt modes x 32 pixels x 3 parts)
// are staged in LDS once per block and serve every wave's rows; the stage
// is double-buffered (the next chunk's loads are in flight while the
// current one is multiplied; one barrier per chunk), and each wave loads
// the gphi values of its next chunk ahead as well.  A wave's sums are
// complete for its rows over the block's k range: with one split the wave
// writes 2 pi times them to grad, otherwise them to part[s][R][M], which
// k_grad_combine adds in split order.  The basis rows are zero-padded to a
// multiple of 16 per basis, so no mode test is needed inside the loop; rows
// past R read row R-1 and are not written.  CS is the number of channels
// summed per load when they share one basis (0: the run-time C), fixed at
// compile time where it can be so that the loads of a chunk issue together;
// CS < 0 selects at run time between separate bases per channel (zc == C)
// and one shared basis.  `mt` (at most MT) is the number of 16-mode tiles
// the basis table holds; tiles beyond it are neither loaded nor multiplied.
// Zs: the split basis, [zc][16 mt][bp/8][3] uint4 (eight pixels of one
// mode, parts hi, mid, lo).  LDS: two stages of 16 MT x kStageLd uint4.
constexpr int kStageLd = 13;   // uint4 per staged mode row: 4 groups x 3 parts, + 1 (banks)

__host__ __device__ __forceinline__ size_t grad_lds_bytes(int mt) {
  return (size_t)2 * 16 * mt * kStageLd * 16;
}

template <int MT, int RT, int W, int CS>
__device__ __forceinline__ void grad_block(int bx, int split, int splits, int mt, int R, int J,
                                           int C, int zc, int M, int bp,
                                           const uint4* __restrict__ Zs,
                                           const float* __restrict__ gphi,
                                           float* __restrict__ grad,
                                           float* __restrict__ part) {
  extern __shared__ uint4 zst[];   // [2][16 mt][kStageLd]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int r0 = (bx * W + wave) * 16 * RT;
  const size_t cstride = (size_t)J * bp;   // between the channels of one (p, j)
  const float* grow[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int r = min(r0 + q * 16 + i16, R - 1);
    grow[q] = gphi + ((size_t)(r / J) * C * J + r % J) * bp + 8 * g;
  }
  floatx4 acc[RT][MT];
#pragma unroll
  for (int q = 0; q < RT; ++q)
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[q][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nchunk = zc * bp / 32;
  const int c_begin = (int)((long)split * nchunk / splits);
  const int n = (int)((long)(split + 1) * nchunk / splits) - c_begin;   // chunks of this block
  const int bp8 = bp / 8;
  const int stage_n = 16 * mt * 12;                                     // uint4 per chunk
  constexpr int kPer = (16 * MT * 12 + 64 * W - 1) / (64 * W);          // per thread, at most
  const int sz = 16 * mt * kStageLd;
  // the basis parts of chunk kk: mode row m, 12 consecutive uint4 (groups
  // 0..3 x parts) from pixel kk % bp of basis kk / bp
  // (held in native vectors, which stay in registers)
  auto stage_load = [&](int kk, u32x4 (&v)[kPer]) {
    const int c = kk / bp, px = kk % bp;
    const u32x4* src =
        reinterpret_cast<const u32x4*>(Zs + ((size_t)c * mt * 16 * bp8 + px / 8) * 3);
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = threadIdx.x + e * 64 * W;
      if (idx < stage_n) v[e] = src[(size_t)(idx / 12) * bp8 * 3 + idx % 12];
    }
  };
  auto stage_store = [&](int buf, const u32x4 (&v)[kPer]) {
    u32x4* dst = reinterpret_cast<u32x4*>(zst + buf * sz);
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = threadIdx.x + e * 64 * W;
      if (idx < stage_n) dst[(idx / 12) * kStageLd + idx % 12] = v[e];
    }
  };
  // the eight gphi values of chunk kk in lane group g for each row tile
  // (with one shared basis, the sum over channels in channel order)
  auto load_a = [&](int kk, float4 (&raw)[RT][2]) {
    const int c = kk / bp, px = kk % bp;
    const bool separate = CS == 1 || (CS < 0 && zc == C);
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const float4* p0 = reinterpret_cast<const float4*>(grow[q] + (separate ? c * cstride : 0) + px);
      raw[q][0] = p0[0];
      raw[q][1] = p0[1];
      if (separate) continue;
      auto add = [&](int ch) {
        const float4* pc = reinterpret_cast<const float4*>(grow[q] + ch * cstride + px);
        const float4 u = pc[0], v = pc[1];
        raw[q][0] = make_float4(raw[q][0].x + u.x, raw[q][0].y + u.y, raw[q][0].z + u.z,
                                raw[q][0].w + u.w);
        raw[q][1] = make_float4(raw[q][1].x + v.x, raw[q][1].y + v.y, raw[q][1].z + v.z,
                                raw[q][1].w + v.w);
      };
      if constexpr (CS > 1) {
#pragma unroll
        for (int ch = 1; ch < CS; ++ch) add(ch);
      } else {
        for (int ch = 1; ch < C; ++ch) add(ch);
      }
    }
  };
  if (n > 0) {
    u32x4 v[kPer];
    stage_load(32 * c_begin, v);
    stage_store(0, v);
  }
  float4 raw[RT][2];
  if (n > 0) load_a(32 * c_begin, raw);
  __syncthreads();
  for (int i = 0; i < n; ++i) {
    const int kk = 32 * (c_begin + i);
    u32x4 v[kPer];
    if (i + 1 < n) stage_load(kk + 32, v);
    Op3 a[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) a[q] = split_op3(raw[q][0], raw[q][1]);
    if (i + 1 < n) load_a(kk + 32, raw);
    const uint4* zb = zst + (i & 1) * sz + i16 * kStageLd + 3 * g;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (t < mt) {
        const Op3 b = load_op3(zb + t * 16 * kStageLd);
#pragma unroll
        for (int q = 0; q < RT; ++q) acc[q][t] = mfma6(a[q], b, acc[q][t]);
      }
    }
    if (i + 1 < n) stage_store((i + 1) & 1, v);
    __syncthreads();
  }
  float* out = splits == 1 ? grad : part + (size_t)split * R * M;
  const float scale = splits == 1 ? 6.283185307179586f : 1.0f;
#pragma unroll
  for (int q = 0; q < RT; ++q)
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int m = t * 16 + i16;
      if (t >= mt || m >= M) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = r0 + q * 16 + 4 * g + e;
        if (row < R) out[(size_t)row * M + m] = scale * acc[q][t][e];
      }
    }
}

// phi^T per channel: D[px][col] = sum_m Z_c[m][px] alpha[col][m], col = p*J + j.
// Block = W waves, (basis, 16 CT columns, a quarter of the band pixels);
// with one shared basis the block writes every channel's phi from one
// product.  The block's coefficient rows (contiguous in alpha) are split
// and staged once in LDS, [col][m/8][part] with the modes padded to Mq (a
// multiple of 32); each wave then walks tiles of 16 pixels x 16 CT columns,
// taking its A parts from the split basis table ZsT[c][px][Mq/8][3] (uint4:
// eight modes of one pixel, loaded one step ahead) and its B parts from
// LDS.  Every basis part a wave loads serves CT column tiles, so the basis
// reads through L2 fall as 1 / CT.
// uint4 row stride of the staged coefficients: odd, so that the 16 columns
// one read touches fall on distinct 16-byte bank groups.
__host__ __device__ __forceinline__ int phase_lds_stride(int Mq) { return (3 * (Mq / 8)) | 1; }

__host__ __device__ __forceinline__ size_t phase_lds_bytes(int ct, int Mq) {
  return (size_t)16 * ct * phase_lds_stride(Mq) * 16;
}

template <int CT, int W>
__device__ __forceinline__ void phase_block(int bx, int by, int R, int J, int C, int zc, int M,
                                            int Mq, int bp, const uint4* __restrict__ ZsT,
                                            const float* __restrict__ theta,
                                            const float* __restrict__ alpha,
                                            float* __restrict__ phi) {
  constexpr int kCols = 16 * CT;
  extern __shared__ uint4 als[];   // [kCols][phase_lds_stride(Mq)]
  const int q8 = Mq / 8, ld = phase_lds_stride(Mq);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int c = bx >> 2, quarter = bx & 3;
  const int col0 = by * kCols;
  const int ncol = min(kCols, R - col0);
  const float* src = alpha + (size_t)col0 * M;
  for (int idx = threadIdx.x; idx < kCols * q8; idx += 64 * W) {
    const int r = idx / q8, m8 = idx % q8;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int m = 8 * m8 + e;
      v[e] = (r < ncol && m < M) ? src[(size_t)r * M + m] : 0.f;
    }
    const Split8 sp = split8(v);
    uint4* dst = als + r * ld + 3 * m8;
    dst[0] = make_uint4(sp.h[0], sp.h[1], sp.h[2], sp.h[3]);
    dst[1] = make_uint4(sp.m[0], sp.m[1], sp.m[2], sp.m[3]);
    dst[2] = make_uint4(sp.l[0], sp.l[1], sp.l[2], sp.l[3]);
  }
  __syncthreads();
  // 16-pixel tiles of the quarter: wave w takes tiles w, w + W, ...
  const int qtiles = bp / 64;
  const int ntile = (qtiles - wave + W - 1) / W;
  const int nct = (ncol + 15) / 16;  // column tiles holding columns
  const int nk = q8 / 4;             // 32-mode chunks per tile
  // (tile, chunk) steps in order; the A parts of the next step are loaded
  // while the current one is multiplied
  auto px_of = [&](int tile) { return quarter * (bp / 4) + (tile * W + wave) * 16; };
  auto load_a = [&](int it) {
    const int px0 = px_of(it / nk), k8 = (it % nk) * 4;
    return load_op3(ZsT + ((size_t)(c * bp + px0 + i16) * q8 + g + k8) * 3);
  };
  const int steps = ntile * nk;
  floatx4 acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  Op3 a;
  if (steps > 0) a = load_a(0);
  for (int it = 0; it < steps; ++it) {
    Op3 an = a;
    if (it + 1 < steps) an = load_a(it + 1);
    const int k8 = (it % nk) * 4;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      if (t < nct) {
        const Op3 b = load_op3(als + (t * 16 + i16) * ld + 3 * (k8 + g));
        acc[t] = mfma6(a, b, acc[t]);
      }
    }
    a = an;
    if (it % nk != nk - 1) continue;
    // the tile is complete: theta added, phi written, sums cleared
    const int px0 = px_of(it / nk);
    const int c_lo = zc == C ? c : 0, c_hi = zc == C ? c + 1 : C;
    for (int ch = c_lo; ch < c_hi; ++ch) {
      const floatx4 th =
          *reinterpret_cast<const floatx4*>(theta + (size_t)ch * bp + px0 + 4 * g);
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int col = col0 + t * 16 + i16;
        if (t >= nct || col >= R) continue;
        const int p = col / J, j = col % J;
        *reinterpret_cast<floatx4*>(phi + (((size_t)p * C + ch) * J + j) * bp + px0 + 4 * g) =
            acc[t] + th;
      }
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
}

}  // namespace contract
}  // namespace mfbd
