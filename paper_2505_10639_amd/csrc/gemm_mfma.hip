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
// basis rows are zero-padded to MT*16 per basis, so no mode test is needed
// inside the loop; rows past R read row R-1 and are not written.
// Schedules: W = 4 with RT = 4 and DEPTH = 2, or W = 8 with RT = 2 and
// DEPTH = 1.  CS is the number of channels summed per load when they share
// one basis (0: the run-time C), fixed at compile time where it can be so
// that the loads of a chunk issue together.
template <int MT, int RT, int W, int DEPTH, int CS>
__global__ __launch_bounds__(64 * W) void k_grad_mfma(int R, int J, int C, int zc, int M, int bp,
                                                      const float* __restrict__ Ztp,
                                                      const float* __restrict__ gphi,
                                                      float* __restrict__ grad,
                                                      float* __restrict__ part) {
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
  const int splits = gridDim.y, split = blockIdx.y;
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

// grad = 2 pi (part[0] + part[1] + ... + part[splits-1]), in that order.
__global__ __launch_bounds__(256) void k_grad_combine(long n, int splits,
                                                      const float* __restrict__ part,
                                                      float* __restrict__ grad) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float v = part[i];
  for (int s = 1; s < splits; ++s) v += part[(size_t)s * n + i];
  grad[i] = 6.283185307179586f * v;
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
  // The coefficient tile is stored mode-major, al[m][col] with row stride
  // ldc = kCols + 4: a B operand element (k, j) of lane (i16 = j, g) is
  // al[(kk + 4g + s) ldc + 16t + i16], and with 4 ldc = 16 (mod 64) the 64
  // lanes of each read fall on distinct banks.  (Column-major rows of
  // Mp + 4 floats, read as float4, gave 4-way conflicts.)
  extern __shared__ float al[];    // [Mp][kCols + 4]
  constexpr int ldc = kCols + 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int c = blockIdx.x >> 2, quarter = blockIdx.x & 3;
  const int col0 = blockIdx.y * kCols;
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

template <int MT, int CS>
void launch_grad_cs(const Dims& d, int zc, int splits, const float* Ztp, const float* gphi,
                    float* grad, float* part, hipStream_t s) {
  const int R = d.P * d.J;
  if (d.grad_waves == 8)
    hipLaunchKernelGGL((k_grad_mfma<MT, 2, 8, 1, CS>), dim3((R + 31) / 32, splits), dim3(512), 0,
                       s, R, d.J, d.C, zc, d.M, d.bandpix(), Ztp, gphi, grad, part);
  else if (grad_row_tiles_of(d) == 3)
    hipLaunchKernelGGL((k_grad_mfma<MT, 3, 4, 2, CS>), dim3((R + 47) / 48, splits), dim3(256), 0,
                       s, R, d.J, d.C, zc, d.M, d.bandpix(), Ztp, gphi, grad, part);
  else
    hipLaunchKernelGGL((k_grad_mfma<MT, 4, 4, 2, CS>), dim3((R + 63) / 64, splits), dim3(256), 0,
                       s, R, d.J, d.C, zc, d.M, d.bandpix(), Ztp, gphi, grad, part);
}

template <int MT>
void launch_grad_t(const Dims& d, int splits, const float* Ztp, const float* gphi, float* grad,
                   float* part, hipStream_t s) {
  const int zc = d.zc > 0 ? d.zc : d.C;
  if (zc == d.C)
    launch_grad_cs<MT, 1>(d, zc, splits, Ztp, gphi, grad, part, s);
  else if (d.C == 2)
    launch_grad_cs<MT, 2>(d, zc, splits, Ztp, gphi, grad, part, s);
  else
    launch_grad_cs<MT, 0>(d, zc, splits, Ztp, gphi, grad, part, s);
}

}  // namespace

int grad_splits_auto(const Dims& d) {
  // Measured on the 64x64 and 128x128 full fields: with fewer row-tile
  // blocks than CUs (256) splitting the pixel sum fills idle CUs; with more,
  // it only evens out the last round and pays when each wave keeps a long
  // run of chunks (128x128, four bases: 1.33 -> 1.03 ms at 2 splits), and
  // it costs when the runs get short (64x64: 40 us unsplit, 50 us at 4).
  const int R = d.P * d.J, W = d.grad_waves == 8 ? 8 : 4;
  const long rows = 16L * grad_row_tiles_of(d);
  const long blocks = (R + rows - 1) / rows;
  const int zc = d.zc > 0 ? d.zc : d.C;
  const int nchunk = zc * d.bandpix() / 16;
  int s = 1;
  while (s < kMaxGradSplits && 2 * s * W <= nchunk) {
    const bool fill = blocks * 2 * s <= 256;
    const bool tail = blocks * s < 512 && nchunk / (2 * s * W) >= 64;
    if (!fill && !(blocks >= 256 && tail)) break;
    s *= 2;
  }
  return s;
}

int grad_splits_of(const Dims& d) { return d.grad_splits > 0 ? d.grad_splits : grad_splits_auto(d); }

int grad_row_tiles_of(const Dims& d) { return d.grad_waves == 8 ? 2 : d.grad_rt == 3 ? 3 : 4; }

hipError_t launch_grad(const Dims& d, const float* Zt, const float* gphi, float* grad,
                       float* part, hipStream_t s) {
  const int mt = (d.M + 15) / 16;
  const int splits = grad_splits_of(d);
  switch (mt) {
#define MFBD_CASE(n) \
  case n: launch_grad_t<n>(d, splits, Zt, gphi, grad, part, s); break;
    MFBD_CASE(1) MFBD_CASE(2) MFBD_CASE(3) MFBD_CASE(4) MFBD_CASE(5) MFBD_CASE(6)
    MFBD_CASE(7) MFBD_CASE(8) MFBD_CASE(9) MFBD_CASE(10) MFBD_CASE(11) MFBD_CASE(12)
    MFBD_CASE(13) MFBD_CASE(14) MFBD_CASE(15) MFBD_CASE(16)
#undef MFBD_CASE
    default: return hipErrorInvalidValue;
  }
  if (splits > 1) {
    const long n = (long)d.P * d.J * d.M;
    hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       splits, part, grad);
  }
  return hipGetLastError();
}

hipError_t launch_phase(const Dims& d, const float* alpha, const float* ZtT, int Mp,
                        const float* thetat, float* phi, hipStream_t s) {
  const int R = d.P * d.J, zc = d.zc > 0 ? d.zc : d.C;
  dim3 grid(zc * 4, (R + kCols - 1) / kCols);
  const size_t lds = (size_t)Mp * (kCols + 4) * sizeof(float);
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
