// Warm-start network: a convolutional regressor from a burst of frames to
// per-frame modal coefficients, trained and run on the matrix cores
// (BF16 operands, FP32 accumulation: v_mfma_f32_16x16x16_bf16).
//
// Architecture (input: J frames of N x N, N = 64, 96 or 128, NHWC with the
// frames as channels):
//   conv 3x3 stride 2 pad 1, J -> 32, ReLU        N -> N/2
//   conv 3x3 stride 2 pad 1, 32 -> 64, ReLU       N/2 -> N/4
//   conv 3x3 stride 2 pad 1, 64 -> 128, ReLU      N/4 -> N/8
//   conv 3x3 stride 2 pad 1, 128 -> 128, ReLU     N/8 -> N/16
//   dense 128 (N/16)^2 -> 512, ReLU               (2048 at N = 64)
//   dense 512 -> J*M (linear), times the per-mode scale
// Convolutions are an explicit im2col followed by one GEMM; the backward
// pass is two GEMMs per layer (weights: dZ^T col, data: dZ W) and a gather
// col2im.  Weights and activations are stored in bfloat16, biases, master
// weights, gradients and Adam moments in FP32.  Every reduction runs in a
// fixed order, so results are bitwise reproducible.
//
// Loss (per frame): the burst mean of the tilt modes is removed from
// prediction and target, and the squared error is the smaller of those to
// the target and to the target with its even-radial-order modes negated,
// the two symmetries that leave the frames unchanged without diversity.
// Mode m's error is weighted by scale_m^2 / mean(scale^2): the loss is the
// wavefront error in units of the mean mode variance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "momfbd.h"

namespace mfbd {
namespace {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  long sam, sak;        // A(m, k) = A[m*sam + k*sak]
  const uint16_t* B;
  long sbk, sbn;        // B(k, n) = B[k*sbk + n*sbn]
  float* C;             // partial products [splits][M][N]
  int kchunk;           // k range of one split, a multiple of 32
};

// C_z = A B over the split's k range.  Block = 4 waves = a 64 x 64 tile;
// wave (wm, wn) owns 32 x 32 = 2 x 2 MFMA tiles.  Operand layout of the
// instruction: lane l supplies A[i = l%16][k = 4(l/16) + 0..3] and
// B[k = 4(l/16) + 0..3][j = l%16]; it returns D[4(l/16) + e][l%16].
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ uint16_t As[64][40];
  __shared__ uint16_t Bs[64][40];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kb = blockIdx.z * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const int wm = wave >> 1, wn = wave & 1;
  const int i16 = lane & 15, kg = lane >> 4;
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + 256 * e;
      int mm, kk;
      if (g.sak == 1) {
        kk = idx & 31;
        mm = idx >> 5;
      } else {
        mm = idx & 63;
        kk = idx >> 6;
      }
      const int m = m0 + mm, k = k0 + kk;
      As[mm][kk] = (m < g.M && k < ke) ? g.A[(long)m * g.sam + (long)k * g.sak] : (uint16_t)0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + 256 * e;
      int nn, kk;
      if (g.sbn == 1) {
        nn = idx & 63;
        kk = idx >> 6;
      } else {
        kk = idx & 31;
        nn = idx >> 5;
      }
      const int n = n0 + nn, k = k0 + kk;
      Bs[nn][kk] = (n < g.N && k < ke) ? g.B[(long)k * g.sbk + (long)n * g.sbn] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 32; ks += 16) {
      short4v a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const uint16_t* pa = &As[wm * 32 + t * 16 + i16][ks + 4 * kg];
        const uint16_t* pb = &Bs[wn * 32 + t * 16 + i16][ks + 4 * kg];
        a[t] = short4v{(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
        b[t] = short4v{(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    __syncthreads();
  }
  float* Cz = g.C + (long)blockIdx.z * g.M * g.N;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 32 + mi * 16 + 4 * kg + e;
        const int n = n0 + wn * 32 + ni * 16 + i16;
        if (m < g.M && n < g.N) Cz[(long)m * g.N + n] = acc[mi][ni][e];
      }
}

// out = sum_z part_z (+ bias) (ReLU), as FP32 and/or bfloat16
__global__ __launch_bounds__(256) void k_epilogue(long MN, int N, int splits,
                                                  const float* __restrict__ part,
                                                  const float* __restrict__ bias, int relu,
                                                  float* __restrict__ out32,
                                                  uint16_t* __restrict__ out16) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= MN) return;
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += part[(long)z * MN + i];
  if (bias) v += bias[i % N];
  if (relu) v = fmaxf(v, 0.f);
  if (out32) out32[i] = v;
  if (out16) out16[i] = f2bf(v);
}

__global__ __launch_bounds__(256) void k_im2col(int B, int H, int W, int Ci,
                                                const uint16_t* __restrict__ x,
                                                uint16_t* __restrict__ col) {
  const int Ho = H / 2, Wo = W / 2;
  const long n = (long)B * Ho * Wo * 9 * Ci;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int ci = (int)(idx % Ci);
  long r = idx / Ci;
  const int kx = (int)(r % 3);
  r /= 3;
  const int ky = (int)(r % 3);
  r /= 3;
  const int ox = (int)(r % Wo);
  r /= Wo;
  const int oy = (int)(r % Ho);
  const int b = (int)(r / Ho);
  const int y = 2 * oy + ky - 1, xx = 2 * ox + kx - 1;
  col[idx] = (y >= 0 && y < H && xx >= 0 && xx < W) ? x[(((long)b * H + y) * W + xx) * Ci + ci]
                                                    : (uint16_t)0;
}

// dx[b][y][x][ci] = sum of the im2col entries that read x[b][y][x][ci]
__global__ __launch_bounds__(256) void k_col2im(int B, int H, int W, int Ci,
                                                const float* __restrict__ dcol,
                                                float* __restrict__ dx) {
  const int Ho = H / 2, Wo = W / 2;
  const long n = (long)B * H * W * Ci;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int ci = (int)(idx % Ci);
  long r = idx / Ci;
  const int x = (int)(r % W);
  r /= W;
  const int y = (int)(r % H);
  const int b = (int)(r / H);
  float s = 0.f;
  for (int ky = 0; ky < 3; ++ky) {
    const int ty = y + 1 - ky;
    if (ty < 0 || (ty & 1) || ty / 2 >= Ho) continue;
    for (int kx = 0; kx < 3; ++kx) {
      const int tx = x + 1 - kx;
      if (tx < 0 || (tx & 1) || tx / 2 >= Wo) continue;
      s += dcol[(((long)b * Ho + ty / 2) * Wo + tx / 2) * (9 * Ci) + (ky * 3 + kx) * Ci + ci];
    }
  }
  dx[idx] = s;
}

// dz = bfloat16(dh * [h > 0]): the ReLU of the layer that produced h
__global__ __launch_bounds__(256) void k_relu_back(long n, const float* __restrict__ dh,
                                                   const uint16_t* __restrict__ h,
                                                   uint16_t* __restrict__ dz) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  dz[i] = f2bf(bf2f(h[i]) > 0.f ? dh[i] : 0.f);
}

__global__ __launch_bounds__(256) void k_cast_bf16(long n, const float* __restrict__ x,
                                                   uint16_t* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// db[n] = sum_m dz[m][n]; one block per column, fixed-order tree
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const uint16_t* __restrict__ dz,
                                                float* __restrict__ db) {
  __shared__ float red[256];
  const int n = blockIdx.x, tid = threadIdx.x;
  float s = 0.f;
  for (int m = tid; m < M; m += 256) s += bf2f(dz[(long)m * N + n]);
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) db[n] = red[0];
}

// frames [B*J][npix] FP32 -> NHWC bfloat16 [B][npix][J]:
// 10 (f / mean - 1) per frame; one block per frame
// (WIDE: the rounded values as floats, for momfbd_cnn_input)
template <bool WIDE = false>
__global__ __launch_bounds__(256) void k_norm_frames(int J, int npix, const float* __restrict__ f,
                                                     uint16_t* __restrict__ x,
                                                     float* __restrict__ xw = nullptr) {
  __shared__ float red[256];
  const int u = blockIdx.x, tid = threadIdx.x;
  const int b = u / J, j = u % J;
  const float* fu = f + (long)u * npix;
  float s = 0.f;
  for (int i = tid; i < npix; i += 256) s += fu[i];
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const float inv = (float)npix / red[0];
  for (int i = tid; i < npix; i += 256) {
    const uint16_t h = f2bf(10.f * (fu[i] * inv - 1.f));
    if (WIDE) xw[((long)b * npix + i) * J + j] = bf2f(h);
    else x[((long)b * npix + i) * J + j] = h;
  }
}

constexpr int kMaxJM = 2048;

// Per burst: scaled prediction alpha = z * scale, loss and dL/dz.
// One block per burst; thread t handles (j, m) = (t / M, t % M) for
// t = tid, tid + 1024.
__global__ __launch_bounds__(1024) void k_burst_loss(int B, int J, int M,
                                                     const float* __restrict__ z,
                                                     const float* __restrict__ target,
                                                     const float* __restrict__ scale,
                                                     const float* __restrict__ weight,
                                                     const int* __restrict__ even,
                                                     double* __restrict__ loss_b,
                                                     float* __restrict__ dz) {
  __shared__ float p[kMaxJM], q[kMaxJM], d1[kMaxJM], d2[kMaxJM], g[kMaxJM];
  __shared__ float e1[64], e2[64];
  __shared__ float tm[4];
  const int b = blockIdx.x, tid = threadIdx.x, JM = J * M;
  // work in units of the per-mode scale (the network's own output units)
  for (int t = tid; t < JM; t += 1024) {
    p[t] = z[(long)b * JM + t];
    q[t] = target[(long)b * JM + t] / scale[t % M];
  }
  __syncthreads();
  if (tid < 4) {           // burst means of the two tilt modes
    const int mm = tid & 1;
    const float* src = tid < 2 ? p : q;
    float s = 0.f;
    for (int jj = 0; jj < J; ++jj) s += src[jj * M + mm];
    tm[tid] = s / J;
  }
  __syncthreads();
  // tilt-centred values replace p and q (each element is read and written by
  // its own thread only)
  for (int t = tid; t < JM; t += 1024) {
    const int m = t % M;
    const float pv = p[t] - (m < 2 ? tm[m] : 0.f);
    const float qv = q[t] - (m < 2 ? tm[2 + m] : 0.f);
    const float sg = even[m] ? -1.f : 1.f;
    d1[t] = weight[m] * (pv - qv) * (pv - qv);
    d2[t] = weight[m] * (pv - sg * qv) * (pv - sg * qv);
    p[t] = pv;
    q[t] = qv;
  }
  __syncthreads();
  if (tid < J) {
    float a = 0.f, c = 0.f;
    for (int mm = 0; mm < M; ++mm) {
      a += d1[tid * M + mm];
      c += d2[tid * M + mm];
    }
    e1[tid] = a;
    e2[tid] = c;
  }
  __syncthreads();
  const float inv = 1.f / ((float)B * J);
  for (int t = tid; t < JM; t += 1024) {
    const int j = t / M, m = t % M;
    const float sg = even[m] ? -1.f : 1.f;
    const bool flip = e2[j] < e1[j];
    g[t] = 2.f * weight[m] * (p[t] - (flip ? sg * q[t] : q[t])) * inv;
  }
  __syncthreads();
  for (int t = tid; t < JM; t += 1024) {
    const int m = t % M;
    float gv = g[t];
    if (m < 2) {
      float s = 0.f;
      for (int jj = 0; jj < J; ++jj) s += g[jj * M + m];
      gv -= s / J;
    }
    dz[(long)b * JM + t] = gv;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int jj = 0; jj < J; ++jj) s += (double)fminf(e1[jj], e2[jj]);
    loss_b[b] = s * (double)inv;
  }
}

__global__ __launch_bounds__(256) void k_scale_pred(long n, int M, const float* __restrict__ z,
                                                    const float* __restrict__ scale,
                                                    float* __restrict__ alpha) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) alpha[i] = z[i] * scale[i % M];
}

__global__ void k_sum_loss(int B, const double* __restrict__ lb, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += lb[b];
  *loss = s;
}

__global__ __launch_bounds__(256) void k_adam(long n, float* __restrict__ w,
                                              const float* __restrict__ g, float* __restrict__ m1,
                                              float* __restrict__ m2, uint16_t* __restrict__ w16,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  const float wi = w[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
  w[i] = wi;
  if (w16) w16[i] = f2bf(wi);
}

// scaled normals -> parameters: He initialisation of the weights, zero biases
__global__ __launch_bounds__(256) void k_init(long n, const float* __restrict__ normals,
                                              const float* __restrict__ std_of,
                                              float* __restrict__ w) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) w[i] = normals[i] * std_of[i];
}

unsigned blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace mfbd

using namespace mfbd;

struct Layer {
  bool conv;
  int ci, co, h;         // conv: input channels, output channels, input side
  int n_in, n_out;       // dense
  long w_off, b_off;     // offsets into the flat parameter vector
  long rows;             // GEMM rows per burst (output pixels) and K
  int K;
};

struct momfbd_cnn_s {
  int N, J, M, batch_max;
  long n_params;
  std::vector<Layer> layers;
  float* scale = nullptr;     // [M] device
  float* weight = nullptr;    // [M] device: scale^2 / mean(scale^2)
  int* even = nullptr;        // [M] device
  float* init_std = nullptr;  // [n_params] device
  size_t ws_bytes = 0;
  // workspace offsets (bytes)
  size_t o_frames, o_x0, o_col[4], o_y[5], o_z, o_part, o_dz, o_dh, o_dz2, o_w16, o_lossb;
  size_t part_floats;
  int device = -1;
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// GEMM through the partial buffer and the epilogue; the split count keeps
// the grid near 2048 blocks when the output is small and K large.
hipError_t gemm(const momfbd_cnn_s* n, char* ws, int M, int N, int K, const uint16_t* A, long sam,
                long sak, const uint16_t* B, long sbk, long sbn, const float* bias, int relu,
                float* out32, uint16_t* out16, hipStream_t s) {
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  const int kc32 = (K + 31) / 32;
  int splits = 1;
  while (splits * 2 <= kc32 && (long)tm * tn * splits * 2 <= 2048 && splits < 256) splits *= 2;
  while ((long)splits * M * N > (long)n->part_floats && splits > 1) splits /= 2;
  if ((long)M * N > (long)n->part_floats) return hipErrorInvalidValue;
  const int kchunk = ((kc32 + splits - 1) / splits) * 32;
  splits = (K + kchunk - 1) / kchunk;
  float* part = reinterpret_cast<float*>(ws + n->o_part);
  GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, part, kchunk};
  hipLaunchKernelGGL(k_gemm_bf16, dim3(tm, tn, splits), dim3(256), 0, s, g);
  const long MN = (long)M * N;
  hipLaunchKernelGGL(k_epilogue, dim3(blocks(MN)), dim3(256), 0, s, MN, N, splits, part, bias,
                     relu, out32, out16);
  return hipGetLastError();
}

// frames of the bursts' first channel: the apodized patches
// W(x - m) + m = IDFT(D) / N^2 of D [B][C][J][N][N/2+1], channel 0
hipError_t frames_from_spectra(const momfbd_cnn_s* n, int B, int C, const void* D, char* ws,
                               hipStream_t s) {
  return launch_frames(n->N, B * n->J, n->J, C * n->J, static_cast<const float2*>(D),
                       reinterpret_cast<float*>(ws + n->o_frames), s);
}

hipError_t run_forward(const momfbd_cnn_s* n, const float* params, const void* D, int B, int C,
                       char* ws, hipStream_t s) {
  hipError_t e = frames_from_spectra(n, B, C, D, ws, s);
  if (e != hipSuccess) return e;
  uint16_t* x0 = reinterpret_cast<uint16_t*>(ws + n->o_x0);
  hipLaunchKernelGGL(k_norm_frames<false>, dim3(B * n->J), dim3(256), 0, s, n->J, n->N * n->N,
                     reinterpret_cast<const float*>(ws + n->o_frames), x0, nullptr);
  const uint16_t* w16 = reinterpret_cast<const uint16_t*>(ws + n->o_w16);
  const uint16_t* h = x0;
  for (size_t l = 0; l < n->layers.size(); ++l) {
    const Layer& L = n->layers[l];
    const float* bias = params + L.b_off;
    const bool last = l + 1 == n->layers.size();
    if (L.conv) {
      uint16_t* col = reinterpret_cast<uint16_t*>(ws + n->o_col[l]);
      const long ncol = (long)B * L.rows * L.K;
      hipLaunchKernelGGL(k_im2col, dim3(blocks(ncol)), dim3(256), 0, s, B, L.h, L.h, L.ci, h, col);
      uint16_t* y = reinterpret_cast<uint16_t*>(ws + n->o_y[l]);
      e = gemm(n, ws, (int)(B * L.rows), L.co, L.K, col, L.K, 1, w16 + L.w_off, 1, L.K, bias, 1,
               nullptr, y, s);
      h = y;
    } else if (!last) {
      uint16_t* y = reinterpret_cast<uint16_t*>(ws + n->o_y[l]);
      e = gemm(n, ws, B, L.n_out, L.n_in, h, L.n_in, 1, w16 + L.w_off, 1, L.n_in, bias, 1, nullptr,
               y, s);
      h = y;
    } else {
      e = gemm(n, ws, B, L.n_out, L.n_in, h, L.n_in, 1, w16 + L.w_off, 1, L.n_in, bias, 0,
               reinterpret_cast<float*>(ws + n->o_z), nullptr, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A network and a workspace that is 256-byte aligned and at least
// momfbd_cnn_sizes' workspace_bytes long.
int check_ws(const momfbd_cnn_s* n, const void* ws, size_t ws_bytes) {
  if (!n) return MOMFBD_EINVAL;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 || ws_bytes < n->ws_bytes)
    return MOMFBD_EWORKSPACE;
  return MOMFBD_OK;
}

int check_net(const momfbd_cnn_s* n, const void* ws, size_t ws_bytes, int B) {
  const int st = check_ws(n, ws, ws_bytes);
  if (st) return st;
  if (B < 1 || B > n->batch_max) return MOMFBD_EINVAL;
  return MOMFBD_OK;
}

int status_of(hipError_t e) { return e == hipSuccess ? MOMFBD_OK : MOMFBD_EDEVICE; }

}  // namespace

extern "C" {

int momfbd_cnn_create(int N, int J, int M, int batch_max, const float* mode_scale,
                      momfbd_cnn* out) {
  if (!out || !mode_scale || J < 1 || M < 2 || batch_max < 1 || (long)J * M > kMaxJM ||
      J > 64)
    return MOMFBD_EINVAL;
  if (N != 64 && N != 96 && N != 128) return MOMFBD_EUNSUPPORTED;
  for (int m = 0; m < M; ++m)
    if (!(mode_scale[m] > 0.f) || !std::isfinite(mode_scale[m])) return MOMFBD_EINVAL;
  momfbd_cnn_s* n = new (std::nothrow) momfbd_cnn_s();
  if (!n) return MOMFBD_EDEVICE;
  n->N = N;
  n->J = J;
  n->M = M;
  n->batch_max = batch_max;
  const int chans[5] = {J, 32, 64, 128, 128};
  long off = 0;
  int side = N;
  for (int l = 0; l < 4; ++l) {
    Layer L{};
    L.conv = true;
    L.ci = chans[l];
    L.co = chans[l + 1];
    L.h = side;
    L.K = 9 * L.ci;
    L.rows = (long)(side / 2) * (side / 2);
    L.w_off = off;
    off += (long)L.co * L.K;
    L.b_off = off;
    off += L.co;
    n->layers.push_back(L);
    side /= 2;
  }
  const int dense_in[2] = {128 * side * side, 512}, dense_out[2] = {512, J * M};
  for (int l = 0; l < 2; ++l) {
    Layer L{};
    L.conv = false;
    L.n_in = dense_in[l];
    L.n_out = dense_out[l];
    L.K = L.n_in;
    L.rows = 1;
    L.w_off = off;
    off += (long)L.n_out * L.n_in;
    L.b_off = off;
    off += L.n_out;
    n->layers.push_back(L);
  }
  n->n_params = off;
  // workspace
  const long Bm = batch_max;
  size_t o = 0;
  n->o_frames = o;
  o = al256(o + (size_t)Bm * J * N * N * sizeof(float));
  n->o_x0 = o;
  o = al256(o + (size_t)Bm * J * N * N * sizeof(uint16_t));
  size_t max_dh = 0;
  for (int l = 0; l < 4; ++l) {
    const Layer& L = n->layers[l];
    n->o_col[l] = o;
    o = al256(o + (size_t)Bm * L.rows * L.K * sizeof(uint16_t));
    n->o_y[l] = o;
    o = al256(o + (size_t)Bm * L.rows * L.co * sizeof(uint16_t));
    max_dh = std::max(max_dh, (size_t)Bm * L.rows * L.K);               // dcol
    max_dh = std::max(max_dh, (size_t)Bm * L.h * L.h * L.ci);           // dx
  }
  n->o_y[4] = o;
  o = al256(o + (size_t)Bm * 512 * sizeof(uint16_t));
  n->o_z = o;
  o = al256(o + (size_t)Bm * J * M * sizeof(float));
  // partial products: the largest GEMM output times a few splits
  size_t part = 0;
  for (const Layer& L : n->layers) {
    part = std::max(part, (size_t)Bm * L.rows * (L.conv ? L.co : L.n_out));
    part = std::max(part, (size_t)(L.conv ? L.co : L.n_out) * L.K * 64);
    part = std::max(part, (size_t)Bm * L.rows * L.K);
  }
  n->part_floats = part;
  n->o_part = o;
  o = al256(o + part * sizeof(float));
  n->o_dz = o;
  o = al256(o + max_dh * sizeof(uint16_t));
  n->o_dz2 = o;
  o = al256(o + max_dh * sizeof(uint16_t));
  n->o_dh = o;
  o = al256(o + max_dh * sizeof(float));
  n->o_w16 = o;
  o = al256(o + (size_t)n->n_params * sizeof(uint16_t));
  n->o_lossb = o;
  o = al256(o + (size_t)Bm * sizeof(double));
  n->ws_bytes = o;
  // tables
  std::vector<int> even(M);
  for (int m = 0; m < M; ++m) {
    const int j = m + 2;
    int r = 0;
    while ((r + 1) * (r + 2) / 2 < j) ++r;
    even[m] = (r % 2 == 0) ? 1 : 0;
  }
  std::vector<float> stdv(n->n_params, 0.f);
  for (const Layer& L : n->layers) {
    const float sd = std::sqrt(2.0f / (float)L.K);
    const long nw = L.conv ? (long)L.co * L.K : (long)L.n_out * L.n_in;
    for (long i = 0; i < nw; ++i) stdv[L.w_off + i] = sd;
  }
  // the last layer starts small: the first predictions are near zero
  const Layer& Ll = n->layers.back();
  for (long i = 0; i < (long)Ll.n_out * Ll.n_in; ++i) stdv[Ll.w_off + i] *= 0.1f;
  std::vector<float> wt(M);
  double mean2 = 0.0;
  for (int m = 0; m < M; ++m) mean2 += (double)mode_scale[m] * mode_scale[m] / M;
  for (int m = 0; m < M; ++m) wt[m] = (float)((double)mode_scale[m] * mode_scale[m] / mean2);
  bool ok = hipGetDevice(&n->device) == hipSuccess &&
            hipMalloc(&n->scale, M * sizeof(float)) == hipSuccess &&
            hipMalloc(&n->weight, M * sizeof(float)) == hipSuccess &&
            hipMemcpy(n->weight, wt.data(), M * sizeof(float), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMalloc(&n->even, M * sizeof(int)) == hipSuccess &&
            hipMalloc(&n->init_std, n->n_params * sizeof(float)) == hipSuccess &&
            hipMemcpy(n->scale, mode_scale, M * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(n->even, even.data(), M * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(n->init_std, stdv.data(), n->n_params * sizeof(float),
                      hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    momfbd_cnn_destroy(n);
    return MOMFBD_EDEVICE;
  }
  *out = n;
  return MOMFBD_OK;
}

int momfbd_cnn_destroy(momfbd_cnn net) {
  if (!net) return MOMFBD_OK;
  if (net->scale) (void)hipFree(net->scale);
  if (net->weight) (void)hipFree(net->weight);
  if (net->even) (void)hipFree(net->even);
  if (net->init_std) (void)hipFree(net->init_std);
  delete net;
  return MOMFBD_OK;
}

int momfbd_cnn_sizes(momfbd_cnn net, size_t* n_params, size_t* workspace_bytes) {
  if (!net) return MOMFBD_EINVAL;
  if (n_params) *n_params = (size_t)net->n_params;
  if (workspace_bytes) *workspace_bytes = net->ws_bytes;
  return MOMFBD_OK;
}

int momfbd_cnn_init(momfbd_cnn net, const float* normals, float* params, void* ws,
                    size_t ws_bytes, void* stream) {
  const int st = check_ws(net, ws, ws_bytes);
  if (st) return st;
  if (!normals || !params) return MOMFBD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_init, dim3(blocks(net->n_params)), dim3(256), 0, s, net->n_params, normals,
                     net->init_std, params);
  hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(net->n_params)), dim3(256), 0, s, net->n_params,
                     params, reinterpret_cast<uint16_t*>(static_cast<char*>(ws) + net->o_w16));
  return status_of(hipGetLastError());
}

int momfbd_cnn_load(momfbd_cnn net, const float* params, void* ws, size_t ws_bytes,
                    void* stream) {
  const int st = check_ws(net, ws, ws_bytes);
  if (st) return st;
  if (!params) return MOMFBD_EINVAL;
  hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(net->n_params)), dim3(256), 0, (hipStream_t)stream,
                     net->n_params, params,
                     reinterpret_cast<uint16_t*>(static_cast<char*>(ws) + net->o_w16));
  return status_of(hipGetLastError());
}

int momfbd_cnn_forward(momfbd_cnn net, const float* params, const void* D, int B, int C,
                       float* alpha, void* ws, size_t ws_bytes, void* stream) {
  int st = check_net(net, ws, ws_bytes, B);
  if (st) return st;
  if (!params || !D || !alpha || C < 1) return MOMFBD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  hipError_t e = run_forward(net, params, D, B, C, w, s);
  if (e != hipSuccess) return MOMFBD_EDEVICE;
  const long n = (long)B * net->J * net->M;
  hipLaunchKernelGGL(k_scale_pred, dim3(blocks(n)), dim3(256), 0, s, n, net->M,
                     reinterpret_cast<const float*>(w + net->o_z), net->scale, alpha);
  return status_of(hipGetLastError());
}

int momfbd_cnn_input(momfbd_cnn net, const void* D, int B, int C, float* x, void* ws,
                     size_t ws_bytes, void* stream) {
  int st = check_net(net, ws, ws_bytes, B);
  if (st) return st;
  if (!D || !x || C < 1) return MOMFBD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  hipError_t e = frames_from_spectra(net, B, C, D, w, s);
  if (e != hipSuccess) return MOMFBD_EDEVICE;
  hipLaunchKernelGGL(k_norm_frames<true>, dim3(B * net->J), dim3(256), 0, s, net->J,
                     net->N * net->N, reinterpret_cast<const float*>(w + net->o_frames), nullptr,
                     x);
  return status_of(hipGetLastError());
}

int momfbd_cnn_loss_grad(momfbd_cnn net, const float* params, const void* D, int C,
                         const float* target, int B, double* loss, float* grad, void* ws,
                         size_t ws_bytes, void* stream) {
  int st = check_net(net, ws, ws_bytes, B);
  if (st) return st;
  if (!params || !D || !target || !loss || !grad || C < 1) return MOMFBD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  hipError_t e = run_forward(net, params, D, B, C, w, s);
  if (e != hipSuccess) return MOMFBD_EDEVICE;
  const int J = net->J, M = net->M, JM = J * M;
  float* dh = reinterpret_cast<float*>(w + net->o_dh);
  uint16_t* dz = reinterpret_cast<uint16_t*>(w + net->o_dz);
  uint16_t* dz2 = reinterpret_cast<uint16_t*>(w + net->o_dz2);
  const uint16_t* w16 = reinterpret_cast<const uint16_t*>(w + net->o_w16);
  double* lb = reinterpret_cast<double*>(w + net->o_lossb);
  hipLaunchKernelGGL(k_burst_loss, dim3(B), dim3(1024), 0, s, B, J, M,
                     reinterpret_cast<const float*>(w + net->o_z), target, net->scale,
                     net->weight, net->even,
                     lb, dh);
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, s, B, lb, loss);
  hipLaunchKernelGGL(k_cast_bf16, dim3(blocks((long)B * JM)), dim3(256), 0, s, (long)B * JM, dh, dz);
  const int nl = (int)net->layers.size();
  for (int l = nl - 1; l >= 0; --l) {
    const Layer& L = net->layers[l];
    // input activation of this layer (bfloat16)
    const uint16_t* hin = l == 0 ? reinterpret_cast<const uint16_t*>(w + net->o_x0)
                                 : reinterpret_cast<const uint16_t*>(w + net->o_y[l - 1]);
    if (!L.conv) {
      // dW = dz^T h_in [n_out][n_in]; db = column sums; dh = dz W [B][n_in]
      e = gemm(net, w, L.n_out, L.n_in, B, dz, 1, L.n_out, hin, L.n_in, 1, nullptr, 0,
               grad + L.w_off, nullptr, s);
      if (e != hipSuccess) return MOMFBD_EDEVICE;
      hipLaunchKernelGGL(k_colsum, dim3(L.n_out), dim3(256), 0, s, B, L.n_out, dz, grad + L.b_off);
      e = gemm(net, w, B, L.n_in, L.n_out, dz, L.n_out, 1, w16 + L.w_off, L.n_in, 1, nullptr, 0, dh,
               nullptr, s);
      if (e != hipSuccess) return MOMFBD_EDEVICE;
      const long nin = (long)B * L.n_in;
      hipLaunchKernelGGL(k_relu_back, dim3(blocks(nin)), dim3(256), 0, s, nin, dh, hin, dz2);
    } else {
      const long Mrows = (long)B * L.rows;
      const uint16_t* col = reinterpret_cast<const uint16_t*>(w + net->o_col[l]);
      e = gemm(net, w, L.co, L.K, (int)Mrows, dz, 1, L.co, col, L.K, 1, nullptr, 0, grad + L.w_off,
               nullptr, s);
      if (e != hipSuccess) return MOMFBD_EDEVICE;
      hipLaunchKernelGGL(k_colsum, dim3(L.co), dim3(256), 0, s, (int)Mrows, L.co, dz,
                         grad + L.b_off);
      if (l == 0) break;
      // dcol = dz W [Mrows][K] into dh; its gather into dx reuses the
      // partial-product buffer, free again once the epilogue has run
      e = gemm(net, w, (int)Mrows, L.K, L.co, dz, L.co, 1, w16 + L.w_off, L.K, 1, nullptr, 0, dh,
               nullptr, s);
      if (e != hipSuccess) return MOMFBD_EDEVICE;
      const long nx = (long)B * L.h * L.h * L.ci;
      float* dx = reinterpret_cast<float*>(w + net->o_part);
      hipLaunchKernelGGL(k_col2im, dim3(blocks(nx)), dim3(256), 0, s, B, L.h, L.h, L.ci, dh, dx);
      hipLaunchKernelGGL(k_relu_back, dim3(blocks(nx)), dim3(256), 0, s, nx, dx, hin, dz2);
    }
    uint16_t* t = dz;
    dz = dz2;
    dz2 = t;
  }
  return status_of(hipGetLastError());
}

int momfbd_cnn_adam(momfbd_cnn net, float* params, const float* grad, float* m1, float* m2,
                    int step, float lr, float beta1, float beta2, float eps, void* ws,
                    size_t ws_bytes, void* stream) {
  const int st = check_ws(net, ws, ws_bytes);
  if (st) return st;
  if (!params || !grad || !m1 || !m2 || step < 1) return MOMFBD_EINVAL;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(net->n_params)), dim3(256), 0, (hipStream_t)stream,
                     net->n_params, params, grad, m1, m2,
                     reinterpret_cast<uint16_t*>(static_cast<char*>(ws) + net->o_w16), lr, beta1,
                     beta2, eps, c1, c2);
  return status_of(hipGetLastError());
}

}  // extern "C"
