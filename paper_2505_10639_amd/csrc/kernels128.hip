// Unit kernels of the MOMFBD hot path for 128x128 patches (gfx950).
//
// One workgroup of four wavefronts (256 lanes) per unit (patch, channel,
// frame); the wave-level transforms are those of ops128.h.  The pupil band is
// 64x64 (rows and columns [32,96) of the grid).  Same algebra as the 64x64
// kernels: forward PSF/OTF, adjoint to dL/dphi, patch preparation, object
// image.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ops128.h"

namespace mfbd {
using namespace n128;

namespace {

constexpr int kUnitF2 = N * HC;        // 8320 float2 per half spectrum
constexpr int kB = 64;                 // band width
constexpr int kBP = kB * kB;           // band pixels
constexpr int kThreads = 256;
constexpr int kXcds = 8;

__device__ __forceinline__ void sync() { __syncthreads(); }

__device__ __forceinline__ float2 expi_turns(float t) {
  const float f = __builtin_amdgcn_fractf(t);
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
}

// op1 column-pass input of lane (q, r): z[n] = y[n] + y[n+32] with
// y[n] = P(32+n, 32+q) W128^{+(32+n) r}, P = A exp(2 pi i t) on the band; the
// modulation is a phase ramp of (32+n) r / 128 turns.
__device__ __forceinline__ void build_pupil(const float* __restrict__ A,
                                            const float* __restrict__ ph, int lane,
                                            float2 (&z)[32]) {
  const int q = lane >> 2, r = lane & 3;
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    const int n1 = n + 32;
    const float2 y0 = cscale(expi_turns(ph[n * kB + q] + (32 + n) * r * (1.0f / 128.0f)),
                             A[n * kB + q]);
    const float2 y1 = cscale(expi_turns(ph[n1 * kB + q] + (32 + n1) * r * (1.0f / 128.0f)),
                             A[n1 * kB + q]);
    z[n] = cadd(y0, y1);
  }
}

// The forward unit transforms through a half-size buffer of floats (real
// parts, then imaginary parts, for both transposes): 34.8 KB of LDS per
// workgroup instead of 68.6 KB, so that registers, not LDS, set how many
// workgroups a CU holds.
template <bool WANT_PSF>
__device__ __forceinline__ void forward128_unit(int u, const ChanTab& ct, int C, int J,
                                                const int* __restrict__ active,
                                                const float* __restrict__ Ab,
                                                const float* __restrict__ phi,
                                                float* __restrict__ psf,
                                                float2* __restrict__ S) {
  __shared__ float Th[LDS_HALF];
  __shared__ float2 Taux[LDS_AUX];
  if (active && !active[u / (J * C)]) return;
  const int lane = threadIdx.x;
  const int c = (u / J) % C;
  float2 p[64];
  {
    float2 z[32];
    __builtin_amdgcn_s_setprio(2);
    build_pupil(Ab + (size_t)c * kBP, phi + (size_t)u * kBP, lane, z);
    __builtin_amdgcn_s_setprio(0);
    fft32<+1>(z);
    op1_cols_put<0>(z, Th, lane);
    sync();
    op1_rows_get<0>(Th, lane, p);
    sync();
    op1_cols_put<1>(z, Th, lane);
  }
  sync();
  op1_rows_get<1>(Th, lane, p);
  op1_rows_fft(p, lane);
  // half the PSF row (op2_rows_values takes s / 2; the factor is exact)
  float s[64];
  const float kap_half = 0.5f * ct.kappa[c];
#pragma unroll
  for (int m = 0; m < 64; ++m) s[m] = kap_half * cabs2(p[m]);
  if (WANT_PSF) {
    float* row = psf + (size_t)u * N * N + (lane >> 1) * N;
    const int e = lane & 1;
#pragma unroll
    for (int m = 0; m < 64; ++m) row[2 * m + e] = 2.0f * s[m];
  }
  float2 v[32];
  {
    float keep[32], send[32], other[32];
    op2_rows_fold(s, keep, send, lane);
    sync();
    xput(send, Th, lane);
    sync();
    xget(Th, lane, other);
    op2_rows_values(keep, other, lane, v);
  }
  sync();
  op2_rows_put<0>(v, Th, lane);
  sync();
  float ax[32], bx[32];
  op2_cols_half_x(Th, lane, ax, bx);
  sync();
  op2_rows_put<1>(v, Th, lane);
  sync();
  float2 X[32], x64;
  op2_cols_half_y(Th, Taux, lane, ax, bx, X);
  sync();
  float2* T2 = reinterpret_cast<float2*>(Th);
  if (lane < 128) x64 = op2_unpack(Taux, T2, lane);
  sync();
  op2_collect(T2, lane, X);
  float2* out = S + (size_t)u * kUnitF2;
#pragma unroll
  for (int m = 0; m < 32; ++m) out[sl_index(lane, m)] = X[m];
  if (lane < 128) out[sl_index64(lane)] = x64;
}

template <bool WANT_PSF>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_forward128(int units, int xcd, ChanTab ct, int C,
                                                        int J, const int* __restrict__ active,
                                                        const float* __restrict__ Ab,
                                                        const float* __restrict__ phi,
                                                        float* __restrict__ psf,
                                                        float2* __restrict__ S) {
  const int u = xcd ? (blockIdx.x % kXcds) * ((units + kXcds - 1) / kXcds) + blockIdx.x / kXcds
                    : blockIdx.x;
  if (u >= units) return;
  forward128_unit<WANT_PSF>(u, ct, C, J, active, Ab, phi, psf, S);
}

// Every unit of every field of a group (XCD order over the group's units).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_forward128_group(GroupArgs ga, int xcd) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  const int g = xcd ? (blockIdx.x % kXcds) * per + blockIdx.x / kXcds : blockIdx.x;
  if (g >= ga.total) return;
  const int2 it = ga.item[g];
  const FieldDesc& F = ga.fd[it.x];
  forward128_unit<false>(it.y, F.ct, F.d.C, F.d.J, F.active, F.Ab, F.w.phi, nullptr,
                        F.w.S);
}

__device__ __forceinline__ void adjoint128_unit(int u, const ChanTab& ct, int C, int J, int K,
                                                const LossArgs& la,
                                                const int* __restrict__ active,
                                                const float* __restrict__ Ab,
                                                const float* __restrict__ phi,
                                                const float2* __restrict__ S,
                                                const float2* __restrict__ O,
                                                float* __restrict__ gphi) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int lane = threadIdx.x;
  const int j = u % J;
  const int c = (u / J) % C;
  const int p = u / (J * C);
  if (active && !active[p]) return;
  const int k = ct.chan_obj[c];
  const float w2 = -2.0f * (la.weights ? la.weights[c * J + j] : 1.0f);

  // G = conj(O)(D - O S) in spectral layout (the frame factor -2 w is applied
  // with 2 kappa after the inverse transform; G(ky, 64) of lanes < 128
  // into Taux[ky]); zero outside the object's spectral support, where D, S
  // and O are not read
  float2 G[32];
  __builtin_amdgcn_s_setprio(2);
  {
    const int r = wave_of(lane);
    constexpr int kOut = kUnitF2 * 8;
    const __amdgpu_buffer_rsrc_t rS = raw_buffer(S + (size_t)u * kUnitF2, kOut),
                                 rD = raw_buffer(la.D + (size_t)u * kUnitF2, kOut),
                                 rO = raw_buffer(O + ((size_t)p * K + k) * kUnitF2, kOut);
    const int fm = la.supp[k * HC + (lane & 63)];
#pragma unroll
    for (int m = 0; m < 32; ++m) {
      const int off = in_support(4 * m + r, N, fm) ? sl_index(lane, m) * 8 : kOut;
      G[m] = adjoint_input(buffer_load_f2(rD, off), buffer_load_f2(rS, off),
                           buffer_load_f2(rO, off));
    }
    if (lane < 128) {
      const int off = in_support(lane, N, la.supp[k * HC + 64]) ? sl_index64(lane) * 8 : kOut;
      Taux[lane] = adjoint_input(buffer_load_f2(rD, off), buffer_load_f2(rS, off),
                                 buffer_load_f2(rO, off));
    }
  }
  __builtin_amdgcn_s_setprio(0);
  sync();
  op3_cols(G, Taux, T, lane);
  sync();
  op3_cols_combine(T, lane, G);
  sync();
  op3_cols_put(G, T, lane);
  sync();
  float g[64];
  {
    float keep[32], send[32], other[32];
    op3_rows_compute(T, lane, keep, send);
    sync();
    xput(send, reinterpret_cast<float*>(T), lane);
    sync();
    xget(reinterpret_cast<const float*>(T), lane, other);
    sync();
    op3_rows_finish(keep, other, lane, g);
  }
  // recompute the PSF amplitude p and form H = -4 w kappa g p
  const float* Ac = Ab + (size_t)c * kBP;
  const float* phu = phi + (size_t)u * kBP;
  {
    float2 z[32];
    build_pupil(Ac, phu, lane, z);
    op1_cols(z, T, lane);
  }
  sync();
  float2 H[64];
  op1_rows(T, lane, H);
  const float k2 = 2.0f * ct.kappa[c] * w2;   // w2: the frame's -2 w
#pragma unroll
  for (int m = 0; m < 64; ++m) H[m] = cscale(H[m], k2 * g[m]);
  sync();
  {
    float2 keep[32], other[32];
    op4_rows_fft(H, keep, T, lane);
    sync();
    xget(T, lane, other);
    sync();
    op4_rows_finish(keep, other, T, lane);
  }
  sync();
  {
    float2 GP[16];
    op4_cols(T, lane, GP);
    const int r = wave_of(lane), q = lane & 63;
    float* gout = gphi + (size_t)u * kBP;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int n = 4 * i + r;
      const float2 pk = cscale(expi_turns(phu[n * kB + q]), Ac[n * kB + q]);
      gout[n * kB + q] = pk.x * GP[i].y - pk.y * GP[i].x;   // Im(conj(P) G_P)
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_adjoint128(
    int units, int xcd, ChanTab ct, int C, int J, int K, LossArgs la,
    const int* __restrict__ active, const float* __restrict__ Ab, const float* __restrict__ phi,
    const float2* __restrict__ S, const float2* __restrict__ O, float* __restrict__ gphi) {
  // XCD-aware order: consecutive units (frames of one patch-object) on one XCD
  const int per = (units + kXcds - 1) / kXcds;
  const int u = xcd ? (blockIdx.x % kXcds) * per + blockIdx.x / kXcds : blockIdx.x;
  if (u >= units) return;
  adjoint128_unit(u, ct, C, J, K, la, active, Ab, phi, S, O, gphi);
}

__global__ __launch_bounds__(kThreads) void k_adjoint128_group(GroupArgs ga, int xcd) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  const int g = xcd ? (blockIdx.x % kXcds) * per + blockIdx.x / kXcds : blockIdx.x;
  if (g >= ga.total) return;
  const int2 it = ga.item[g];
  const FieldDesc& F = ga.fd[it.x];
  adjoint128_unit(it.y, F.ct, F.d.C, F.d.J, F.d.K, F.la, F.active, F.Ab, F.w.phi,
                  F.w.S, F.w.O, F.w.gphi);
}

__global__ __launch_bounds__(kThreads) void k_prepare128(int units, int C, int J, int H, int W,
                                                         int stride, int nx,
                                                         const float* __restrict__ frames,
                                                         const float* __restrict__ apod,
                                                         float2* __restrict__ D) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  __shared__ float red[kThreads];
  const int u = blockIdx.x;
  if (u >= units) return;
  const int lane = threadIdx.x;
  const int j = u % J;
  const int c = (u / J) % C;
  const int p = u / (J * C);
  const int y0 = (p / nx) * stride, x0 = (p % nx) * stride;
  float* Tf = reinterpret_cast<float*>(T);
  const float* src = frames + ((size_t)(c * J + j) * H + y0) * W + x0;
  for (int e = lane; e < N * N; e += kThreads) {
    const int r = e >> 7, x = e & 127;
    Tf[r * 129 + x] = src[(size_t)r * W + x];
  }
  sync();
  const int y = lane >> 1, e = lane & 1;
  float s[64];
  float sum = 0.f;
#pragma unroll
  for (int m = 0; m < 64; ++m) {
    s[m] = Tf[y * 129 + 2 * m + e];
    sum += s[m];
  }
  red[lane] = sum;
  sync();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (lane < h) red[lane] += red[lane + h];
    sync();
  }
  const float mean = red[0] * (1.0f / (N * N));
  const float* wr = apod + y * N;
  // half the apodized row (op2_rows_values takes s / 2)
#pragma unroll
  for (int m = 0; m < 64; ++m) s[m] = 0.5f * (wr[2 * m + e] * (s[m] - mean) + mean);
  float2 X[32], x64;
  {
    float keep[32], send[32], other[32];
    op2_rows_fold(s, keep, send, lane);
    xput(send, Tf, lane);
    sync();
    xget(Tf, lane, other);
    sync();
    op2_rows_finish(keep, other, T, lane);
  }
  sync();
  op2_cols(T, Taux, lane, X);
  sync();
  if (lane < 128) x64 = op2_unpack(Taux, T, lane);
  sync();
  op2_collect(T, lane, X);
  float2* out = D + (size_t)u * kUnitF2;
#pragma unroll
  for (int m = 0; m < 32; ++m) out[sl_index(lane, m)] = X[m];
  if (lane < 128) out[sl_index64(lane)] = x64;
}

// out = IDFT(A B) / N^2 + sg nz for one half spectrum A (times B when B is
// given; plus sg times the noise image nz when nz is given).
__device__ __forceinline__ void inverse_item(const float2* __restrict__ A,
                                             const float2* __restrict__ B,
                                             float* __restrict__ out,
                                             const float* __restrict__ nz, float sg) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  const int lane = threadIdx.x;
  float2 X[32];
#pragma unroll
  for (int m = 0; m < 32; ++m)
    X[m] = B ? cmul(A[sl_index(lane, m)], B[sl_index(lane, m)]) : A[sl_index(lane, m)];
  if (lane < 128)
    Taux[lane] = B ? cmul(A[sl_index64(lane)], B[sl_index64(lane)]) : A[sl_index64(lane)];
  sync();
  op3_cols(X, Taux, T, lane);
  sync();
  op3_cols_combine(T, lane, X);
  sync();
  op3_cols_put(X, T, lane);
  sync();
  float g[64];
  {
    float keep[32], send[32], other[32];
    op3_rows_compute(T, lane, keep, send);
    sync();
    xput(send, reinterpret_cast<float*>(T), lane);
    sync();
    xget(reinterpret_cast<const float*>(T), lane, other);
    op3_rows_finish(keep, other, lane, g);
  }
  const int r = (lane >> 1) * N, e = lane & 1;
  float* row = out + r;
  const float inv = 1.0f / (N * N);
#pragma unroll
  for (int m = 0; m < 64; ++m)
    row[2 * m + e] = g[m] * inv + (nz ? sg * nz[r + 2 * m + e] : 0.f);
}

// Item it = (it / per, it % per), `stride` items between consecutive values
// of it / per (object images: per = items, stride 0).
__global__ __launch_bounds__(kThreads) void k_objimg128(int items, int per, int stride,
                                                        const float2* __restrict__ O,
                                                        float* __restrict__ obj) {
  const int it = blockIdx.x;
  if (it >= items) return;
  inverse_item(O + ((size_t)(it / per) * stride + it % per) * kUnitF2, nullptr,
               obj + (size_t)it * N * N, nullptr, 0.f);
}

// Synthetic frames i = IDFT(O_k S_u) / N^2 + sigma_p n_u into [C][J][P*N][N].
__global__ __launch_bounds__(kThreads) void k_synth128(int units, int P, int C, int J, int K,
                                                       ChanTab ct,
                                                       const float2* __restrict__ O,
                                                       const float2* __restrict__ S,
                                                       const float* __restrict__ noise,
                                                       const float* __restrict__ sigma,
                                                       float* __restrict__ field) {
  const int u = blockIdx.x;
  if (u >= units) return;
  const int j = u % J, c = (u / J) % C, p = u / (J * C);
  inverse_item(O + ((size_t)p * K + ct.chan_obj[c]) * kUnitF2, S + (size_t)u * kUnitF2,
               field + ((size_t)(c * J + j) * P + p) * N * N, noise + (size_t)u * N * N,
               sigma[p]);
}

}  // namespace

hipError_t launch_forward128(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                             const float* phi, float* psf, float2* S, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const dim3 grid(d.xcd_fwd ? kXcds * ((units + kXcds - 1) / kXcds) : units);
  if (psf)
    hipLaunchKernelGGL(k_forward128<true>, grid, dim3(kThreads), 0, s, units, d.xcd_fwd, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  else
    hipLaunchKernelGGL(k_forward128<false>, grid, dim3(kThreads), 0, s, units, d.xcd_fwd, ct, d.C,
                       d.J, active, Ab, phi, psf, S);
  return hipGetLastError();
}

hipError_t launch_adjoint128(const Dims& d, const ChanTab& ct, const LossArgs& la,
                             const int* active, const float* Ab, const float* phi,
                             const float2* S, const float2* O, float* gphi, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const int per = (units + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_adjoint128, dim3(d.xcd_adj ? kXcds * per : units), dim3(kThreads), 0, s,
                     units, d.xcd_adj, ct, d.C, d.J,
                     d.K, la, active, Ab, phi, S, O, gphi);
  return hipGetLastError();
}

hipError_t launch_forward128_group(const GroupArgs& ga, int xcd, hipStream_t s) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_forward128_group, dim3(xcd ? kXcds * per : ga.total), dim3(kThreads), 0,
                     s, ga, xcd);
  return hipGetLastError();
}

hipError_t launch_adjoint128_group(const GroupArgs& ga, int xcd, hipStream_t s) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_adjoint128_group, dim3(xcd ? kXcds * per : ga.total), dim3(kThreads), 0,
                     s, ga, xcd);
  return hipGetLastError();
}

hipError_t launch_prepare128(const Dims& d, const float* frames, int H, int W, int stride,
                             const float* apod, float2* D, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const int nx = (W - N) / stride + 1;
  hipLaunchKernelGGL(k_prepare128, dim3(units), dim3(kThreads), 0, s, units, d.C, d.J, H, W,
                     stride, nx, frames, apod, D);
  return hipGetLastError();
}

hipError_t launch_objimg128(const Dims& d, const float2* O, float* obj, hipStream_t s) {
  const int items = d.P * d.K;
  hipLaunchKernelGGL(k_objimg128, dim3(items), dim3(kThreads), 0, s, items, items, 0, O, obj);
  return hipGetLastError();
}

hipError_t launch_frames128(int items, int per, int stride, const float2* D, float* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_objimg128, dim3(items), dim3(kThreads), 0, s, items, per, stride, D, out);
  return hipGetLastError();
}

hipError_t launch_synth128(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                           const float* noise, const float* sigma, float* field, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  hipLaunchKernelGGL(k_synth128, dim3(units), dim3(kThreads), 0, s, units, d.P, d.C, d.J, d.K,
                     ct, O, S, noise, sigma, field);
  return hipGetLastError();
}

}  // namespace mfbd
