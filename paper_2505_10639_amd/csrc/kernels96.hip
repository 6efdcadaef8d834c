// Unit kernels of the MOMFBD hot path for 96x96 patches (gfx950).
//
// One workgroup = two wavefronts = one unit (patch p, channel c, frame j);
// lanes 0..95 carry the lines of the 96-point transforms, lanes 96..127 only
// take part in the barriers.  Same stages as the 64x64 kernels:
//   forward : phase -> pupil -> inverse 2-D DFT -> |.|^2 -> forward 2-D DFT
//   adjoint : G = conj(O)(D - O S) -> inverse DFT -> H = -4 w kappa g p
//             -> forward DFT on the pupil band -> dL/dphi = Im(conj(P) G_P)
//   prepare : patch cut, mean removal, apodization, mean restore, 2-D DFT
//   objimg  : object spectrum -> real image / N^2
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ops96.h"

namespace mfbd {
using namespace n96;

namespace {

constexpr int kUnitF2 = N * HC;        // 4704
constexpr int kB = 48;                 // band width
constexpr int kBP = kB * kB;           // band pixels, 2304
constexpr int kThreads = 128;
constexpr int kXcds = 8;

__device__ __forceinline__ void sync() { __syncthreads(); }

__device__ __forceinline__ float2 expi_turns(float t) {
  const float f = __builtin_amdgcn_fractf(t);
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
}

// Input of op1_cols for lane (q,b): y[n] = P(24+n, 24+q) W96^{+b(24+n)}.
__device__ __forceinline__ void build_pupil(const float* __restrict__ A,
                                            const float* __restrict__ ph, int lane,
                                            float2 (&y)[48]) {
  const int q = lane >> 1, b = lane & 1;
#pragma unroll
  for (int n = 0; n < 48; ++n) {
    const float a = A[n * kB + q];
    const float t = ph[n * kB + q] + (b ? (24 + n) * (1.0f / 96.0f) : 0.0f);
    y[n] = cscale(expi_turns(t), a);
  }
}

template <bool WANT_PSF>
__device__ __forceinline__ void forward96_unit(int u, const ChanTab& ct, int C, int J,
                                                const int* __restrict__ active,
                                                const float* __restrict__ Ab,
                                                const float* __restrict__ phi,
                                                float* __restrict__ psf,
                                                float2* __restrict__ S) {
  __shared__ float2 T[LDS_MAIN];
  __shared__ float2 Taux[LDS_AUX];
  if (active && !active[u / (J * C)]) return;
  const int lane = threadIdx.x;
  const bool on = lane < LANES;
  const int c = (u / J) % C;
  if (on) {
    float2 y[48];
    __builtin_amdgcn_s_setprio(2);
    build_pupil(Ab + c * kBP, phi + (size_t)u * kBP, lane, y);
    __builtin_amdgcn_s_setprio(0);
    op1_cols(y, T, lane);
  }
  sync();
  float se[48], so[48];
  if (on) {
    float2 pe[48], po[48];
    op1_rows(T, lane, pe, po);
    const float kap = ct.kappa[c];
#pragma unroll
    for (int n = 0; n < 48; ++n) {
      se[n] = kap * cabs2(pe[n]);
      so[n] = kap * cabs2(po[n]);
    }
    if (WANT_PSF) {
      float* row = psf + (size_t)u * N * N + lane * N;
#pragma unroll
      for (int n = 0; n < 48; ++n) {
        row[2 * n] = se[n];
        row[2 * n + 1] = so[n];
      }
    }
  }
  sync();
  if (on) op2_rows(se, so, T, lane);
  sync();
  float2 X[48];
  if (on) op2_cols(T, Taux, lane, X);
  sync();
  float2 x48;
  if (on) x48 = op2_unpack(Taux, T, lane);
  sync();
  if (on) {
    op2_collect(T, lane, X);
    float2* out = S + (size_t)u * kUnitF2;
#pragma unroll
    for (int m = 0; m < 48; ++m) out[sl_index(lane, m)] = X[m];
    out[sl_index48(lane)] = x48;
  }
}

template <bool WANT_PSF>
__global__ __launch_bounds__(kThreads) void k_forward96(int units, int xcd, ChanTab ct, int C,
                                                        int J, const int* __restrict__ active,
                                                        const float* __restrict__ Ab,
                                                        const float* __restrict__ phi,
                                                        float* __restrict__ psf,
                                                        float2* __restrict__ S) {
  const int u = xcd ? (blockIdx.x % kXcds) * ((units + kXcds - 1) / kXcds) + blockIdx.x / kXcds
                    : blockIdx.x;
  if (u >= units) return;
  forward96_unit<WANT_PSF>(u, ct, C, J, active, Ab, phi, psf, S);
}

// Every unit of every field of a group (XCD order over the group's units).
__global__ __launch_bounds__(kThreads) void k_forward96_group(GroupArgs ga, int xcd) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  const int g = xcd ? (blockIdx.x % kXcds) * per + blockIdx.x / kXcds : blockIdx.x;
  if (g >= ga.total) return;
  const int2 it = ga.item[g];
  const FieldDesc& F = ga.fd[it.x];
  forward96_unit<false>(it.y, F.ct, F.d.C, F.d.J, F.active, F.Ab, F.w.phi, nullptr,
                        F.w.S);
}

// Two waves per SIMD: the kernel's register demand is a few registers over
// the 256 that allow it, and holding it there (a 32-byte spill) makes the
// kernel a third faster than one wave per SIMD.
__device__ __forceinline__ void adjoint96_unit(int u, const ChanTab& ct, int C, int J, int K,
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
  const bool on = lane < LANES;
  const int j = u % J, c = (u / J) % C, p = u / (J * C);
  if (active && !active[p]) return;
  const int k = ct.chan_obj[c];
  const float w2 = -2.0f * (la.weights ? la.weights[c * J + j] : 1.0f);
  float2 G[48];
  __builtin_amdgcn_s_setprio(2);
  if (on) {
    // zero outside the object's spectral support, where D, S and O are not read
    constexpr int kOut = kUnitF2 * 8;
    const __amdgpu_buffer_rsrc_t rS = raw_buffer(S + (size_t)u * kUnitF2, kOut),
                                 rD = raw_buffer(la.D + (size_t)u * kUnitF2, kOut),
                                 rO = raw_buffer(O + ((size_t)p * K + k) * kUnitF2, kOut);
    const int fm = la.supp[k * HC + (lane >> 1)];
#pragma unroll
    for (int m = 0; m < 48; ++m) {
      const int off = in_support(2 * m + (lane & 1), N, fm) ? sl_index(lane, m) * 8 : kOut;
      G[m] = adjoint_input(buffer_load_f2(rD, off), buffer_load_f2(rS, off),
                           buffer_load_f2(rO, off));
    }
    const int off = in_support(lane, N, la.supp[k * HC + 48]) ? sl_index48(lane) * 8 : kOut;
    op3_gather(adjoint_input(buffer_load_f2(rD, off), buffer_load_f2(rS, off),
                             buffer_load_f2(rO, off)),
               Taux, lane);
  }
  __builtin_amdgcn_s_setprio(0);
  sync();
  if (on) op3_cols(G, Taux, T, lane);
  sync();
  float ge[48], go[48];
  if (on) op3_rows(T, lane, ge, go);
  sync();
  const float* Ac = Ab + c * kBP;
  const float* phu = phi + (size_t)u * kBP;
  if (on) {
    float2 y[48];
    build_pupil(Ac, phu, lane, y);
    op1_cols(y, T, lane);
  }
  sync();
  float2 Gr[48];
  if (on) op14_rows(T, lane, ge, go, 2.0f * ct.kappa[c] * w2, Gr);   // w2: the frame's -2 w
  sync();
  if (on) op14_write(Gr, T, lane);
  sync();
  if (on) {
    float2 GP[24];
    op4_cols(T, lane, GP);
    const int b = lane & 1, q = lane >> 1;
    float* gout = gphi + (size_t)u * kBP;
#pragma unroll
    for (int i = 0; i < 24; ++i) {
      const int n = 2 * i + b;
      const float2 pk = cscale(expi_turns(phu[n * kB + q]), Ac[n * kB + q]);
      gout[n * kB + q] = pk.x * GP[i].y - pk.y * GP[i].x;   // Im(conj(P) G_P)
    }
  }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_adjoint96(
    int units, int xcd, ChanTab ct, int C, int J, int K, LossArgs la,
    const int* __restrict__ active, const float* __restrict__ Ab, const float* __restrict__ phi,
    const float2* __restrict__ S, const float2* __restrict__ O, float* __restrict__ gphi) {
  // XCD-aware order: consecutive units (frames of one patch-object) on one XCD
  const int per = (units + kXcds - 1) / kXcds;
  const int u = xcd ? (blockIdx.x % kXcds) * per + blockIdx.x / kXcds : blockIdx.x;
  if (u >= units) return;
  adjoint96_unit(u, ct, C, J, K, la, active, Ab, phi, S, O, gphi);
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_adjoint96_group(GroupArgs ga, int xcd) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  const int g = xcd ? (blockIdx.x % kXcds) * per + blockIdx.x / kXcds : blockIdx.x;
  if (g >= ga.total) return;
  const int2 it = ga.item[g];
  const FieldDesc& F = ga.fd[it.x];
  adjoint96_unit(it.y, F.ct, F.d.C, F.d.J, F.d.K, F.la, F.active, F.Ab, F.w.phi,
                  F.w.S, F.w.O, F.w.gphi);
}

__global__ __launch_bounds__(kThreads) void k_prepare96(int units, int C, int J, int H, int W,
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
  const bool on = lane < LANES;
  const int j = u % J, c = (u / J) % C, p = u / (J * C);
  const int y0 = (p / nx) * stride, x0 = (p % nx) * stride;
  const float* src = frames + ((size_t)(c * J + j) * H + y0) * W + x0;
  float se[48], so[48];
  float sum = 0.f;
  if (on) {
    const float* row = src + (size_t)lane * W;
#pragma unroll
    for (int n = 0; n < 48; ++n) {
      se[n] = row[2 * n];
      so[n] = row[2 * n + 1];
      sum += se[n] + so[n];
    }
  }
  red[lane] = sum;
  sync();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (lane < h) red[lane] += red[lane + h];
    sync();
  }
  const float mean = red[0] * (1.0f / (N * N));
  if (on) {
    const float* wr = apod + lane * N;
#pragma unroll
    for (int n = 0; n < 48; ++n) {
      se[n] = wr[2 * n] * (se[n] - mean) + mean;
      so[n] = wr[2 * n + 1] * (so[n] - mean) + mean;
    }
    op2_rows(se, so, T, lane);
  }
  sync();
  float2 X[48];
  if (on) op2_cols(T, Taux, lane, X);
  sync();
  float2 x48;
  if (on) x48 = op2_unpack(Taux, T, lane);
  sync();
  if (on) {
    op2_collect(T, lane, X);
    float2* out = D + (size_t)u * kUnitF2;
#pragma unroll
    for (int m = 0; m < 48; ++m) out[sl_index(lane, m)] = X[m];
    out[sl_index48(lane)] = x48;
  }
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
  const bool on = lane < LANES;
  float2 X[48];
  if (on) {
#pragma unroll
    for (int m = 0; m < 48; ++m)
      X[m] = B ? cmul(A[sl_index(lane, m)], B[sl_index(lane, m)]) : A[sl_index(lane, m)];
    op3_gather(B ? cmul(A[sl_index48(lane)], B[sl_index48(lane)]) : A[sl_index48(lane)], Taux,
               lane);
  }
  sync();
  if (on) op3_cols(X, Taux, T, lane);
  sync();
  if (on) {
    float ge[48], go[48];
    op3_rows(T, lane, ge, go);
    float* row = out + lane * N;
    const float inv = 1.0f / (N * N);
#pragma unroll
    for (int n = 0; n < 48; ++n) {
      row[2 * n] = ge[n] * inv + (nz ? sg * nz[lane * N + 2 * n] : 0.f);
      row[2 * n + 1] = go[n] * inv + (nz ? sg * nz[lane * N + 2 * n + 1] : 0.f);
    }
  }
}

// Item it = (it / per, it % per), `stride` items between consecutive values
// of it / per (object images: per = items, stride 0).
__global__ __launch_bounds__(kThreads) void k_objimg96(int items, int per, int stride,
                                                       const float2* __restrict__ O,
                                                       float* __restrict__ obj) {
  const int it = blockIdx.x;
  if (it >= items) return;
  inverse_item(O + ((size_t)(it / per) * stride + it % per) * kUnitF2, nullptr,
               obj + (size_t)it * N * N, nullptr, 0.f);
}

// Synthetic frames i = IDFT(O_k S_u) / N^2 + sigma_p n_u into [C][J][P*N][N].
__global__ __launch_bounds__(kThreads) void k_synth96(int units, int P, int C, int J, int K,
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

hipError_t launch_forward96(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                            const float* phi, float* psf, float2* S, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const dim3 grid(d.xcd_fwd ? kXcds * ((units + kXcds - 1) / kXcds) : units);
  if (psf)
    hipLaunchKernelGGL(k_forward96<true>, grid, dim3(kThreads), 0, s, units, d.xcd_fwd, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  else
    hipLaunchKernelGGL(k_forward96<false>, grid, dim3(kThreads), 0, s, units, d.xcd_fwd, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  return hipGetLastError();
}

hipError_t launch_adjoint96(const Dims& d, const ChanTab& ct, const LossArgs& la,
                            const int* active, const float* Ab, const float* phi, const float2* S,
                            const float2* O, float* gphi, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const int per = (units + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_adjoint96, dim3(d.xcd_adj ? kXcds * per : units), dim3(kThreads), 0, s,
                     units, d.xcd_adj, ct, d.C, d.J,
                     d.K, la, active, Ab, phi, S, O, gphi);
  return hipGetLastError();
}

hipError_t launch_forward96_group(const GroupArgs& ga, int xcd, hipStream_t s) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_forward96_group, dim3(xcd ? kXcds * per : ga.total), dim3(kThreads), 0,
                     s, ga, xcd);
  return hipGetLastError();
}

hipError_t launch_adjoint96_group(const GroupArgs& ga, int xcd, hipStream_t s) {
  const int per = (ga.total + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_adjoint96_group, dim3(xcd ? kXcds * per : ga.total), dim3(kThreads), 0,
                     s, ga, xcd);
  return hipGetLastError();
}

hipError_t launch_prepare96(const Dims& d, const float* frames, int H, int W, int stride,
                            const float* apod, float2* D, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const int nx = (W - N) / stride + 1;
  hipLaunchKernelGGL(k_prepare96, dim3(units), dim3(kThreads), 0, s, units, d.C, d.J, H, W,
                     stride, nx, frames, apod, D);
  return hipGetLastError();
}

hipError_t launch_objimg96(const Dims& d, const float2* O, float* obj, hipStream_t s) {
  const int items = d.P * d.K;
  hipLaunchKernelGGL(k_objimg96, dim3(items), dim3(kThreads), 0, s, items, items, 0, O, obj);
  return hipGetLastError();
}

hipError_t launch_frames96(int items, int per, int stride, const float2* D, float* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_objimg96, dim3(items), dim3(kThreads), 0, s, items, per, stride, D, out);
  return hipGetLastError();
}

hipError_t launch_synth96(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                          const float* noise, const float* sigma, float* field, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  hipLaunchKernelGGL(k_synth96, dim3(units), dim3(kThreads), 0, s, units, d.P, d.C, d.J, d.K, ct,
                     O, S, noise, sigma, field);
  return hipGetLastError();
}

}  // namespace mfbd
