// Unit kernels of the MOMFBD hot path for 64x64 patches (gfx950).
//
// One workgroup = one wavefront = one unit (patch p, channel c, frame j).
//   forward : phase -> pupil -> inverse 2-D DFT -> |.|^2 (unit-sum PSF)
//             -> forward 2-D DFT (OTF half spectrum)
//   fwdobj  : (a launch schedule) one workgroup of up to 12 waves per
//             (patch, object): the forward of its units, then the Wiener
//             object O_k = N_k / Q_k and the patch loss in FP64 with the
//             object kernel's own per-pair code (object.hip)
//   adjoint : G = conj(O)(D - O S) -> inverse DFT -> H = -4 w kappa g p
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

// Ordering of a unit's LDS exchanges: SYNC 0, the workgroup barrier (a
// one-wave workgroup); SYNC 1, for a unit that is one wave of a larger
// workgroup, the wave's own order only: a wave's LDS accesses complete in
// issue order, so fences at wavefront scope that keep the compiler from
// moving accesses across them are enough.
template <int SYNC>
__device__ __forceinline__ void unit_sync() {
  if constexpr (SYNC == 0) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remapping block b to unit (b mod 8) * per + b / 8 gives every XCD a
// contiguous run of units, so the frames of one patch-object (which share the
// object spectrum) meet in the same L2.  The grid has 8 * per blocks.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_unit(int per) {
  const int b = blockIdx.x;
  return (b % kXcds) * per + b / kXcds;
}
__host__ __device__ inline int xcd_per(int units) { return (units + kXcds - 1) / kXcds; }

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

// The two transposes go through a half-size buffer (real parts, then
// imaginary parts): 9.2 KB of LDS per wave lets a CU hold the 12 waves its
// registers allow, against 9 with the full-size buffer.
// Unit u of a field on the wave's LDS (Th, Taux); the OTF is stored to S and
// left in X (lane's values at sl_index) and x32 (at sl_index32).
template <bool WANT_PSF, int SYNC>
__device__ __forceinline__ void forward64_core(float2* Th, float2* Taux, int u, const ChanTab& ct,
                                               int C, int J, const int* __restrict__ active,
                                               const float* __restrict__ Ab,
                                               const float* __restrict__ phi,
                                               float* __restrict__ psf,
                                               float2* __restrict__ S, float2 (&X)[32],
                                               float2& x32) {
  float* Tf = reinterpret_cast<float*>(Th);
  if (active && !active[u / (J * C)]) return;
  const int lane = threadIdx.x & 63;
  const int c = (u / J) % C;
  float2 pe[32], po[32];
  {
    float2 y[32];
    // a wave that is issuing its loads runs at raised priority, so that
    // they go out ahead of the transform work of the waves beside it
    __builtin_amdgcn_s_setprio(2);
    build_pupil(Ab + c * kBandPix, phi + (size_t)u * kBandPix, lane, y);
    __builtin_amdgcn_s_setprio(0);
    fft32<+1>(y);
    op1_cols_put<0>(y, Tf, lane);
    unit_sync<SYNC>();
    op1_rows_get0(Tf, lane, pe);
    unit_sync<SYNC>();
    op1_cols_put<1>(y, Tf, lane);
  }
  unit_sync<SYNC>();
  op1_rows_get1(Tf, lane, pe, po);
  // half the PSF row (op2_rows_values takes s / 2; the factor is exact)
  const float kap_half = 0.5f * ct.kappa[c];
  float se[32], so[32];
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    se[n] = kap_half * cabs2(pe[n]);
    so[n] = kap_half * cabs2(po[n]);
  }
  if (WANT_PSF) {
    float* row = psf + (size_t)u * N * N + lane * N;
#pragma unroll
    for (int n = 0; n < 32; ++n) {
      row[2 * n] = 2.0f * se[n];
      row[2 * n + 1] = 2.0f * so[n];
    }
  }
  float2 v[32];
  op2_rows_values(se, so, v);
  unit_sync<SYNC>();
  op2_rows_put<0>(v, Tf, lane);
  unit_sync<SYNC>();
  op2_cols_get<0>(Tf, lane, X);
  unit_sync<SYNC>();
  op2_rows_put<1>(v, Tf, lane);
  unit_sync<SYNC>();
  op2_cols_get<1>(Tf, lane, X);
  op2_cols_finish(X, Taux, lane);
  unit_sync<SYNC>();
  x32 = op2_unpack(Taux, Th, lane);
  unit_sync<SYNC>();
  op2_collect(Th, lane, X);
  float2* out = S + (size_t)u * kUnitF2;
#pragma unroll
  for (int m = 0; m < 32; ++m) out[sl_index(lane, m)] = X[m];
  out[sl_index32(lane)] = x32;
}

// Unit u of a field (the kernel of one plan and the group kernel both
// resolve u, then run this).
template <bool WANT_PSF>
__device__ __forceinline__ void forward64_unit(int u, const ChanTab& ct, int C, int J,
                                               const int* __restrict__ active,
                                               const float* __restrict__ Ab,
                                               const float* __restrict__ phi,
                                               float* __restrict__ psf,
                                               float2* __restrict__ S) {
  __shared__ float2 Th[LDS_HALF / 2];
  __shared__ float2 Taux[LDS_AUX];
  float2 X[32], x32;
  forward64_core<WANT_PSF, 0>(Th, Taux, u, ct, C, J, active, Ab, phi, psf, S, X, x32);
}

template <bool WANT_PSF>
__global__ __launch_bounds__(64) void k_forward64(int units, int xcd, ChanTab ct, int C, int J,
                                                  const int* __restrict__ active,
                                                  const float* __restrict__ Ab,
                                                  const float* __restrict__ phi,
                                                  float* __restrict__ psf,
                                                  float2* __restrict__ S) {
  const int u = xcd ? xcd_unit(xcd_per(units)) : blockIdx.x;
  if (u >= units) return;
  forward64_unit<WANT_PSF>(u, ct, C, J, active, Ab, phi, psf, S);
}

// Every unit of every field of a group; the XCD order runs over the group's
// unit sequence (fields in order, each field's units in order).
__global__ __launch_bounds__(64) void k_forward64_group(GroupArgs ga, int xcd) {
  const int g = xcd ? xcd_unit(xcd_per(ga.total)) : blockIdx.x;
  if (g >= ga.total) return;
  const int2 it = ga.item[g];
  const FieldDesc& F = ga.fd[it.x];
  forward64_unit<false>(it.y, F.ct, F.d.C, F.d.J, F.active, F.Ab, F.w.phi, nullptr,
                        F.w.S);
}

// Forward and Wiener object of one (patch, object) plane per workgroup of
// kFusedWaves waves.  Wave w computes unit w of the plane (the object's
// channels in order, each channel's frames in order) and stores its OTF to
// S as k_forward64 does; after the barrier the workgroup's threads take the
// plane's frequency pairs as k_object<64, 1> does (blocks of 256 pairs, one
// pair per thread, the same per-pair code and the same tree sums of the loss
// terms), so that O and the loss partials equal those of the two separate
// launches bit for bit.  The OTFs it reads back were written by its own
// waves moments before and come from the caches, not HBM: per step S
// crosses HBM once less, and one launch is saved.  The workgroup holds
// 110.6 KB of LDS, so a CU runs one at a time: the 12 waves its registers
// allow the forward transforms in any case.  But every CU then alternates a
// transform phase and a memory phase in step with the others, and no second
// workgroup fills the gaps: measured no faster than the two launches, it is
// a launch schedule (object_fused), off by default.
constexpr int kWaveLds = LDS_HALF / 2 + LDS_AUX;   // float2 per wave (transforms)
constexpr int kObjParts = object_blocks(N, 1);     // 256-pair blocks of a plane
constexpr int kFusedThreads = 64 * kFusedWaves;
static_assert(kObjParts * 256 * sizeof(double) <= kFusedWaves * kWaveLds * sizeof(float2),
              "the loss terms of a plane fit the transforms' LDS");

__global__ __launch_bounds__(kFusedThreads) void k_fwdobj64(int K, ChanTab ct, int C, int J,
                                                            LossArgs la,
                                                            const int* __restrict__ active,
                                                            const float* __restrict__ Ab,
                                                            const float* __restrict__ phi,
                                                            float2* __restrict__ S,
                                                            float2* __restrict__ O,
                                                            double* __restrict__ loss_part) {
  __shared__ float2 lds[kFusedWaves * kWaveLds];
  const int plane = blockIdx.x, p = plane / K, k = plane % K;
  if (active && !active[p]) return;
  const int w = threadIdx.x >> 6;
  const int c0 = ct.obj_first[k];
  if (w < (ct.obj_first[k + 1] - c0) * J) {
    float2 X[32], x32;
    const int u = (p * C + ct.obj_chans[c0 + w / J]) * J + w % J;
    forward64_core<false, 1>(lds + w * kWaveLds, lds + w * kWaveLds + LDS_HALF / 2, u, ct, C,
                             J, nullptr, Ab, phi, nullptr, S, X, x32);
  }
  // every unit's S is written (visible to the workgroup after the barrier)
  // and the transforms are done with LDS
  __syncthreads();
  constexpr int kPairs = kUnitF2 / 2;
  double* red = reinterpret_cast<double*>(lds);
  for (int f2 = threadIdx.x; f2 < kObjParts * 256; f2 += kFusedThreads) {
    double acc = 0.0;
    if (f2 < kPairs) acc += object_pair<N>(f2, p, k, C, J, K, ct, la, S, O);
    red[f2] = acc;
  }
  __syncthreads();
  // the object kernel's sums over each block of 256 pairs, all blocks at once
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    for (int t = threadIdx.x; t < kObjParts * s2; t += kFusedThreads) {
      const int part = t / s2, i = t % s2;
      red[part * 256 + i] += red[part * 256 + i + s2];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < kObjParts)
    loss_part[(size_t)plane * kObjParts + threadIdx.x] = red[threadIdx.x * 256];
}

__device__ __forceinline__ void adjoint64_unit(int u, const ChanTab& ct, int C, int J, int K,
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
  const float2* Su = S + (size_t)u * kUnitF2;
  const float2* Du = la.D + (size_t)u * kUnitF2;
  const float2* Ok = O + ((size_t)p * K + k) * kUnitF2;
  const float* Ac = Ab + c * kBandPix;
  const float* phu = phi + (size_t)u * kBandPix;
  // the pupil band field (recomputed below to form p) depends only on phi:
  // build it first so that its loads overlap those of G
  // raised priority while the loads of phi, D, S and O are issued
  __builtin_amdgcn_s_setprio(2);
  float2 y[32];
  build_pupil(Ac, phu, lane, y);

  // G = conj(O) (D - O S) in spectral layout (the frame factor -2 w is
  // applied with 2 kappa after the inverse transform); zero outside the
  // object's spectral support, where D, S and O are not read
  constexpr int kOut = kUnitF2 * 8;
  const __amdgpu_buffer_rsrc_t rD = raw_buffer(Du, kOut), rS = raw_buffer(Su, kOut),
                               rO = raw_buffer(Ok, kOut);
  const int fm = la.supp[k * HC + (lane >> 1)];
  float2 G[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) {
    const int off = in_support(2 * m + (lane & 1), N, fm) ? sl_index(lane, m) * 8 : kOut;
    const float2 o = buffer_load_f2(rO, off);
    G[m] = cmul(cconj(o), csub(buffer_load_f2(rD, off), cmul(o, buffer_load_f2(rS, off))));
  }
  float2 g32;
  {
    const int off = in_support(lane, N, la.supp[k * HC + 32]) ? sl_index32(lane) * 8 : kOut;
    const float2 o = buffer_load_f2(rO, off);
    g32 = cmul(cconj(o), csub(buffer_load_f2(rD, off), cmul(o, buffer_load_f2(rS, off))));
  }
  __builtin_amdgcn_s_setprio(0);
  op3_gather(g32, Taux, lane);
  wave_sync();
  op3_cols(G, Taux, T, lane);
  wave_sync();
  float ge[32], go[32];
  op3_rows(T, lane, ge, go);
  wave_sync();

  // recompute the pupil band transform, then H = -4 w kappa g p and its
  // forward transform to the band, half a row spectrum at a time
  op1_cols(y, T, lane);
  wave_sync();
  float2 Gr[32];
  op14_rows(T, lane, ge, go, 2.0f * ct.kappa[c] * w2, Gr);   // w2: the frame's -2 w
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

__global__ __launch_bounds__(64) void k_adjoint64(int units, int xcd, ChanTab ct, int C, int J,
                                                  int K,
                                                  LossArgs la, const int* __restrict__ active,
                                                  const float* __restrict__ Ab,
                                                  const float* __restrict__ phi,
                                                  const float2* __restrict__ S,
                                                  const float2* __restrict__ O,
                                                  float* __restrict__ gphi) {
  const int u = xcd ? xcd_unit(xcd_per(units)) : blockIdx.x;
  if (u >= units) return;
  adjoint64_unit(u, ct, C, J, K, la, active, Ab, phi, S, O, gphi);
}

__global__ __launch_bounds__(64) void k_adjoint64_group(GroupArgs ga, int xcd) {
  const int g = xcd ? xcd_unit(xcd_per(ga.total)) : blockIdx.x;
  if (g >= ga.total) return;
  const int2 it = ga.item[g];
  const FieldDesc& F = ga.fd[it.x];
  adjoint64_unit(it.y, F.ct, F.d.C, F.d.J, F.d.K, F.la, F.active, F.Ab, F.w.phi,
                 F.w.S, F.w.O, F.w.gphi);
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
  const float2 x32 = op2_unpack(Taux, T, lane);
  wave_sync();
  op2_collect(T, lane, X);
  float2* out = D + (size_t)u * kUnitF2;
#pragma unroll
  for (int m = 0; m < 32; ++m) out[sl_index(lane, m)] = X[m];
  out[sl_index32(lane)] = x32;
}

// out = IDFT(A B) / N^2 + sg nz for one half spectrum A (times B when B is
// given; plus sg times the noise image nz when nz is given): the restored
// object image, or a synthetic frame.
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
  op3_gather(B ? cmul(A[sl_index32(lane)], B[sl_index32(lane)]) : A[sl_index32(lane)], Taux,
             lane);
  wave_sync();
  op3_cols(X, Taux, T, lane);
  wave_sync();
  float ge[32], go[32];
  op3_rows(T, lane, ge, go);
  float* row = out + lane * N;
  const float inv = 1.0f / (N * N);
  if (nz) {
    const float* nr = nz + lane * N;
#pragma unroll
    for (int n = 0; n < 32; ++n) {
      row[2 * n] = ge[n] * inv + sg * nr[2 * n];
      row[2 * n + 1] = go[n] * inv + sg * nr[2 * n + 1];
    }
  } else {
#pragma unroll
    for (int n = 0; n < 32; ++n) {
      row[2 * n] = ge[n] * inv;
      row[2 * n + 1] = go[n] * inv;
    }
  }
}

// Item it = (it / per, it % per) of spectra laid out with `stride` items
// between consecutive values of it / per (object images: per = items,
// stride 0; channel 0 of bursts [B][C][J]: per = J, stride = C J).
__global__ __launch_bounds__(64) void k_objimg64(int items, int per, int stride,
                                                 const float2* __restrict__ O,
                                                 float* __restrict__ obj) {
  const int it = blockIdx.x;
  if (it >= items) return;
  inverse_item(O + ((size_t)(it / per) * stride + it % per) * kUnitF2, nullptr,
               obj + (size_t)it * N * N, nullptr, 0.f);
}

// Synthetic frames: i = IDFT(O_k S_u) / N^2 + sigma_p n_u for unit u = (p, c, j),
// written to the field layout [C][J][P*N][N] that the prepare kernel reads
// with a patch grid of one column (stride N).
__global__ __launch_bounds__(64) void k_synth64(int units, int P, int C, int J, int K, ChanTab ct,
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

hipError_t launch_synth64(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                          const float* noise, const float* sigma, float* field, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  hipLaunchKernelGGL(k_synth64, dim3(units), dim3(64), 0, s, units, d.P, d.C, d.J, d.K, ct, O, S,
                     noise, sigma, field);
  return hipGetLastError();
}

hipError_t launch_forward64(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                            const float* phi, float* psf, float2* S, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const dim3 grid(d.xcd_fwd ? kXcds * xcd_per(units) : units);
  if (psf)
    hipLaunchKernelGGL(k_forward64<true>, grid, dim3(64), 0, s, units, d.xcd_fwd, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  else
    hipLaunchKernelGGL(k_forward64<false>, grid, dim3(64), 0, s, units, d.xcd_fwd, ct, d.C, d.J,
                       active, Ab, phi, psf, S);
  return hipGetLastError();
}

hipError_t launch_fwdobj64(const Dims& d, const ChanTab& ct, const LossArgs& la,
                           const int* active, const float* Ab, const float* phi, float2* S,
                           float2* O, double* loss_pk, hipStream_t s) {
  hipLaunchKernelGGL(k_fwdobj64, dim3(d.P * d.K), dim3(kFusedThreads), 0, s, d.K, ct, d.C, d.J,
                     la, active, Ab, phi, S, O, loss_pk);
  return hipGetLastError();
}

hipError_t launch_adjoint64(const Dims& d, const ChanTab& ct, const LossArgs& la,
                            const int* active, const float* Ab, const float* phi, const float2* S,
                            const float2* O, float* gphi, hipStream_t s) {
  const int units = d.P * d.C * d.J;
  const dim3 grid(d.xcd_adj ? kXcds * xcd_per(units) : units);
  hipLaunchKernelGGL(k_adjoint64, grid, dim3(64), 0, s, units, d.xcd_adj, ct, d.C, d.J, d.K, la,
                     active, Ab, phi, S, O, gphi);
  return hipGetLastError();
}

hipError_t launch_forward64_group(const GroupArgs& ga, int xcd, hipStream_t s) {
  const dim3 grid(xcd ? kXcds * xcd_per(ga.total) : ga.total);
  hipLaunchKernelGGL(k_forward64_group, grid, dim3(64), 0, s, ga, xcd);
  return hipGetLastError();
}

hipError_t launch_adjoint64_group(const GroupArgs& ga, int xcd, hipStream_t s) {
  const dim3 grid(xcd ? kXcds * xcd_per(ga.total) : ga.total);
  hipLaunchKernelGGL(k_adjoint64_group, grid, dim3(64), 0, s, ga, xcd);
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
  hipLaunchKernelGGL(k_objimg64, dim3(items), dim3(64), 0, s, items, items, 0, O, obj);
  return hipGetLastError();
}

hipError_t launch_frames64(int items, int per, int stride, const float2* D, float* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_objimg64, dim3(items), dim3(64), 0, s, items, per, stride, D, out);
  return hipGetLastError();
}

}  // namespace mfbd
