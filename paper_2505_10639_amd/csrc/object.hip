// Wiener object and patch loss (Eqs. object_optimization and loss_momfbd),
// and the size dispatch of the unit kernels.
//
// Each (patch, object) plane of the half spectrum is cut into blocks of 256
// threads, each thread taking PPT pairs of adjacent frequencies (16-byte
// loads; PPT is a launch schedule the autotuner picks); every
// block leaves one FP64 partial of the loss, summed per patch in a fixed
// order by k_loss_sum.  One pass over D and S: N = sum w D conj(S),
// Q = gamma + sum w |S|^2 and E = sum w |D|^2 are accumulated in FP64, where
// the products of FP32 inputs are exact, so the loss term E - |N|^2/Q (the
// loss at the Wiener object, equal to the residual form
// sum w |D - O S|^2 + gamma |O|^2) keeps full accuracy.  On the half spectrum
// the columns 1..N/2-1 stand for two frequencies and count twice.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mfbd {

namespace {

// Block `blk` of a field: plane blk / kBlocks = (patch, object), part
// blk % kBlocks of that plane; its loss partial goes to loss_part[blk].
template <int NN, int PPT>
__device__ __forceinline__ void object_block(int blk, int C, int J, int K, const ChanTab& ct,
                                             const LossArgs& la,
                                             const int* __restrict__ active,
                                             const float2* __restrict__ S,
                                             float2* __restrict__ O,
                                             double* __restrict__ loss_part) {
  constexpr int kPairs = NN * (NN / 2 + 1) / 2;
  constexpr int kBlocks = object_blocks(NN, PPT);
  __shared__ double red[256];
  const int plane = blk / kBlocks, part = blk % kBlocks;
  const int p = plane / K, k = plane % K;
  if (active && !active[p]) return;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int e = 0; e < PPT; ++e) {
    const int f2 = (part * PPT + e) * 256 + tid;
    if (f2 >= kPairs) break;
    acc += object_pair<NN>(f2, p, k, C, J, K, ct, la, S, O);
  }
  red[tid] = acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (tid < s2) red[tid] += red[tid + s2];
    __syncthreads();
  }
  if (tid == 0) loss_part[blk] = red[0];
}

template <int NN, int PPT>
__global__ __launch_bounds__(256) void k_object(int P, int C, int J, int K, ChanTab ct,
                                                LossArgs la, const int* __restrict__ active,
                                                const float2* __restrict__ S,
                                                float2* __restrict__ O,
                                                double* __restrict__ loss_part) {
  // planes from the last patch to the first: the forward kernel has just
  // written S from the first unit to the last, so the most recently written
  // OTFs, the ones still held by the memory-side cache, are read first (and
  // the adjoint, walking forward, meets first the spectra read here last)
  object_block<NN, PPT>(gridDim.x - 1 - blockIdx.x, C, J, K, ct, la, active, S, O, loss_part);
}

// Every (patch, object) plane of every field of a group (one pair per thread).
template <int NN>
__global__ __launch_bounds__(256) void k_object_group(GroupArgs ga) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  object_block<NN, 1>(it.y, F.d.C, F.d.J, F.d.K, F.ct, F.la, F.active, F.w.S, F.w.O,
                      F.w.loss_pk);
}

// loss[p] = sum over objects and their blocks, in order (loss_sum_patch)
__global__ __launch_bounds__(256) void k_loss_sum(int P, int nper, const int* __restrict__ active,
                                                  const double* __restrict__ loss_part,
                                                  double* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  loss_sum_patch(p, nper, active, loss_part, loss);
}

// blocks of 256 patches of one field
__global__ __launch_bounds__(256) void k_loss_sum_group(GroupArgs ga, int nb) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  const int p = it.y * 256 + threadIdx.x;
  if (p >= F.d.P) return;
  loss_sum_patch(p, F.d.K * nb, F.active, F.w.loss_pk, F.loss);
}

// gamma_k(u) = gamma0_k + lambda_k (4 sin^2(pi u_x/N) + 4 sin^2(pi u_y/N)) on
// the half spectrum: the smoothness prior lambda_k ||grad o_k||^2 (periodic
// forward differences) written as a per-frequency Wiener constant.
__global__ __launch_bounds__(256) void k_smoothness(int N, int K, PriorTab t,
                                                    float* __restrict__ gamma) {
  const int HC = N / 2 + 1;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= K * N * HC) return;
  const int k = i / (N * HC), r = i % (N * HC);
  const int uy = r / HC, ux = r % HC;
  const double sy = sinpi((double)uy / N), sx = sinpi((double)ux / N);
  gamma[i] = (float)((double)t.gamma0[k] + (double)t.lambda[k] * 4.0 * (sy * sy + sx * sx));
}

}  // namespace

hipError_t launch_smoothness(int N, int K, const PriorTab& t, float* gamma, hipStream_t s) {
  const int n = K * N * (N / 2 + 1);
  hipLaunchKernelGGL(k_smoothness, dim3((n + 255) / 256), dim3(256), 0, s, N, K, t, gamma);
  return hipGetLastError();
}

template <int NN>
void launch_object_n(const Dims& d, const ChanTab& ct, const LossArgs& la, const int* active,
                     const float2* S, float2* O, double* loss_pk, hipStream_t s) {
  const int ppt = d.obj_ppt;
  const dim3 grid(d.P * d.K * object_blocks(NN, ppt));
  if (ppt == 4)
    hipLaunchKernelGGL((k_object<NN, 4>), grid, dim3(256), 0, s, d.P, d.C, d.J, d.K, ct, la,
                       active, S, O, loss_pk);
  else if (ppt == 2)
    hipLaunchKernelGGL((k_object<NN, 2>), grid, dim3(256), 0, s, d.P, d.C, d.J, d.K, ct, la,
                       active, S, O, loss_pk);
  else
    hipLaunchKernelGGL((k_object<NN, 1>), grid, dim3(256), 0, s, d.P, d.C, d.J, d.K, ct, la,
                       active, S, O, loss_pk);
}

LossSum loss_sum_of(const Dims& d, const int* active, const double* loss_pk, double* loss) {
  // the fused forward/object kernel leaves the partials of one pair per thread
  const int ppt = fused_object(d) ? 1 : d.obj_ppt;
  return LossSum{d.P, d.K * object_blocks(d.N, ppt), active, loss_pk, loss};
}

hipError_t launch_loss_sum(const LossSum& ls, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_sum, dim3((ls.P + 255) / 256), dim3(256), 0, s, ls.P, ls.nper,
                     ls.active, ls.loss_part, ls.loss);
  return hipGetLastError();
}

hipError_t launch_object(const Dims& d, const ChanTab& ct, const LossArgs& la, const int* active,
                         const float2* S, float2* O, double* loss_pk, double* loss,
                         hipStream_t s, bool sum_loss) {
  if (d.N == 64)
    launch_object_n<64>(d, ct, la, active, S, O, loss_pk, s);
  else if (d.N == 96)
    launch_object_n<96>(d, ct, la, active, S, O, loss_pk, s);
  else
    launch_object_n<128>(d, ct, la, active, S, O, loss_pk, s);
  if (!sum_loss) return hipGetLastError();
  return launch_loss_sum(loss_sum_of(d, active, loss_pk, loss), s);
}

hipError_t launch_object_group(int N, const GroupArgs& ga_blocks, const GroupArgs& ga_patches,
                               hipStream_t s) {
  const dim3 grid(ga_blocks.total);
  if (N == 64)
    hipLaunchKernelGGL(k_object_group<64>, grid, dim3(256), 0, s, ga_blocks);
  else if (N == 96)
    hipLaunchKernelGGL(k_object_group<96>, grid, dim3(256), 0, s, ga_blocks);
  else
    hipLaunchKernelGGL(k_object_group<128>, grid, dim3(256), 0, s, ga_blocks);
  hipLaunchKernelGGL(k_loss_sum_group, dim3(ga_patches.total), dim3(256), 0, s, ga_patches,
                     object_blocks(N, 1));
  return hipGetLastError();
}

hipError_t launch_forward_group(int N, const GroupArgs& ga, int xcd, hipStream_t s) {
  return N == 64   ? launch_forward64_group(ga, xcd, s)
         : N == 96 ? launch_forward96_group(ga, xcd, s)
                   : launch_forward128_group(ga, xcd, s);
}

hipError_t launch_adjoint_group(int N, const GroupArgs& ga, int xcd, hipStream_t s) {
  return N == 64   ? launch_adjoint64_group(ga, xcd, s)
         : N == 96 ? launch_adjoint96_group(ga, xcd, s)
                   : launch_adjoint128_group(ga, xcd, s);
}

hipError_t launch_forward(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                          const float* phi, float* psf, float2* S, hipStream_t s) {
  return d.N == 64   ? launch_forward64(d, ct, active, Ab, phi, psf, S, s)
         : d.N == 96 ? launch_forward96(d, ct, active, Ab, phi, psf, S, s)
                     : launch_forward128(d, ct, active, Ab, phi, psf, S, s);
}

hipError_t launch_adjoint(const Dims& d, const ChanTab& ct, const LossArgs& la, const int* active,
                          const float* Ab, const float* phi, const float2* S, const float2* O,
                          float* gphi, hipStream_t s) {
  return d.N == 64   ? launch_adjoint64(d, ct, la, active, Ab, phi, S, O, gphi, s)
         : d.N == 96 ? launch_adjoint96(d, ct, la, active, Ab, phi, S, O, gphi, s)
                     : launch_adjoint128(d, ct, la, active, Ab, phi, S, O, gphi, s);
}

hipError_t launch_prepare(const Dims& d, const float* frames, int H, int W, int stride,
                          const float* apod, float2* D, hipStream_t s) {
  return d.N == 64   ? launch_prepare64(d, frames, H, W, stride, apod, D, s)
         : d.N == 96 ? launch_prepare96(d, frames, H, W, stride, apod, D, s)
                     : launch_prepare128(d, frames, H, W, stride, apod, D, s);
}

hipError_t launch_frames(int N, int items, int per, int stride, const float2* D, float* out,
                         hipStream_t s) {
  return N == 64   ? launch_frames64(items, per, stride, D, out, s)
         : N == 96 ? launch_frames96(items, per, stride, D, out, s)
                   : launch_frames128(items, per, stride, D, out, s);
}

hipError_t launch_synth(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                        const float* noise, const float* sigma, float* field, hipStream_t s) {
  return d.N == 64   ? launch_synth64(d, ct, O, S, noise, sigma, field, s)
         : d.N == 96 ? launch_synth96(d, ct, O, S, noise, sigma, field, s)
                     : launch_synth128(d, ct, O, S, noise, sigma, field, s);
}

hipError_t launch_objimg(const Dims& d, const float2* O, float* obj, hipStream_t s) {
  return d.N == 64   ? launch_objimg64(d, O, obj, s)
         : d.N == 96 ? launch_objimg96(d, O, obj, s)
                     : launch_objimg128(d, O, obj, s);
}

}  // namespace mfbd
