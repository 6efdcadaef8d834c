// Dense modal contractions for a group of fields (all of one patch size):
// one launch covers the phase tiles, or the gradient row tiles, of every
// field, each block finding its field from the stage's prefix sums.  The
// bodies are those of the single-plan kernels (contract_mfma.h); fields with
// fewer modes than the group's largest skip the mode tiles they lack.
#include <hip/hip_runtime.h>

#include "contract_mfma.h"
#include "internal.h"

namespace mfbd {
namespace {


__device__ __forceinline__ int zc_of(const Dims& d) { return d.zc > 0 ? d.zc : d.C; }

// grid (4 * largest zc, phase tiles of all fields)
__global__ __launch_bounds__(64 * kPhaseWaves) void k_phase_group(GroupArgs ga) {
  const int2 it = ga.item[blockIdx.y];
  const FieldDesc& F = ga.fd[it.x];
  const int zc = zc_of(F.d);
  if ((int)blockIdx.x >= 4 * zc) return;
  contract::phase_block<kPhaseCols / 16, kPhaseWaves>(blockIdx.x, it.y, F.d.P * F.d.J, F.d.J, F.d.C, zc,
                                        F.d.M, F.Mq, F.d.bandpix(), F.ZsT, F.thetat, F.alpha,
                                        F.w.phi);
}

// grid (row blocks of all fields, splits); W = 4 waves, RT row tiles each
template <int MT, int RT>
__global__ __launch_bounds__(256) void k_grad_group(GroupArgs ga) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  contract::grad_block<MT, RT, 4, -1>(it.y, blockIdx.y, gridDim.y, (F.d.M + 15) / 16,
                                      F.d.P * F.d.J, F.d.J, F.d.C, zc_of(F.d), F.d.M,
                                      F.d.bandpix(), F.Zs, F.w.gphi, F.grad, F.w.gpart);
}

// grad = 2 pi (part[0] + ... + part[splits-1]) per field, in split order;
// blocks of 256 coefficients of one field
__global__ __launch_bounds__(256) void k_grad_combine_group(GroupArgs ga, int splits) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  const long n = (long)F.d.P * F.d.J * F.d.M, i = (long)it.y * 256 + threadIdx.x;
  if (i >= n) return;
  float v = F.w.gpart[i];
  for (int s = 1; s < splits; ++s) v += F.w.gpart[(size_t)s * n + i];
  F.grad[i] = 6.283185307179586f * v;
}

template <int MT, int RT>
hipError_t launch_grad_group_rt(const GroupArgs& ga, int splits, hipStream_t s) {
  const size_t lds = contract::grad_lds_bytes(MT);
  if (lds > 65536) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grad_group<MT, RT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grad_group<MT, RT>), dim3(ga.total, splits), dim3(256), lds, s, ga);
  return hipGetLastError();
}

template <int MT>
hipError_t launch_grad_group_t(const GroupArgs& ga, int row_tiles, int splits, hipStream_t s) {
  if (row_tiles == 3) return launch_grad_group_rt<MT, 3>(ga, splits, s);
  if (row_tiles == 2) return launch_grad_group_rt<MT, 2>(ga, splits, s);
  return launch_grad_group_rt<MT, 4>(ga, splits, s);
}

}  // namespace

hipError_t launch_phase_group(const GroupArgs& ga, int zc_max, int Mq_max, hipStream_t s) {
  const size_t lds = contract::phase_lds_bytes(kPhaseCols / 16, Mq_max);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_phase_group),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_phase_group, dim3(4 * zc_max, ga.total), dim3(64 * kPhaseWaves), lds, s,
                     ga);
  return hipGetLastError();
}

// ga_tiles: row blocks of 64 * row_tiles rows per field; ga_elems: blocks of
// 256 of the P J M coefficients per field
hipError_t launch_grad_group(const GroupArgs& ga_tiles, const GroupArgs& ga_elems, int mt_max,
                             int row_tiles, int splits, hipStream_t s) {
  hipError_t e;
  switch (mt_max) {
#define MFBD_CASE(n) \
  case n: e = launch_grad_group_t<n>(ga_tiles, row_tiles, splits, s); break;
    MFBD_CASE(1) MFBD_CASE(2) MFBD_CASE(3) MFBD_CASE(4) MFBD_CASE(5) MFBD_CASE(6)
    MFBD_CASE(7) MFBD_CASE(8) MFBD_CASE(9) MFBD_CASE(10) MFBD_CASE(11) MFBD_CASE(12)
    MFBD_CASE(13) MFBD_CASE(14) MFBD_CASE(15) MFBD_CASE(16)
#undef MFBD_CASE
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (splits > 1)
    hipLaunchKernelGGL(k_grad_combine_group, dim3(ga_elems.total), dim3(256), 0, s, ga_elems,
                       splits);
  return hipGetLastError();
}

}  // namespace mfbd
