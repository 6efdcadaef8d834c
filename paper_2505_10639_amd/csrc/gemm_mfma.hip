// Dense modal contractions of one plan on the matrix cores: the kernels and
// their launchers (bodies and operand layout in contract_mfma.h).
#include <hip/hip_runtime.h>

#include "contract_mfma.h"
#include "internal.h"

namespace mfbd {
namespace {

using contract::floatx4;

template <int MT, int RT, int W, int CS>
__global__ __launch_bounds__(64 * W) void k_grad_mfma(int R, int J, int C, int zc, int M, int bp,
                                                      const uint4* __restrict__ Zs,
                                                      const float* __restrict__ gphi,
                                                      float* __restrict__ grad,
                                                      float* __restrict__ part) {
  contract::grad_block<MT, RT, W, CS>(blockIdx.x, blockIdx.y, gridDim.y, MT, R, J, C, zc, M, bp,
                                      Zs, gphi, grad, part);
}

template <int CT, int W>
__global__ __launch_bounds__(64 * W) void k_phase_mfma(int R, int J, int C, int zc, int M, int Mq,
                                                    int bp,
                                                    const uint4* __restrict__ ZsT,
                                                    const float* __restrict__ theta,
                                                    const float* __restrict__ alpha,
                                                    float* __restrict__ phi) {
  contract::phase_block<CT, W>(blockIdx.x, blockIdx.y, R, J, C, zc, M, Mq, bp, ZsT, theta,
                               alpha, phi);
}

// Dynamic LDS beyond the default 64 KB needs the kernel's attribute.
hipError_t allow_lds(const void* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// grad = 2 pi (part[0] + part[1] + ... + part[splits-1]), in that order;
// the blocks past the gradient's (`cblocks`) sum the per-patch loss when the
// call asks for it (ls.P > 0), saving that sum a launch of its own.
__global__ __launch_bounds__(256) void k_grad_combine(long n, int splits, int cblocks,
                                                      const float* __restrict__ part,
                                                      float* __restrict__ grad, LossSum ls) {
  if ((int)blockIdx.x >= cblocks) {
    const int p = ((int)blockIdx.x - cblocks) * 256 + threadIdx.x;
    if (p < ls.P) loss_sum_patch(p, ls.nper, ls.active, ls.loss_part, ls.loss);
    return;
  }
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float v = part[i];
  for (int s = 1; s < splits; ++s) v += part[(size_t)s * n + i];
  grad[i] = 6.283185307179586f * v;
}

template <int MT, int RT, int W, int CS>
hipError_t launch_grad_k(const Dims& d, int zc, int splits, const uint4* Zs, const float* gphi,
                         float* grad, float* part, hipStream_t s) {
  const int R = d.P * d.J, rows = 16 * RT * W;
  const size_t lds = contract::grad_lds_bytes(MT);
  const hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_grad_mfma<MT, RT, W, CS>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_grad_mfma<MT, RT, W, CS>), dim3((R + rows - 1) / rows, splits),
                     dim3(64 * W), lds, s, R, d.J, d.C, zc, d.M, d.bandpix(), Zs, gphi, grad,
                     part);
  return hipGetLastError();
}

template <int MT, int CS>
hipError_t launch_grad_cs(const Dims& d, int zc, int splits, const uint4* Zs, const float* gphi,
                          float* grad, float* part, hipStream_t s) {
  if (d.grad_waves == 8) return launch_grad_k<MT, 2, 8, CS>(d, zc, splits, Zs, gphi, grad, part, s);
  switch (grad_row_tiles_of(d)) {
    case 2: return launch_grad_k<MT, 2, 4, CS>(d, zc, splits, Zs, gphi, grad, part, s);
    case 3: return launch_grad_k<MT, 3, 4, CS>(d, zc, splits, Zs, gphi, grad, part, s);
    default: return launch_grad_k<MT, 4, 4, CS>(d, zc, splits, Zs, gphi, grad, part, s);
  }
}

template <int MT>
hipError_t launch_grad_t(const Dims& d, int splits, const uint4* Zs, const float* gphi,
                         float* grad, float* part, hipStream_t s) {
  const int zc = d.zc > 0 ? d.zc : d.C;
  if (zc == d.C) return launch_grad_cs<MT, 1>(d, zc, splits, Zs, gphi, grad, part, s);
  if (d.C == 2) return launch_grad_cs<MT, 2>(d, zc, splits, Zs, gphi, grad, part, s);
  return launch_grad_cs<MT, 0>(d, zc, splits, Zs, gphi, grad, part, s);
}

}  // namespace

int grad_splits_auto(const Dims& d) {
  // Enough workgroups for two per CU (512), as long as every split keeps at
  // least 8 chunks of 32 pixels to pipeline through its LDS stages.
  const int R = d.P * d.J, W = d.grad_waves == 8 ? 8 : 4;
  const long rows = 16L * grad_row_tiles_of(d) * W;
  const long blocks = (R + rows - 1) / rows;
  const int zc = d.zc > 0 ? d.zc : d.C;
  const int nchunk = zc * d.bandpix() / 32;
  int s = 1;
  while (s < kMaxGradSplits && blocks * s < 512 && nchunk / (2 * s) >= 8) s *= 2;
  return s;
}

int grad_splits_of(const Dims& d) { return d.grad_splits > 0 ? d.grad_splits : grad_splits_auto(d); }

int grad_row_tiles_of(const Dims& d) {
  return d.grad_waves == 8 ? 2 : (d.grad_rt == 3 || d.grad_rt == 2) ? d.grad_rt : 4;
}

hipError_t launch_grad(const Dims& d, const uint4* Zs, const float* gphi, float* grad,
                       float* part, hipStream_t s, const LossSum* ls) {
  const int mt = (d.M + 15) / 16;
  const int splits = grad_splits_of(d);
  hipError_t e;
  switch (mt) {
#define MFBD_CASE(n) \
  case n: e = launch_grad_t<n>(d, splits, Zs, gphi, grad, part, s); break;
    MFBD_CASE(1) MFBD_CASE(2) MFBD_CASE(3) MFBD_CASE(4) MFBD_CASE(5) MFBD_CASE(6)
    MFBD_CASE(7) MFBD_CASE(8) MFBD_CASE(9) MFBD_CASE(10) MFBD_CASE(11) MFBD_CASE(12)
    MFBD_CASE(13) MFBD_CASE(14) MFBD_CASE(15) MFBD_CASE(16)
#undef MFBD_CASE
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (splits > 1) {
    const long n = (long)d.P * d.J * d.M;
    const int cblocks = (int)((n + 255) / 256);
    const LossSum none{0, 0, nullptr, nullptr, nullptr};
    const LossSum& l = ls ? *ls : none;
    hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)(cblocks + (l.P + 255) / 256)), dim3(256),
                       0, s, n, splits, cblocks, part, grad, l);
    return hipGetLastError();
  }
  if (ls) return launch_loss_sum(*ls, s);
  return hipGetLastError();
}

// Phase blocks.  Automatic shape: 128 columns and 8 waves when the staged
// coefficients fit 128 KB of LDS, else 64 columns (4 waves) within 64 KB,
// else 32.  Every basis part read serves all the block's columns, so the
// widest block that fits reads the basis least often.  A plan may select
// 64 columns with 8 waves (two blocks per CU where their LDS allows) or
// 128 columns with 16 waves (more waves issuing matrix-core work per CU).
template <int CT, int W>
hipError_t launch_phase_ct(const Dims& d, const float* alpha, const uint4* ZsT, int Mq,
                           const float* thetat, float* phi, hipStream_t s) {
  const int R = d.P * d.J, zc = d.zc > 0 ? d.zc : d.C;
  const dim3 grid(zc * 4, (R + 16 * CT - 1) / (16 * CT));
  const size_t lds = contract::phase_lds_bytes(CT, Mq);
  const hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_phase_mfma<CT, W>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_phase_mfma<CT, W>), grid, dim3(64 * W), lds, s, R, d.J, d.C, zc, d.M, Mq,
                     d.bandpix(), ZsT, thetat, alpha, phi);
  return hipGetLastError();
}

bool phase_shape_fits(int ct, int waves, int Mq) {
  const bool listed = (ct == 8 && waves == 8) || (ct == 4 && waves == 8) || (ct == 8 && waves == 16);
  return listed && contract::phase_lds_bytes(ct, Mq) <= 128 * 1024;
}

void phase_shape_of(const Dims& d, int Mq, int* ct, int* waves) {
  if (d.phase_ct > 0 && phase_shape_fits(d.phase_ct, d.phase_waves, Mq)) {
    *ct = d.phase_ct;
    *waves = d.phase_waves;
  } else if (contract::phase_lds_bytes(8, Mq) <= 128 * 1024) {
    *ct = 8;
    *waves = 8;
  } else if (contract::phase_lds_bytes(4, Mq) <= 64 * 1024) {
    *ct = 4;
    *waves = 4;
  } else {
    *ct = 2;
    *waves = 4;
  }
}

hipError_t launch_phase(const Dims& d, const float* alpha, const uint4* ZsT, int Mq,
                        const float* thetat, float* phi, hipStream_t s) {
  int ct = 0, w = 0;
  phase_shape_of(d, Mq, &ct, &w);
  if (ct == 8 && w == 16) return launch_phase_ct<8, 16>(d, alpha, ZsT, Mq, thetat, phi, s);
  if (ct == 8) return launch_phase_ct<8, 8>(d, alpha, ZsT, Mq, thetat, phi, s);
  if (ct == 4 && w == 8) return launch_phase_ct<4, 8>(d, alpha, ZsT, Mq, thetat, phi, s);
  if (ct == 4) return launch_phase_ct<4, 4>(d, alpha, ZsT, Mq, thetat, phi, s);
  return launch_phase_ct<2, 4>(d, alpha, ZsT, Mq, thetat, phi, s);
}

}  // namespace mfbd
