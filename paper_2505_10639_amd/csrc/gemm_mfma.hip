// Dense modal contractions of one plan on the matrix cores: the kernels and
// their launchers (bodies and operand layout in contract_mfma.h).
#include <hip/hip_runtime.h>

#include "contract_mfma.h"
#include "internal.h"

namespace mfbd {
namespace {

using contract::floatx4;
using contract::kCols;

template <int MT, int RT, int W, int CS>
__global__ __launch_bounds__(64 * W) void k_grad_mfma(int R, int J, int C, int zc, int M, int bp,
                                                      const uint4* __restrict__ Zs,
                                                      const float* __restrict__ gphi,
                                                      float* __restrict__ grad,
                                                      float* __restrict__ part) {
  contract::grad_block<MT, RT, W, CS>(blockIdx.x, blockIdx.y, gridDim.y, MT, R, J, C, zc, M, bp,
                                      Zs, gphi, grad, part);
}

__global__ __launch_bounds__(256) void k_phase_mfma(int R, int J, int C, int zc, int M, int Mq,
                                                    int bp,
                                                    const uint4* __restrict__ ZsT,
                                                    const float* __restrict__ theta,
                                                    const float* __restrict__ alpha,
                                                    float* __restrict__ phi) {
  contract::phase_block(blockIdx.x, blockIdx.y, R, J, C, zc, M, Mq, bp, ZsT, theta, alpha, phi);
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

template <int MT, int CS>
void launch_grad_cs(const Dims& d, int zc, int splits, const uint4* Zs, const float* gphi,
                    float* grad, float* part, hipStream_t s) {
  const int R = d.P * d.J;
  if (d.grad_waves == 8)
    hipLaunchKernelGGL((k_grad_mfma<MT, 2, 8, CS>), dim3((R + 31) / 32, splits), dim3(512), 0,
                       s, R, d.J, d.C, zc, d.M, d.bandpix(), Zs, gphi, grad, part);
  else if (grad_row_tiles_of(d) == 3)
    hipLaunchKernelGGL((k_grad_mfma<MT, 3, 4, CS>), dim3((R + 47) / 48, splits), dim3(256), 0,
                       s, R, d.J, d.C, zc, d.M, d.bandpix(), Zs, gphi, grad, part);
  else
    hipLaunchKernelGGL((k_grad_mfma<MT, 4, 4, CS>), dim3((R + 63) / 64, splits), dim3(256), 0,
                       s, R, d.J, d.C, zc, d.M, d.bandpix(), Zs, gphi, grad, part);
}

template <int MT>
void launch_grad_t(const Dims& d, int splits, const uint4* Ztp, const float* gphi, float* grad,
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

hipError_t launch_grad(const Dims& d, const uint4* Zt, const float* gphi, float* grad,
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

hipError_t launch_phase(const Dims& d, const float* alpha, const uint4* ZsT, int Mq,
                        const float* thetat, float* phi, hipStream_t s) {
  const int R = d.P * d.J, zc = d.zc > 0 ? d.zc : d.C;
  dim3 grid(zc * 4, (R + kCols - 1) / kCols);
  const size_t lds = (size_t)kCols * contract::phase_lds_stride(Mq) * sizeof(uint4);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_phase_mfma),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_phase_mfma, grid, dim3(256), lds, s, R, d.J, d.C, zc, d.M, Mq, d.bandpix(),
                     ZsT, thetat, alpha, phi);
  return hipGetLastError();
}

}  // namespace mfbd
