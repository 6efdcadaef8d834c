// Power spectrum of a restored (mosaicked) image and its average over
// 30-degree sectors along the +-45 degree directions, as a function of the
// radial frequency (Sect. "Results": averaging over all angles would pick up
// the power that the periodic continuation of the field puts on the axes).
//
//   P(u) = |DFT(w (x - mean))|^2 on the L x L grid, L a power of two;
//   bin k = round(|u|), u in (-L/2, L/2]; sector: 30..60 degrees from the
//   axes in every quadrant.  Both decisions are integer tests:
//   (2k-1)^2 <= 4|u|^2 < (2k+1)^2 and u_x^2 <= 3 u_y^2, u_y^2 <= 3 u_x^2.
//
// The 2-D transform is two passes of radix-2 Stockham FFTs of whole rows in
// LDS (natural order, twiddles from sincospi), each pass writing its output
// transposed.  Every sum runs in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "momfbd.h"

namespace mfbd {
namespace {

// The image mean in two passes: kMeanBlocks contiguous chunks, each summed
// by one block (strided per thread, then a tree), and the chunk sums by one
// block; every sum in a fixed order.
constexpr int kMeanBlocks = 256;
__device__ __forceinline__ double block_sum256(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void k_mean_part(long n, const float* __restrict__ x,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  const long chunk = (n + kMeanBlocks - 1) / kMeanBlocks;
  const long lo = (long)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) s += (double)x[i];
  const double tot = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_mean_final(long n, const double* __restrict__ part,
                                                    double* __restrict__ mean) {
  __shared__ double red[256];
  const double tot = block_sum256(part[threadIdx.x], red);
  if (threadIdx.x == 0) *mean = tot / (double)n;
}

// One row per block: FFT of length L in LDS, written transposed
// (out[c][row]).  First pass: real input w (x - mean); second pass: complex
// input, output |X|^2.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_fft_rows(int L, const float* __restrict__ x,
                                                  const float* __restrict__ win,
                                                  const double* __restrict__ mean,
                                                  const float2* __restrict__ cin,
                                                  float2* __restrict__ cout,
                                                  float* __restrict__ pout) {
  extern __shared__ float2 buf[];
  float2* a = buf;
  float2* b = buf + L;
  const int row = blockIdx.x, t = threadIdx.x;
  if (FIRST) {
    const float m = (float)*mean;
    for (int i = t; i < L; i += 256) {
      const long g = (long)row * L + i;
      const float w = win ? win[g] : 1.f;
      a[i] = make_float2(w * (x[g] - m), 0.f);
    }
  } else {
    for (int i = t; i < L; i += 256) a[i] = cin[(long)row * L + i];
  }
  __syncthreads();
  const int half = L / 2;
  for (int ns = 1; ns < L; ns *= 2) {
    for (int j = t; j < half; j += 256) {
      const float2 v0 = a[j], u1 = a[j + half];
      const int r = j % ns;
      float sn, cs;
      sincospif(-(float)r / (float)ns, &sn, &cs);
      const float2 v1 = make_float2(u1.x * cs - u1.y * sn, u1.x * sn + u1.y * cs);
      const int d = (j / ns) * ns * 2 + r;
      b[d] = make_float2(v0.x + v1.x, v0.y + v1.y);
      b[d + ns] = make_float2(v0.x - v1.x, v0.y - v1.y);
    }
    __syncthreads();
    float2* tmp = a;
    a = b;
    b = tmp;
  }
  for (int c = t; c < L; c += 256) {
    const float2 v = a[c];
    if (FIRST)
      cout[(long)c * L + row] = v;
    else
      pout[(long)c * L + row] = v.x * v.x + v.y * v.y;
  }
}

// Per row u_y and bin k: the sum and count of P over the sector members.
__global__ __launch_bounds__(256) void k_sector_rows(int L, int nbins,
                                                     const float* __restrict__ P,
                                                     double* __restrict__ rsum,
                                                     int* __restrict__ rcnt) {
  const int y = blockIdx.x;
  const long uy = y > L / 2 ? y - L : y;
  const long base = 4 * uy * uy;
  for (int k = threadIdx.x; k < nbins; k += 256) {
    // bin k holds (2k-1)^2 <= 4|u|^2 < (2k+1)^2 (bin 0: u = 0 only)
    const long lo = k == 0 ? -1 : (2L * k - 1) * (2L * k - 1) - base;   // 4 ux^2 >= lo
    const long hi = (2L * k + 1) * (2L * k + 1) - base;   // 4 ux^2 <  hi
    double s = 0.0;
    int cnt = 0;
    if (hi > 0) {
      long a = lo <= 0 ? 0 : (long)ceil(sqrt((double)lo / 4.0));
      while (a > 0 && 4 * (a - 1) * (a - 1) >= lo) --a;
      while (4 * a * a < lo) ++a;
      long bnd = (long)floor(sqrt((double)(hi - 1) / 4.0));
      while (4 * (bnd + 1) * (bnd + 1) < hi) ++bnd;
      while (bnd >= 0 && 4 * bnd * bnd >= hi) --bnd;
      for (long ux = a; ux <= bnd; ++ux) {
        for (int sg = 0; sg < 2; ++sg) {
          if (sg == 1 && ux == 0) continue;
          const long v = sg ? -ux : ux;
          if (v > L / 2 || v <= -L / 2) continue;
          if (v == 0 || uy == 0 || v * v > 3 * uy * uy || uy * uy > 3 * v * v) continue;
          s += (double)P[(long)y * L + (v >= 0 ? v : v + L)];
          ++cnt;
        }
      }
    }
    rsum[(long)y * nbins + k] = s;
    rcnt[(long)y * nbins + k] = cnt;
  }
}

// One block per bin: the per-row sums and counts of the bin over all rows
// (strided per thread, then a tree).
__global__ __launch_bounds__(256) void k_sector_bins(int L, int nbins,
                                                     const double* __restrict__ rsum,
                                                     const int* __restrict__ rcnt,
                                                     double* __restrict__ out,
                                                     int* __restrict__ counts) {
  __shared__ double red[256];
  __shared__ long redc[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  long c = 0;
  for (int y = t; y < L; y += 256) {
    s += rsum[(long)y * nbins + k];
    c += rcnt[(long)y * nbins + k];
  }
  redc[t] = c;
  const double tot = block_sum256(s, red);   // its barriers also order redc
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) redc[t] += redc[t + h];
    __syncthreads();
  }
  if (t == 0) {
    out[k] = redc[0] > 0 ? tot / (double)redc[0] : 0.0;
    if (counts) counts[k] = (int)redc[0];
  }
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

bool pow2(int L) { return L >= 16 && L <= 4096 && (L & (L - 1)) == 0; }

}  // namespace
}  // namespace mfbd

using namespace mfbd;

extern "C" {

int momfbd_power_spectrum_workspace(int L, int nbins, size_t* bytes) {
  if (!bytes || !pow2(L) || nbins < 1 || nbins > L) return MOMFBD_EINVAL;
  *bytes = al256((kMeanBlocks + 1) * sizeof(double)) + al256((size_t)L * L * sizeof(float2)) +
           al256((size_t)L * nbins * sizeof(double)) + al256((size_t)L * nbins * sizeof(int));
  return MOMFBD_OK;
}

int momfbd_power_spectrum(int L, const float* image, const float* window, float* power,
                          double* sector, int* counts, int nbins, void* ws, size_t ws_bytes,
                          void* stream) {
  size_t need = 0;
  int st = momfbd_power_spectrum_workspace(L, nbins, &need);
  if (st) return st;
  if (!image || !power) return MOMFBD_EINVAL;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 || ws_bytes < need) return MOMFBD_EWORKSPACE;
  if (hipGetLastError() != hipSuccess) return MOMFBD_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  double* mean = reinterpret_cast<double*>(w);
  double* mean_part = mean + 1;
  size_t o = al256((kMeanBlocks + 1) * sizeof(double));
  float2* T = reinterpret_cast<float2*>(w + o);
  o += al256((size_t)L * L * sizeof(float2));
  double* rsum = reinterpret_cast<double*>(w + o);
  o += al256((size_t)L * nbins * sizeof(double));
  int* rcnt = reinterpret_cast<int*>(w + o);
  const size_t lds = 2 * (size_t)L * sizeof(float2);
  if (lds > 65536) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_rows<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_rows<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return MOMFBD_EDEVICE;
  }
  hipLaunchKernelGGL(k_mean_part, dim3(kMeanBlocks), dim3(256), 0, s, (long)L * L, image,
                     mean_part);
  hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(256), 0, s, (long)L * L, mean_part, mean);
  hipLaunchKernelGGL(k_fft_rows<true>, dim3(L), dim3(256), lds, s, L, image, window, mean,
                     nullptr, T, nullptr);
  hipLaunchKernelGGL(k_fft_rows<false>, dim3(L), dim3(256), lds, s, L, nullptr, nullptr, nullptr,
                     T, nullptr, power);
  if (sector) {
    hipLaunchKernelGGL(k_sector_rows, dim3(L), dim3(256), 0, s, L, nbins, power, rsum, rcnt);
    hipLaunchKernelGGL(k_sector_bins, dim3(nbins), dim3(256), 0, s, L, nbins, rsum, rcnt, sector,
                       counts);
  }
  return hipGetLastError() == hipSuccess ? MOMFBD_OK : MOMFBD_EDEVICE;
}

}  // extern "C"
