// Post-processing of the restored objects.
//
//   filter : the Fourier filters of Sect. "Fourier filtering" applied to the
//            Wiener object spectrum O_k of every (patch, object):
//            top-hat with a cosine transition between f_l and f_u (units of
//            the diffraction-limit frequency), or the Loefdahl-Scharmer
//            filter H = 1 - eta sum w|S|^2 / |sum w D conj(S)|^2 (eta the
//            noise power per frequency of a frame; the printed ratio is
//            eta = 1) clipped (H < 0.2 -> 0, H > 1 -> 1), 3x3 median on the
//            periodic frequency grid, and restricted to the region
//            4-connected to the zero frequency.
//   mosaic : sum_p w o_p / sum_p w over the patches covering each pixel, with
//            the separable cosine taper w of Sect. "Division in patches and
//            apodization".
//
// The filter works on the full N x N grid in LDS (H is symmetric under
// u -> -u, so the half spectrum reads suffice); the island search is a
// label propagation from the origin repeated until no label changes (at
// N = 64 on one 64-bit word per row, in one wave).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mfbd {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline float tophat_value(int uy, int ux, int N, const FilterSpec& f) {
  const int sy = uy > N / 2 ? uy - N : uy, sx = ux > N / 2 ? ux - N : ux;
  const double r = sqrt((double)(sy * sy + sx * sx)) / (double)f.diff_limit;
  if (r <= (double)f.f_lo) return 1.f;
  if (r >= (double)f.f_hi) return 0.f;
  return (float)(0.5 * (1.0 + cos(kPi * (r - (double)f.f_lo) / ((double)f.f_hi - (double)f.f_lo))));
}

// The median of nine values without branches: sort each of the three
// triples, then the median of (largest low, median middle, smallest high)
// is the median of all nine; it is one of the inputs, so it is exact.
__device__ inline float med3(float a, float b, float c) {
  return fmaxf(fminf(a, b), fminf(fmaxf(a, b), c));
}
__device__ inline float median9(const float v[9]) {
  float lo[3], mi[3], hi[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const float a = v[3 * t], b = v[3 * t + 1], c = v[3 * t + 2];
    const float l = fminf(a, b), h = fmaxf(a, b);
    lo[t] = fminf(l, c);
    mi[t] = fmaxf(l, fminf(h, c));
    hi[t] = fmaxf(h, c);
  }
  return med3(fmaxf(fmaxf(lo[0], lo[1]), lo[2]), med3(mi[0], mi[1], mi[2]),
              fminf(fminf(hi[0], hi[1]), hi[2]));
}

// Cells of m reachable from x by steps toward higher (up) or lower (down)
// bits through m: a doubling fill, six shifts for any run length.
__device__ inline unsigned long long fill_up(unsigned long long x, unsigned long long m) {
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    x |= m & (x << s);
    m &= m << s;
  }
  return x;
}
__device__ inline unsigned long long fill_down(unsigned long long x, unsigned long long m) {
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    x |= m & (x >> s);
    m &= m >> s;
  }
  return x;
}
__device__ inline unsigned long long shfl64(unsigned long long v, int lane) {
  const int lo = __shfl(static_cast<int>(v & 0xffffffffull), lane);
  const int hi = __shfl(static_cast<int>(v >> 32), lane);
  return (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
         static_cast<unsigned>(lo);
}

template <int NN>
__global__ __launch_bounds__(256) void k_filter(int C, int J, int K, ChanTab ct, FilterTab ft,
                                                const float2* __restrict__ D,
                                                const float* __restrict__ weights,
                                                const float2* __restrict__ S,
                                                float2* __restrict__ O, float* __restrict__ Hout) {
  constexpr int HC = NN / 2 + 1, UNIT = NN * HC, GRID = NN * NN;
  extern __shared__ float lds[];
  float* A = lds;          // clipped H, then the labels
  float* B = lds + GRID;   // median-filtered H
  __shared__ int changed;
  const int tid = threadIdx.x;
  const int p = blockIdx.x / K, k = blockIdx.x % K;
  const FilterSpec f = ft.f[k];
  float2* Ok = O + ((size_t)p * K + k) * UNIT;
  float* Hk = Hout ? Hout + ((size_t)p * K + k) * UNIT : nullptr;
  if (f.kind != kFilterScharmer) {
    for (int i = tid; i < UNIT; i += 256) {
      const float h = f.kind == kFilterTophat ? tophat_value(i / HC, i % HC, NN, f) : 1.f;
      float2 o = Ok[i];
      Ok[i] = make_float2(o.x * h, o.y * h);
      if (Hk) Hk[i] = h;
    }
    return;
  }
  const int c0 = ct.obj_first[k], c1 = ct.obj_first[k + 1];
  // the clipped H on the half spectrum (into B), the loads of four frames
  // issued before their sums (which run in frame order)
  auto acc = [&](double w, float2 d, float2 s, double& nr, double& ni, double& den) {
    nr += w * ((double)d.x * s.x + (double)d.y * s.y);
    ni += w * ((double)d.y * s.x - (double)d.x * s.y);
    den += w * ((double)s.x * s.x + (double)s.y * s.y);
  };
  for (int i = tid; i < UNIT; i += 256) {
    double nr = 0.0, ni = 0.0, den = 0.0;
    for (int ci = c0; ci < c1; ++ci) {
      const int c = ct.obj_chans[ci];
      const size_t u0 = (size_t)(p * C + c) * J * UNIT + i;
      const float* wc = weights ? weights + c * J : nullptr;
      int j = 0;
      for (; j + 4 <= J; j += 4) {
        float2 d[4], s[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          d[e] = D[u0 + (size_t)(j + e) * UNIT];
          s[e] = S[u0 + (size_t)(j + e) * UNIT];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc(wc ? (double)wc[j + e] : 1.0, d[e], s[e], nr, ni, den);
      }
      for (; j < J; ++j)
        acc(wc ? (double)wc[j] : 1.0, D[u0 + (size_t)j * UNIT], S[u0 + (size_t)j * UNIT], nr, ni,
            den);
    }
    const double mag = nr * nr + ni * ni;
    double h = mag > 0.0 ? 1.0 - (double)f.noise_power * den / mag : 0.0;
    h = h < 0.2 ? 0.0 : (h > 1.0 ? 1.0 : h);
    B[i] = (float)h;
  }
  __syncthreads();
  // the full grid: a frequency right of the half spectrum takes its mirror
  // -u (the conjugate pair has the same |num| and den)
  for (int i = tid; i < GRID; i += 256) {
    const int y = i / NN, x = i % NN;
    const int hy = x > NN / 2 ? (NN - y) % NN : y, hx = x > NN / 2 ? NN - x : x;
    A[i] = B[hy * HC + hx];
  }
  __syncthreads();
  for (int i = tid; i < GRID; i += 256) {
    const int y = i / NN, x = i % NN;
    float v[9];
    int n = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx)
        v[n++] = A[((y + dy + NN) % NN) * NN + (x + dx + NN) % NN];
    B[i] = median9(v);
  }
  __syncthreads();
  if constexpr (NN == 64) {
    // the island search on bit masks: row y of the grid is a 64-bit word,
    // held by lane y of the first wave; each sweep takes the rows above and
    // below, the periodic neighbours within the row, and the runs of the
    // row, until no word changes (the same 4-connected set as the label
    // propagation below)
    __shared__ unsigned long long Mrow[NN];
    for (int y = tid >> 6; y < NN; y += 4) {
      const unsigned long long m = __ballot(B[y * NN + (tid & 63)] > 0.f);
      if ((tid & 63) == 0) Mrow[y] = m;
    }
    __syncthreads();
    if (tid < 64) {
      const int y = tid;
      const unsigned long long m = Mrow[y];
      unsigned long long l = y == 0 ? (m & 1ull) : 0ull;
      for (int it = 0; it < GRID; ++it) {
        const unsigned long long v = shfl64(l, (y + NN - 1) % NN) | shfl64(l, (y + 1) % NN);
        unsigned long long x = l | (v & m);
        x |= ((x << 1) | (x >> 63) | (x >> 1) | (x << 63)) & m;
        x = fill_down(fill_up(x, m), m);
        const int ch = x != l;
        l = x;
        if (!__any(ch)) break;
      }
      Mrow[y] = l;
    }
    __syncthreads();
    for (int i = tid; i < UNIT; i += 256) {
      const int y = i / HC, x = i % HC;
      const float h = (Mrow[y] >> x) & 1ull ? B[y * NN + x] : 0.f;
      float2 o = Ok[i];
      Ok[i] = make_float2(o.x * h, o.y * h);
      if (Hk) Hk[i] = h;
    }
    return;
  }
  int* L = reinterpret_cast<int*>(A);
  for (int i = tid; i < GRID; i += 256) L[i] = (i == 0 && B[0] > 0.f) ? 1 : 0;
  __syncthreads();
  // labels only go from 0 to 1, so concurrent sweeps reach the same fixed
  // point; every pass that changes something adds a cell, so at most GRID
  // passes run
  for (int it = 0; it < GRID; ++it) {
    if (tid == 0) changed = 0;
    __syncthreads();
    int ch = 0;
    for (int i = tid; i < GRID; i += 256) {
      if (L[i] || !(B[i] > 0.f)) continue;
      const int y = i / NN, x = i % NN;
      if (L[((y + 1) % NN) * NN + x] | L[((y + NN - 1) % NN) * NN + x] |
          L[y * NN + (x + 1) % NN] | L[y * NN + (x + NN - 1) % NN]) {
        L[i] = 1;
        ch = 1;
      }
    }
    if (ch) atomicOr(&changed, 1);
    __syncthreads();
    const int go = changed;
    __syncthreads();
    if (!go) break;
  }
  for (int i = tid; i < UNIT; i += 256) {
    const int g = (i / HC) * NN + i % HC;
    const float h = L[g] ? B[g] : 0.f;
    float2 o = Ok[i];
    Ok[i] = make_float2(o.x * h, o.y * h);
    if (Hk) Hk[i] = h;
  }
}

__device__ inline double taper1(int x, int N, int b) {
  const int e = min(x, N - 1 - x);
  return e < b ? 0.5 * (1.0 - cos(kPi * (e + 0.5) / b)) : 1.0;
}

__global__ __launch_bounds__(256) void k_mosaic(int N, int K, int nx, int ny, int stride,
                                                int border, int Hm, int Wm,
                                                const float* __restrict__ obj,
                                                float* __restrict__ out) {
  // the 1-D taper of the block's patches, once per block (N <= 128)
  __shared__ double tw[128];
  for (int e = threadIdx.x; e < N; e += 256) tw[e] = taper1(e, N, border);
  __syncthreads();
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)K * Hm * Wm) return;
  const int k = (int)(idx / ((long)Hm * Wm));
  const int r = (int)(idx % ((long)Hm * Wm));
  const int y = r / Wm, x = r % Wm;
  const int ly = y - N + 1, lx = x - N + 1;
  const int iy0 = ly <= 0 ? 0 : (ly + stride - 1) / stride, iy1 = min(ny - 1, y / stride);
  const int ix0 = lx <= 0 ? 0 : (lx + stride - 1) / stride, ix1 = min(nx - 1, x / stride);
  double acc = 0.0, ws = 0.0;
  for (int iy = iy0; iy <= iy1; ++iy) {
    const int ey = y - iy * stride;
    const double wy = tw[ey];
    for (int ix = ix0; ix <= ix1; ++ix) {
      const int ex = x - ix * stride;
      const double w = wy * tw[ex];
      acc += w * (double)obj[(((size_t)(iy * nx + ix) * K + k) * N + ey) * N + ex];
      ws += w;
    }
  }
  out[idx] = (float)(acc / ws);
}

}  // namespace

hipError_t launch_filter(const Dims& d, const ChanTab& ct, const FilterTab& ft, const float2* D,
                         const float* weights, const float2* S, float2* O, float* H,
                         hipStream_t s) {
  const size_t lds = 2 * (size_t)d.N * d.N * sizeof(float);
  if (d.N == 64) {
    hipLaunchKernelGGL(k_filter<64>, dim3(d.P * d.K), dim3(256), lds, s, d.C, d.J, d.K, ct, ft,
                       D, weights, S, O, H);
  } else if (d.N == 96) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_filter<96>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_filter<96>, dim3(d.P * d.K), dim3(256), lds, s, d.C, d.J, d.K, ct, ft,
                       D, weights, S, O, H);
  } else {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_filter<128>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_filter<128>, dim3(d.P * d.K), dim3(256), lds, s, d.C, d.J, d.K, ct, ft,
                       D, weights, S, O, H);
  }
  return hipGetLastError();
}

hipError_t launch_mosaic(const Dims& d, const float* obj, int ny, int nx, int stride, int border,
                         float* out, hipStream_t s) {
  const int Hm = (ny - 1) * stride + d.N, Wm = (nx - 1) * stride + d.N;
  const long n = (long)d.K * Hm * Wm;
  hipLaunchKernelGGL(k_mosaic, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d.N, d.K, nx,
                     ny, stride, border, Hm, Wm, obj, out);
  return hipGetLastError();
}

}  // namespace mfbd
