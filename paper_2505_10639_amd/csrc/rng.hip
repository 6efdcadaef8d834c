// Standard normal draws from a counter-based generator, for the synthetic
// bursts that train the warm-start network: Philox4x32-10 (Salmon, Moraes,
// Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011)
// gives four 32-bit words per 128-bit counter, and the Box-Muller transform
// turns each pair of words into two normals.
//
// Draw i of a call uses block b = counter0 + i / 4 (the counter words are
// the low and high halves of b, then of `stream_id`), key = the two halves
// of `seed`; words (x0, x1) give draws 4b, 4b+1 and (x2, x3) draws 4b+2,
// 4b+3:
//   u1 = (x0 >> 8) + 1/2) 2^-24,  u2 = ((x1 >> 8) + 1/2) 2^-24   (in (0, 1))
//   r = sqrt(-2 ln u1),  z0 = r cos(2 pi u2),  z1 = r sin(2 pi u2).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "momfbd.h"

namespace mfbd {
namespace {

constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;   // round multipliers
constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u; // key increments

struct Words {
  uint32_t x[4];
};

// Ten rounds of Philox4x32 on counter c with key (k0, k1).
__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(kMul0, c0), lo0 = kMul0 * c0;
    const uint32_t hi1 = __umulhi(kMul1, c2), lo1 = kMul1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return Words{{c0, c1, c2, c3}};
}

__device__ __forceinline__ float2 box_muller(uint32_t a, uint32_t b) {
  const float u1 = ((float)(a >> 8) + 0.5f) * 5.9604644775390625e-8f;   // 2^-24
  const float u2 = ((float)(b >> 8) + 0.5f) * 5.9604644775390625e-8f;
  const float r = sqrtf(-2.0f * logf(u1));
  float s, c;
  sincosf(6.283185307179586f * u2, &s, &c);
  return make_float2(r * c, r * s);
}

// One thread per block of four draws.
__global__ __launch_bounds__(256) void k_normal(uint64_t seed, uint64_t stream_id,
                                                uint64_t counter0, long n,
                                                float* __restrict__ out,
                                                uint32_t* __restrict__ bits) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long i0 = 4 * t;
  if (i0 >= n) return;
  const uint64_t b = counter0 + (uint64_t)t;
  const Words w = philox4x32_10((uint32_t)b, (uint32_t)(b >> 32), (uint32_t)stream_id,
                                (uint32_t)(stream_id >> 32), (uint32_t)seed,
                                (uint32_t)(seed >> 32));
  const float2 z01 = box_muller(w.x[0], w.x[1]);
  const float2 z23 = box_muller(w.x[2], w.x[3]);
  const float z[4] = {z01.x, z01.y, z23.x, z23.y};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (i0 + e >= n) break;
    out[i0 + e] = z[e];
    if (bits) bits[i0 + e] = w.x[e];
  }
}

}  // namespace
}  // namespace mfbd

extern "C" int momfbd_random_normal(unsigned long long seed, unsigned long long stream_id,
                                    unsigned long long counter0, size_t n, float* out,
                                    unsigned int* bits, void* stream) {
  if (!out || n == 0 || n > (size_t(1) << 40)) return MOMFBD_EINVAL;
  if (hipGetLastError() != hipSuccess) return MOMFBD_EDEVICE;
  const long threads = (long)((n + 3) / 4);
  hipLaunchKernelGGL(mfbd::k_normal, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, (uint64_t)seed, (uint64_t)stream_id,
                     (uint64_t)counter0, (long)n, out, reinterpret_cast<uint32_t*>(bits));
  return hipGetLastError() == hipSuccess ? MOMFBD_OK : MOMFBD_EDEVICE;
}
