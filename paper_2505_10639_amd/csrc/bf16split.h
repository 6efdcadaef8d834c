// Exact three-way bf16 split of FP32 values, for FP32 contractions on the
// bf16 matrix cores.
//
// x = hi + mid + lo exactly, each term a bf16 (the upper 16 bits of an FP32
// word): hi is x with its low 16 bits cleared (8 significant bits); the
// remainder r = x - hi is exact (the 16 bits cleared) and splits the same
// way into mid and lo = r - mid (exact, at most 8 significant bits).  This
// holds for x = 0 and every |x| >= 2^-110; below, lo keeps only the bits
// from 2^-133 (the smallest bf16 step) up.  A
// product x y is then formed from the six partial products whose orders
// (hi 0, mid 1, lo 2) add up to at most 2.  With |mid| < 2^-7 |x| and
// |lo| < 2^-15 |x|, the three left out are below 2^-21 |x y| together
// (FP32 rounds at 2^-24), and a sum of such products is as accurate as its
// FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#define MFBD_SPLIT_HDI __host__ __device__ __forceinline__

namespace mfbd {

MFBD_SPLIT_HDI uint32_t f2u(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_bit_cast(uint32_t, x);
#else
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return u;
#endif
}

MFBD_SPLIT_HDI float u2f(uint32_t u) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_bit_cast(float, u);
#else
  float x;
  std::memcpy(&x, &u, 4);
  return x;
#endif
}

// The three bf16 parts of x, each as an FP32 word whose low 16 bits are zero
// (lo is cut to its upper 16 bits too: a no-op for |x| >= 2^-110, and for
// smaller x the bits that no bf16 holds, which must not reach the packed
// neighbour).
MFBD_SPLIT_HDI void split3_words(float x, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = f2u(x) & 0xFFFF0000u;
  const float r = x - u2f(h);
  m = f2u(r) & 0xFFFF0000u;
  l = f2u(r - u2f(m)) & 0xFFFF0000u;
}

// Eight values -> three groups of eight packed bf16 (element e in bits
// 16 (e & 1) of word e >> 1): the operand of one 16x16x32 bf16 MFMA per part.
struct Split8 {
  uint32_t h[4], m[4], l[4];
};

MFBD_SPLIT_HDI Split8 split8(const float (&v)[8]) {
  Split8 s;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t h0, m0, l0, h1, m1, l1;
    split3_words(v[2 * w], h0, m0, l0);
    split3_words(v[2 * w + 1], h1, m1, l1);
    s.h[w] = (h0 >> 16) | h1;
    s.m[w] = (m0 >> 16) | m1;
    s.l[w] = (l0 >> 16) | l1;
  }
  return s;
}

}  // namespace mfbd
