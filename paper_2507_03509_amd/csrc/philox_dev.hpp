// Counter-based noise for the amplifier model.
//
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): a 4 x 64-bit counter block is mixed by ten rounds
// of two 64 x 64 -> 128-bit multiplications (multipliers 0xD2E7470EE14C6C93
// and 0xCA5A826395121157), a word permutation and an xor with the 2 x 64-bit
// key; the key advances by the Weyl constants 0x9E3779B97F4A7C15 and
// 0xBB67AE8584CAA73B between rounds.  Every (key, counter) pair is an
// independent draw, so any lane can produce the noise of any time sample
// without state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssfm {

struct u64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                uint64_t c3, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {{c0, c1, c2, c3}};
}

// u = ((w >> 41) + 1/2) * 2^-23: 23 random bits plus a half, exact in FP32,
// strictly inside (0, 1).
__device__ __forceinline__ float word_to_uniform(uint64_t w) {
  return ((float)(uint32_t)(w >> 41) + 0.5f) * 0x1p-23f;
}

// Box-Muller: (g1, g2) = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2), two
// independent standard normals.
__device__ __forceinline__ float2 box_muller(uint64_t w1, uint64_t w2) {
  const float u1 = word_to_uniform(w1);
  const float u2 = word_to_uniform(w2);
  const float rad = sqrtf(-2.0f * logf(u1));
  float s, c;
  sincospif(2.0f * u2, &s, &c);
  return make_float2(rad * c, rad * s);
}

}  // namespace ssfm
