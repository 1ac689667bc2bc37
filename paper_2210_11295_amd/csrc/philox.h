// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), host and device.
//
// The paper draws each Omega^(i) from a seeded generator (section 4) without
// naming one; a counter-based generator lets every block, row and sample be
// drawn independently and in parallel from (seed, block, index), so the GPU
// builds its tables without any sequential state.  Stream layout:
//   key = (seed, 0); counter = (index word, block, tag, 0);
//   tag 1: row sample R; tag 2: input signs D; tag 3: output signs Dt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsrht {

enum : uint64_t { kTagR = 1, kTagD = 2, kTagDt = 3 };

struct Philox4 {
  uint64_t w[4];
};

__host__ __device__ inline void mul_hilo64(uint64_t a, uint64_t b, uint64_t &hi,
                                           uint64_t &lo) {
  unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
  hi = (uint64_t)(prod >> 64);
  lo = (uint64_t)prod;
}

// Ten rounds; the key is bumped by the Weyl increments between rounds.
__host__ __device__ inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1,
                                                 uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    uint64_t hi0, lo0, hi1, lo1;
    mul_hilo64(M0, c0, hi0, lo0);
    mul_hilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  Philox4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

// Bit `bit` (0..255) of the 256-bit output, bit b living in word b/64.
__host__ __device__ inline uint32_t philox_bit(const Philox4 &o, uint32_t bit) {
  return (uint32_t)(o.w[bit >> 6] >> (bit & 63)) & 1u;
}

// 32 consecutive bits starting at a multiple of 32.
__host__ __device__ inline uint32_t philox_word32(const Philox4 &o, uint32_t bit0) {
  return (uint32_t)(o.w[bit0 >> 6] >> (bit0 & 63));
}

}  // namespace bsrht
