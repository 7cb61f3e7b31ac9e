// Counter-based random numbers of the sampler (used when the caller passes
// no explicit random numbers): Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11), ten rounds of two 32 x 32 -> 64-bit products with the constants
// 0xD2511F53 and 0xCD9E8D57 on a 128-bit counter, the 64-bit key advanced by
// the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
#pragma once
#include "common.hpp"

namespace fire {

struct U4 {
  uint32_t x[4];
};

FIRE_DEV U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.x[2];
    U4 n;
    n.x[0] = (uint32_t)(p1 >> 32) ^ c.x[1] ^ k0;
    n.x[1] = (uint32_t)p1;
    n.x[2] = (uint32_t)(p0 >> 32) ^ c.x[3] ^ k1;
    n.x[3] = (uint32_t)p0;
    c = n;
  }
  return c;
}

// uniform in (0, 1) with 53 random bits from two 32-bit words
FIRE_DEV double unit53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * 0x1.0p-53;
}

// One Metropolis proposal's draws: the step xi (three normals, Box-Muller on
// blocks 0 and 1) and the acceptance uniform (block 2).  Counter (w, e +
// 2^16 b, lo32(c), hi32(c)), key (lo32(seed), hi32(seed)).
FIRE_DEV void proposal_randoms(uint64_t seed, uint64_t c, int e, int w, double xi[3], double& u) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  U4 o[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    U4 ctr;
    ctr.x[0] = (uint32_t)w;
    ctr.x[1] = (uint32_t)e + ((uint32_t)b << 16);
    ctr.x[2] = (uint32_t)c;
    ctr.x[3] = (uint32_t)(c >> 32);
    o[b] = philox4x32_10(ctr, k0, k1);
  }
  const double u1 = unit53(o[0].x[0], o[0].x[1]), u2 = unit53(o[0].x[2], o[0].x[3]);
  const double u3 = unit53(o[1].x[0], o[1].x[1]), u4 = unit53(o[1].x[2], o[1].x[3]);
  const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
  const double twopi = 6.283185307179586476925;
  xi[0] = r1 * cos(twopi * u2);
  xi[1] = r1 * sin(twopi * u2);
  xi[2] = r2 * cos(twopi * u4);
  u = unit53(o[2].x[0], o[2].x[1]);
}

}  // namespace fire
