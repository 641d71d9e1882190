// Counter-based normal deviates for Langevin dynamics: Philox4x32-10
// (Salmon, Moraes, Dror and Shaw, SC'11) and the Box-Muller transform.
// Each ion's deviates depend only on (seed, step, half, ion), so any thread
// can draw them without state and the stream is the same for any launch
// shape or batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace maze {

// Ten rounds on counter c with key (k0, k1): each round multiplies words 0
// and 2 by the two Philox constants, keeps high and low halves and mixes in
// words 1, 3 and the key; the key advances by the two Weyl constants
// between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t w0 = hi1 ^ c[1] ^ k0, w2 = hi0 ^ c[3] ^ k1;
    c[0] = w0;
    c[1] = lo1;
    c[2] = w2;
    c[3] = lo0;
  }
}

// Deviates of ion i for OVRVO half step `half` of step `step`: counter
// (i, half, step mod 2^32, step div 2^32), key (seed mod 2^32, seed div
// 2^32); u1 = (x + 1) 2^-32 in (0, 1], u2 = x' 2^-32; z = (r cos, r sin) of
// words (0, 1) and r cos of words (2, 3), r = sqrt(-2 ln u1).
__device__ __forceinline__ void langevin_normals(uint64_t seed, long long step, int half, int i,
                                                 double z[3]) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)half, (uint32_t)((uint64_t)step & 0xFFFFFFFFull),
                   (uint32_t)((uint64_t)step >> 32)};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  const double s = 0x1p-32;
  const double two_pi = 6.283185307179586;
  const double u1a = ((double)c[0] + 1.0) * s, u2a = (double)c[1] * s;
  const double u1b = ((double)c[2] + 1.0) * s, u2b = (double)c[3] * s;
  const double ra = sqrt(-2.0 * log(u1a)), rb = sqrt(-2.0 * log(u1b));
  z[0] = ra * cos(two_pi * u2a);
  z[1] = ra * sin(two_pi * u2a);
  z[2] = rb * cos(two_pi * u2b);
}

}  // namespace maze
