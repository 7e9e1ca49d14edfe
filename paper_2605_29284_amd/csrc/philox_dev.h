// Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011) and Box-Muller normals on the
// device.  Each round multiplies counter words 0 and 2 by the published odd
// constants, keeps the high and low halves of the 64-bit products, and mixes the
// high halves with words 1 and 3 and the round key; the key advances by the two
// published Weyl increments between rounds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

namespace krig {

struct u32x4 {
  uint32_t v[4];
};

__host__ __device__ inline u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c.v[0];
    const uint64_t p1 = (uint64_t)M1 * c.v[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    u32x4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
  }
  return c;
}

// (x + 1/2) / 2^32, exact in FP64
__host__ __device__ inline double u01_f64(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

// two N(0,1) values from two 32-bit words (FP64 arithmetic)
__device__ inline void box_muller_f64(uint32_t x0, uint32_t x1, double& n0, double& n1) {
  const double u0 = u01_f64(x0), u1 = u01_f64(x1);
  const double r = sqrt(-2.0 * log(u0));
  double s, c;
  sincospi(2.0 * u1, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

// the same two normals with the logarithm, square root and sine/cosine in FP32 (the uniforms
// are formed in FP64 and rounded once): a few ulp of FP32, for samplers that compute in FP32
__device__ inline void box_muller_f32(uint32_t x0, uint32_t x1, float& n0, float& n1) {
  const float u0 = (float)u01_f64(x0), u1 = (float)u01_f64(x1);
  const float r = sqrtf(-2.0f * logf(u0));
  float s, c;
  sincospif(2.0f * u1, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

enum { STREAM_CE = 0, STREAM_NUGGET = 1 };

}  // namespace krig
