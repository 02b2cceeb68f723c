// Counter-based Gaussian test matrix Omega for the sketch (Algorithm 1's
// Gaussian block Omega_i; Theorem "projector"'s n x (k+p) Gaussian Omega).
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) followed by the
// Box-Muller transform (Box & Muller, 1958).
//   key     = (seed mod 2^32, seed >> 32)
//   counter = (row r, column c >> 2, stream, 0)
//   words (x0,x1) feed columns 4j, 4j+1 and (x2,x3) feed 4j+2, 4j+3:
//     u1 = (xa + 1) 2^-32,  u2 = xb 2^-32,
//     z_even = sqrt(-2 ln u1) cos(2 pi u2),  z_odd = sqrt(-2 ln u1) sin(2 pi u2).
// Columns are global, so a narrower Omega is a prefix of a wider one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rg {

struct U4 { uint32_t x[4]; };

__host__ __device__ inline U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                            uint32_t c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  U4 o; o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
  return o;
}

// four normals for row r, columns 4j..4j+3, in double precision
__device__ inline void gauss4_f64(uint64_t seed, uint32_t stream, uint32_t r, uint32_t j,
                                  double z[4]) {
  U4 w = philox4x32_10(r, j, stream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double two32 = 2.3283064365386963e-10;  // 2^-32
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double u1 = ((double)w.x[2 * h] + 1.0) * two32;
    double u2 = (double)w.x[2 * h + 1] * two32;
    double rad = sqrt(-2.0 * log(u1));
    double ang = 2.0 * 3.141592653589793 * u2;
    z[2 * h] = rad * cos(ang);
    z[2 * h + 1] = rad * sin(ang);
  }
}

// the same four normals evaluated in single precision (hardware log/sin/cos
// of the uniform in revolutions); used by the fp32 and bf16 paths
__device__ inline void gauss4_f32(uint64_t seed, uint32_t stream, uint32_t r, uint32_t j,
                                  float z[4]) {
  U4 w = philox4x32_10(r, j, stream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
  const float two32 = 2.3283064365386963e-10f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float u1 = ((float)w.x[2 * h] + 1.0f) * two32;   // may round to 1.0: ln -> 0, fine
    if (w.x[2 * h] == 0xFFFFFFFFu) u1 = 1.0f;
    float u2 = (float)(w.x[2 * h + 1] >> 8) * 5.9604644775390625e-08f;  // 2^-24 grid, < 1
    float rad = __fsqrt_rn(-2.0f * __logf(u1));
    float s, c;
    __sincosf(6.283185307179586f * u2, &s, &c);
    z[2 * h] = rad * c;
    z[2 * h + 1] = rad * s;
  }
}

}  // namespace rg
