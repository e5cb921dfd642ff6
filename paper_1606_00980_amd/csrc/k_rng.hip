// Counter-based random vectors for Algorithm 2 (z1, z2 ~ N(0, I)) and for
// Hutchinson probes (Rademacher +-1): Philox4x32 with 10 rounds, as published
// by Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as
// 1, 2, 3", SC'11).
//
// Element layout (shared with every consumer of these vectors):
//   normals    : pair q = e / 2 uses counter (q_lo, q_hi, s_lo, s_hi) and key
//                (seed_lo, seed_hi); words (w0..w3) give two 53-bit uniforms
//                u1 = ((w1:w0) >> 11 + 0.5) 2^-53, u2 = ((w3:w2) >> 11 + 0.5) 2^-53,
//                and Box-Muller gives e = 2q: sqrt(-2 ln u1) cos(2 pi u2),
//                e = 2q + 1: sqrt(-2 ln u1) sin(2 pi u2);
//   Rademacher : block q = e / 128 uses the same counter form; bit (e % 128) of
//                the 128-bit word string w0 | w1 << 32 | ... selects +1 (set)
//                or -1 (clear);
//   Gamma      : element e, attempt t (t < 64) uses blocks 128 e + 2 t (x, the
//                Box-Muller normal of the cosine branch) and 128 e + 2 t + 1
//                (the acceptance uniform from (w1:w0)); for shape < 1 the boost
//                uniform comes from (w3:w2) of block 128 e + 1.  The method is
//                Marsaglia and Tsang's ("A simple method for generating gamma
//                variables", ACM TOMS 2000); after 64 rejections the value is
//                d = a - 1/3.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace gp {

namespace {

constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    const uint64_t p0 = (uint64_t)PHILOX_M0 * c.x;
    const uint64_t p1 = (uint64_t)PHILOX_M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ inline U4 draw(uint64_t q, uint64_t seed, uint64_t stream) {
  return philox4x32_10(U4{(uint32_t)q, (uint32_t)(q >> 32), (uint32_t)stream, (uint32_t)(stream >> 32)},
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ inline double uniform53(uint32_t lo, uint32_t hi) {
  const uint64_t m = (((uint64_t)hi << 32) | lo) >> 11;
  return ((double)m + 0.5) * 0x1.0p-53;
}

__global__ __launch_bounds__(256) void k_normal(uint64_t seed, uint64_t stream, size_t n, double* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * q >= n) return;
  const U4 w = draw(q, seed, stream);
  const double u1 = uniform53(w.x, w.y), u2 = uniform53(w.z, w.w);
  const double rad = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  out[2 * q] = rad * c;
  if (2 * q + 1 < n) out[2 * q + 1] = rad * s;
}

__global__ __launch_bounds__(256) void k_rademacher(uint64_t seed, uint64_t stream, size_t n,
                                                    int8_t* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t e0 = q * 128;
  if (e0 >= n) return;
  const U4 w = draw(q, seed, stream);
  const uint32_t words[4] = {w.x, w.y, w.z, w.w};
  const size_t cnt = n - e0 < 128 ? n - e0 : 128;
  for (size_t i = 0; i < cnt; ++i) out[e0 + i] = ((words[i >> 5] >> (i & 31)) & 1u) ? (int8_t)1 : (int8_t)-1;
}

// out[e] = scale[e] (1 when scale is null) times a Gamma(shape, 1) variate.
__global__ __launch_bounds__(256) void k_gamma(uint64_t seed, uint64_t stream, size_t n, double shape,
                                               const double* __restrict__ scale, double* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double a = shape >= 1.0 ? shape : shape + 1.0;
  const double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
  double g = d;
  for (int t = 0; t < 64; ++t) {
    const uint64_t q = (uint64_t)e * 128u + 2u * (uint64_t)t;
    const U4 wa = draw(q, seed, stream), wb = draw(q + 1, seed, stream);
    const double u1 = uniform53(wa.x, wa.y), u2 = uniform53(wa.z, wa.w);
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    const double x = sqrt(-2.0 * log(u1)) * cs;
    const double u = uniform53(wb.x, wb.y);
    const double b = 1.0 + c * x;
    const double v = b * b * b;
    if (!(v > 0.0)) continue;
    const double x2 = x * x;
    if (u < 1.0 - 0.0331 * x2 * x2 || log(u) < 0.5 * x2 + d * (1.0 - v + log(v))) {
      g = d * v;
      break;
    }
  }
  if (shape < 1.0) {
    const U4 wb = draw((uint64_t)e * 128u + 1u, seed, stream);
    g *= pow(uniform53(wb.z, wb.w), 1.0 / shape);
  }
  out[e] = g * (scale ? scale[e] : 1.0);
}

__global__ __launch_bounds__(256) void k_philox_raw(uint64_t seed, uint64_t stream, size_t nblocks,
                                                    uint32_t* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nblocks) return;
  const U4 w = draw(q, seed, stream);
  out[4 * q + 0] = w.x;
  out[4 * q + 1] = w.y;
  out[4 * q + 2] = w.z;
  out[4 * q + 3] = w.w;
}

}  // namespace

hipError_t launch_rng_normal(hipStream_t s, uint64_t seed, uint64_t stream, size_t n, double* out) {
  if (n == 0) return hipSuccess;
  const size_t pairs = (n + 1) / 2;
  GP_LAUNCH(k_normal, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, seed, stream, n, out);
  return hipGetLastError();
}

hipError_t launch_rng_gamma(hipStream_t s, uint64_t seed, uint64_t stream, size_t n, double shape,
                            const double* scale, double* out) {
  if (n == 0) return hipSuccess;
  GP_LAUNCH(k_gamma, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, stream, n, shape, scale, out);
  return hipGetLastError();
}

hipError_t launch_rng_rademacher(hipStream_t s, uint64_t seed, uint64_t stream, size_t n, int8_t* out) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 127) / 128;
  GP_LAUNCH(k_rademacher, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s, seed, stream, n, out);
  return hipGetLastError();
}

hipError_t launch_rng_raw(hipStream_t s, uint64_t seed, uint64_t stream, size_t nblocks, uint32_t* out) {
  if (nblocks == 0) return hipSuccess;
  GP_LAUNCH(k_philox_raw, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0, s, seed, stream, nblocks,
                     out);
  return hipGetLastError();
}

}  // namespace gp
