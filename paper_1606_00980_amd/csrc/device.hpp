// Device helpers: wavefront reductions, XCD-aware work mapping and
// grouped-launch lookup.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace gp {

constexpr int WAVE = 64;
constexpr int NXCD = 8;   // accelerator complex dies; workgroups are dealt to them round-robin

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ inline int wave_sum_int(int v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Workgroup id -> work item such that the items handled by one XCD form one
// contiguous range (neighbouring voxel tiles then share that XCD's L2).
__device__ inline int xcd_remap(int bid, int W) {
  const int xcd = bid % NXCD, slot = bid / NXCD;
  const int base = W / NXCD, rem = W % NXCD;
  return xcd * base + (xcd < rem ? xcd : rem) + slot;
}

// Which problem of a grouped launch owns work item w.
__device__ inline int find_prob(const Prob* __restrict__ probs, int nprob, int w) {
  int p = 0;
  while (p + 1 < nprob && w >= probs[p + 1].work_begin) ++p;
  return p;
}

// Sum partials[v][r][0..nt) for one right-hand side across one wavefront in a
// fixed order (strided per lane, then a butterfly): the result depends only on
// the operator's tiling, never on which other right-hand sides share the launch.
template <int NV>
__device__ inline void sum_partials(const double* part, int R, int stride, int nt, int r, double (&s)[NV]) {
  const int lane = threadIdx.x % WAVE;
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  const __attribute__((address_space(1))) double* g = (const __attribute__((address_space(1))) double*)part;
  for (int t = lane; t < nt; t += WAVE) {
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] += g[((size_t)v * R + r) * stride + t];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = wave_sum(s[v]);
}

}  // namespace gp
