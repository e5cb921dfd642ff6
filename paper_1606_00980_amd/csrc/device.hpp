// Device helpers: wavefront reductions, XCD-aware work mapping, grouped-launch
// lookup and the last-workgroup handshake used for deterministic reductions.
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

// Called by every workgroup of problem `pr` after its partial results are
// stored.  Returns true in exactly one workgroup, the last one to arrive, after
// making every other workgroup's stores visible to it.
__device__ inline bool arrive_last(const Prob& pr) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(pr.counter, 1u);
    s_last = (prev == (unsigned)(pr.work_count - 1)) ? 1 : 0;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// Sum partials[v][r][0..nt) for one right-hand side across one wavefront in a
// fixed order (strided per lane, then a butterfly): the result depends only on
// the operator's tiling, never on which other right-hand sides share the launch.
template <int NV>
__device__ inline void sum_partials(const double* part, int R, int nt, int r, double (&s)[NV]) {
  const int lane = threadIdx.x % WAVE;
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  for (int t = lane; t < nt; t += WAVE) {
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] += part[((size_t)v * R + r) * nt + t];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = wave_sum(s[v]);
}

// Count right-hand sides per phase and publish the summary; resets the counter.
__device__ inline void publish_summary(const Prob& pr) {
  __shared__ int s_cnt[3][TILE / WAVE];
  __syncthreads();
  int c[3] = {0, 0, 0};
  for (int r = threadIdx.x; r < pr.R; r += blockDim.x) {
    const int ph = pr.st[r].phase;
    c[0] += ph == PH_OUTER;
    c[1] += ph == PH_INNER;
    c[2] += ph == PH_DONE;
  }
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  for (int i = 0; i < 3; ++i) {
    const int s = wave_sum_int(c[i]);
    if (lane == 0) s_cnt[i][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / WAVE;
    for (int i = 0; i < 3; ++i) {
      int t = 0;
      for (int j = 0; j < nw; ++j) t += s_cnt[i][j];
      pr.summary[i] = t;
    }
    __threadfence();
    atomicExch(pr.counter, 0u);
  }
}

}  // namespace gp
