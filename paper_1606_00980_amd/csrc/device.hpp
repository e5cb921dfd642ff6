// Device helpers: wavefront reductions, XCD-aware work mapping and
// grouped-launch lookup.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace gp {

constexpr int WAVE = 64;
constexpr int NXCD = 8;   // accelerator complex dies; workgroups are dealt to them round-robin

// a * b + c rounded once (explicit, independent of the compiler's choice to
// contract a product and a sum)
__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// NV values summed over the wavefront together, every lane receiving all NV
// totals: M halving exchanges (distances 32, 16, ... for the next power of two
// 2^M >= NV) leave each lane a partial of value lane >> (6 - M), a butterfly
// over the remaining distances completes it, and the totals are read back
// from one lane per value.  The order of the additions is fixed.
template <int NV>
__device__ inline void wave_sums(double (&a)[NV]) {
  constexpr int M = NV <= 1 ? 0 : NV <= 2 ? 1 : NV <= 4 ? 2 : 3;
  constexpr int NP = 1 << M;
  static_assert(NV <= 8, "at most 8 values");
  const int lane = threadIdx.x % WAVE;
  double b[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) b[i] = i < NV ? a[i] : 0.0;
#pragma unroll
  for (int st = 0; st < M; ++st) {
    const int dist = 32 >> st;
    const int half = NP >> (st + 1);
    const bool hi = (lane & dist) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double keep = hi ? b[i + half] : b[i];
      const double send = hi ? b[i] : b[i + half];
      b[i] = keep + __shfl_xor(send, dist, WAVE);
    }
  }
  double e = b[0];
#pragma unroll
  for (int dist = 32 >> M; dist > 0; dist >>= 1) e += __shfl_xor(e, dist, WAVE);
  const long long eb = __builtin_bit_cast(long long, e);
  const int lo = (int)eb, hi = (int)(eb >> 32);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const unsigned l = (unsigned)__builtin_amdgcn_readlane(lo, i * (64 >> M));
    const unsigned h = (unsigned)__builtin_amdgcn_readlane(hi, i * (64 >> M));
    a[i] = __builtin_bit_cast(double, ((unsigned long long)h << 32) | l);
  }
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

// Raw buffer access: a wave-uniform descriptor (base address, size in bytes)
// held in scalar registers, a per-lane 32-bit byte offset and a wave-uniform
// byte offset.  Address arithmetic then stays off the vector ALU.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;   // raw buffer, 32-bit data format (gfx9)

__device__ __forceinline__ Rsrc make_rsrc(const void* base, size_t bytes) {
  const unsigned n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)n, RSRC_WORD3);
}
template <typename T> __device__ __forceinline__ T bload(Rsrc r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ float bload<float>(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ int bload<int>(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(int, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(Rsrc r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(Rsrc r, unsigned voff, unsigned soff, double v) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 0);
}

// A [rows][N] array (one right-hand side's [K][N] vector, or a packed [NB][N]
// block array) of T: row i of voxel n is ld(i, n * sizeof(T)).
template <typename T> struct Slab {
  Rsrc rs;
  unsigned row;   // N * sizeof(T), the byte stride of a row
  __device__ __forceinline__ Slab(const void* base, int rows, int N)
      : rs(make_rsrc(base, (size_t)rows * N * sizeof(T))), row((unsigned)N * (unsigned)sizeof(T)) {}
  __device__ __forceinline__ T ld(int i, unsigned voff) const { return bload<T>(rs, voff, (unsigned)i * row); }
  __device__ __forceinline__ void st(int i, unsigned voff, T v) const { bstore(rs, voff, (unsigned)i * row, v); }
};

// Which problem of a grouped launch owns work item w (of the inner or the
// outer work decomposition).
template <bool OUTER = false>
__device__ inline int find_prob(const Prob* __restrict__ probs, int nprob, int w) {
  int p = 0;
  while (p + 1 < nprob && w >= (OUTER ? probs[p + 1].work_begin_o : probs[p + 1].work_begin)) ++p;
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
  wave_sums<NV>(s);
}

}  // namespace gp
