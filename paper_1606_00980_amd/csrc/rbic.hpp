// Kernels of the incomplete Cholesky preconditioning on the red-black voxel order (the
// preconditioner M of Algorithm 2, steps 6-7, as a zero-fill factor in K x K
// voxel blocks).
//
// Order the voxels red (even x + y + z) first, then black.  Q splits as
//   [ D_R  E ]      D_R = blkdiag(Q_nn) over red voxels, D_B likewise,
//   [ E'  D_B ]     E = -diag(alpha) on every (red, black) adjacent pair,
// since no two voxels of one colour are adjacent.  The block IC(0) factor is
// then L = [ L_R 0 ; E' L_R^{-T}  L_B ] with L_R L_R' = D_R exactly and
// L_B L_B' = blkdiag(S_m), the diagonal blocks of the Schur complement
//   S = D_B - E' D_R^{-1} E,   S_m = Q_mm - sum_{n ~ m} diag(alpha) Q_nn^{-1} diag(alpha)
// (the fill that S has between black voxels sharing a red neighbour is what
// the zero-fill rule drops).  M = L L' equals Q except in that dropped fill,
// so M^{-1} Q is the identity on the red rows.  PCG with M from a start value
// whose red residual rows vanish keeps them zero, and its black iterates are
// those of PCG on S x_B = c_B, c_B = b_B - E' D_R^{-1} b_R, preconditioned by
// blkdiag(S_m) -- a local (per-voxel) preconditioner.  The solver below runs
// that half-size iteration in the one-reduction PCG form of the main solver:
//   red stage   : u_n = Q_nn^{-1} (alpha .* sum_{m ~ n} v_m)       (red voxels)
//   black stage : (S v)_m = Q_mm v_m - alpha .* sum_{n ~ m} u_n    (black voxels)
// and recovers x_R = Q_nn^{-1} (b_n + alpha .* sum_{m ~ n} x_m) at the end,
// which makes the red residual rows vanish, so ||b - Q x|| = ||c_B - S x_B||.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "launch.hpp"
#include "pcg.hpp"
#include "spd.hpp"

namespace gp {
namespace {

template <typename T> struct RbT;
template <> struct RbT<double> {
  __device__ static const double* D(const RbDev& b) { return b.D64; }
  __device__ static const double* S(const RbDev& b) { return b.S64; }
  __device__ static const double* P(const RbDev& b) { return b.P64; }
  __device__ static double alpha(const RbDev& b, int k) { return b.alpha64[k]; }
};
template <> struct RbT<float> {
  __device__ static const float* D(const RbDev& b) { return b.D32; }
  __device__ static const float* S(const RbDev& b) { return b.S32; }
  __device__ static const float* P(const RbDev& b) { return b.P32; }
  __device__ static float alpha(const RbDev& b, int k) { return b.alpha32[k]; }
};

// Sum NV per-thread values over the workgroup in a fixed order and store
// value v at part[v * vstride + at].  Every thread of the workgroup calls it.
template <int NV>
__device__ inline void block_sums(double (&v)[NV], double* part, size_t vstride, size_t at) {
  __shared__ double sh[NV][TILE / WAVE];
  __syncthreads();   // a previous call's readers are done with sh
  wave_deposit<NV>(&sh[0][0], 0, v);
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < TILE / WAVE; ++w) s += sh[threadIdx.x][w];
    part[(size_t)threadIdx.x * vstride + at] = s;
  }
}

// y = A x, A symmetric, given by its packed entries A.ld(i, voff).
template <typename T, int K>
__device__ __forceinline__ void packed_apply(const Slab<T>& A, unsigned voff, const T (&x)[K], T (&y)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) y[k] = 0;
  sym_apply<K>([&](int i) { return A.ld(i, voff); }, x, y);
}

// Block sums of NV values for each right-hand side of a work item, with the
// cross-wavefront step done once for the whole item: add() reduces within the
// wavefront and parks the result in LDS; flush() waits once and writes
// part[v * vstride + r * pstride + tile] for the right-hand sides added.
template <int NV>
struct ItemSums {
  double (*sh)[NV][TILE / WAVE];
  unsigned mask = 0;   // right-hand sides (relative to r0) added
  __device__ ItemSums() {
    __shared__ double buf[RCMAX][NV][TILE / WAVE];
    sh = buf;
  }
  __device__ void add(int rl, const double (&v)[NV]) {
    // the NV values summed over the wavefront together (halving exchanges)
    wave_deposit<NV>(&sh[0][0][0], rl, v);
    mask |= 1u << rl;
  }
  __device__ void flush(double* part, size_t vstride, int r0, int nr, int pstride, int tile) {
    __syncthreads();
    for (int t = threadIdx.x; t < nr * NV; t += TILE) {
      const int rl = t / NV, i = t % NV;
      if (!((mask >> rl) & 1u)) continue;
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < TILE / WAVE; ++w) s += sh[rl][i][w];
      part[(size_t)i * vstride + (size_t)(r0 + rl) * pstride + tile] = s;
    }
  }
};

// sum over the six neighbour slots of vector v (rows of one right-hand side),
// a missing neighbour (-1) contributing zero.  Branch free: a missing slot
// loads entry 0 (a valid address) and drops it with a select, so the loads of
// all six neighbours are in flight together.
template <typename T, int K>
__device__ __forceinline__ void neighbour_sum(const int (&nb)[6], const Slab<T>& v, T (&s)[K]) {
  T t[6][K];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const unsigned o = nb[d] < 0 ? 0u : (unsigned)nb[d] * (unsigned)sizeof(T);
#pragma unroll
    for (int k = 0; k < K; ++k) t[d][k] = v.ld(k, o);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] += nb[d] < 0 ? (T)0 : t[d][k];
  }
}

// Work items of a grouped solver-round launch over the members of one K group:
// black-tile items (256 black positions, a chunk of Rc right-hand sides) for the
// inner stages, red-tile items for the red stage, and black-tile items of a
// chunk of Rco right-hand sides for the outer step.  A member's items are
// numbered from its first item by block of tiles (tbB or tbR of them), then
// chunk, then tile, and the launch's items are dealt to the XCDs in contiguous
// ranges: an XCD sweeps a block's tiles once per chunk, with the block's
// voxel blocks and the chunk's vectors around the tiles in its L2.
enum RbWhich : int { RBW_BLACK = 0, RBW_RED = 1, RBW_OUTER = 2 };

struct RbWork {
  int p, tile, r0, r1;
  bool first;   // the member's first item (takes the profiling counts)
};

template <int WHICH>
__device__ __forceinline__ int rb_first_item(const RbProb& P) {
  return WHICH == RBW_BLACK ? P.wB : WHICH == RBW_RED ? P.wR : P.wO;
}

template <int WHICH>
__device__ inline RbWork rb_item(const RbProb* __restrict__ probs, int nprob) {
  const int wi = xcd_remap(blockIdx.x, gridDim.x);
  int p = 0;
  while (p + 1 < nprob && wi >= rb_first_item<WHICH>(probs[p + 1])) ++p;
  const RbProb& P = probs[p];
  const int loc = wi - rb_first_item<WHICH>(P);
  const int rc = WHICH == RBW_OUTER ? P.Rco : P.Rc;
  const int nch = WHICH == RBW_OUTER ? P.ncho : P.nch;
  const int nt = WHICH == RBW_RED ? P.rb.ntR : P.rb.ntB;
  const int tb = WHICH == RBW_RED ? P.rb.tbR : P.rb.tbB;
  // block of tb tiles (the last one shorter), then chunk, then tile
  const int per = tb * nch;
  const int blk = loc / per, rem = loc - blk * per;
  const int len = min(tb, nt - blk * tb);
  RbWork w;
  w.p = p;
  w.tile = blk * tb + rem % len;
  w.r0 = (rem / len) * rc;
  w.r1 = min(P.pr.R, w.r0 + rc);
  w.first = loc == 0;
  return w;
}

// While profiling: one count in `slot` per launch in which some right-hand
// side of the member is in `phase` (the launches that move its blocks), taken
// by the member's first item before any state can change.
__device__ inline void count_launch(const RbProb& P, const RbWork& w, int phase, int slot) {
  if (P.rb.prof && w.first && threadIdx.x == 0) {
    for (int r = 0; r < P.pr.R; ++r) {
      if (P.pr.st[r].phase == phase) {
        atomicAdd((unsigned long long*)&P.rb.prof[slot], 1ull);
        break;
      }
    }
  }
}

// Where the split writes the first refinement of a zero start value (r, p of
// the item's right-hand sides, and the refinement partials of right-hand side
// r0 + r of the solve); r == nullptr: not taken.
template <typename T>
struct RbFirst {
  T* r;
  T* p;
  double* part;
  size_t vstride;
  int pstride, r0;
};

// Right-hand sides the refinement step works on: those in the outer phase,
// except the first step from a zero start value, which the split takes.
__device__ __forceinline__ bool refine_active(const RbDev& rb, const RhsState& s) {
  return s.phase == PH_OUTER && !(rb.zero_start && s.outer == 0);
}
// A voxel's packed symmetric K x K block, held in registers across the
// right-hand sides of a work item when HOLD, else read per use.
template <typename T, int K, bool HOLD>
struct Packed {
  Slab<T> s;
  unsigned o;
  T v[HOLD ? Tri<K>::NB : 1];
  __device__ __forceinline__ Packed(const T* base, int n, unsigned off) : s(base, Tri<K>::NB, n), o(off) {
    if constexpr (HOLD) {
#pragma unroll
      for (int e = 0; e < Tri<K>::NB; ++e) v[e] = s.ld(e, o);
    }
  }
  __device__ __forceinline__ T operator()(int e) const {
    if constexpr (HOLD)
      return v[e];
    else
      return s.ld(e, o);
  }
};
// Hold NBLK blocks when they take at most 96 registers.
template <typename T, int K, int NBLK> struct HoldRb {
  static constexpr bool v = NBLK * Tri<K>::NB * (int)sizeof(T) <= 384;
};

// One right-hand side's [K][n] vector of T (right-hand side r of a batch starts
// at r * K * n), a voxel's K values moved together: a kernel issues all loads
// of a voxel before its first store, since a wait for a load also waits for
// every store issued before it (one counter for both).
template <typename T, int K> struct RbVec {
  Slab<T> s;
  __device__ __forceinline__ RbVec(const T* base, int n) : s(base, K, n) {}
  __device__ __forceinline__ void load(int i, T (&v)[K]) const {
    const unsigned o = (unsigned)i * (unsigned)sizeof(T);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = s.ld(k, o);
  }
  __device__ __forceinline__ void store(int i, const T (&v)[K]) const {
    const unsigned o = (unsigned)i * (unsigned)sizeof(T);
#pragma unroll
    for (int k = 0; k < K; ++k) s.st(k, o, v[k]);
  }
};

// sum over the six neighbour slots of the vector v, a missing neighbour (-1)
// contributing zero (branch free, as neighbour_sum)
template <typename T, int K>
__device__ __forceinline__ void neighbour_sum_v(const int (&nb)[6], const RbVec<T, K>& v, T (&s)[K]) {
  neighbour_sum<T, K>(nb, v.s, s);
}

// The red-stage vector u of an FP32 inner solve of two or more right-hand
// sides stores them in pairs, [ceil(R/2)][K][NR][2]: row k of red position j
// holds (u_{2h}, u_{2h+1}) in 8 bytes, so the black stage gathers a pair's two
// values with one access per neighbour and row (half the gather instructions
// of two separate rows).  A single right-hand side keeps [K][NR] (pair width
// 1: its gathers stay contiguous), and so do FP64 inner vectors and K above
// UPAIR_KMAX (where a pair's gathers would not fit in registers).
template <typename T, int K> struct UPaired {
  static constexpr bool v = sizeof(T) == 4 && K <= UPAIR_KMAX;
};

template <int K> struct UPairs {
  Rsrc rs;
  unsigned row;   // NR * 4 * width bytes
  unsigned sh;    // log2 of the pair width (0 or 1)
  // the pair (or single row set) holding right-hand side r; w: pair width
  __device__ __forceinline__ UPairs(const float* u, int r, int NR, int w)
      : rs(make_rsrc(u + (size_t)(r >> (w >> 1)) * K * NR * w, (size_t)K * NR * 4 * w)),
        row((unsigned)NR * 4u * (unsigned)w), sh((unsigned)w >> 1) {}
  // both values of row k at red position j (pair width 2)
  __device__ __forceinline__ void ld2(int k, int j, float& a, float& b) const {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (unsigned)j * 8u, (unsigned)k * row, 0);
    // the elements copied out first: a bit cast of a vector element in place
    // reads the vector's first element
    const unsigned lo = v[0], hi = v[1];
    a = __builtin_bit_cast(float, lo);
    b = __builtin_bit_cast(float, hi);
  }
  // the value of right-hand side 2h + half alone (half = 0 at width 1)
  __device__ __forceinline__ float ld1(int k, int j, int half) const {
    return bload<float>(rs, ((unsigned)j << (2u + sh)) + 4u * (unsigned)half, (unsigned)k * row);
  }
  __device__ __forceinline__ void st2(int k, int j, float a, float b) const {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
    V2 v;
    v[0] = __builtin_bit_cast(unsigned, a);
    v[1] = __builtin_bit_cast(unsigned, b);
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (unsigned)j * 8u, (unsigned)k * row, 0);
  }
  __device__ __forceinline__ void st1(int k, int j, int half, float a) const {
    bstore(rs, ((unsigned)j << (2u + sh)) + 4u * (unsigned)half, (unsigned)k * row, a);
  }
};

// neighbour_sum over both right-hand sides of a pair (the additions in
// neighbour_sum's order, so each sum is bitwise the single one's)
template <int K>
__device__ __forceinline__ void neighbour_sum_pair(const int (&nb)[6], const UPairs<K>& u, float (&s0)[K],
                                                   float (&s1)[K]) {
  float t0[6][K], t1[6][K];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int j = nb[d] < 0 ? 0 : nb[d];
#pragma unroll
    for (int k = 0; k < K; ++k) u.ld2(k, j, t0[d][k], t1[d][k]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) s0[k] = s1[k] = 0.0f;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s0[k] += nb[d] < 0 ? 0.0f : t0[d][k];
      s1[k] += nb[d] < 0 ? 0.0f : t1[d][k];
    }
  }
}

// neighbour_sum of right-hand side 2h + half of a pair alone
template <int K>
__device__ __forceinline__ void neighbour_sum_half(const int (&nb)[6], const UPairs<K>& u, int half,
                                                   float (&s)[K]) {
  float t[6][K];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int j = nb[d] < 0 ? 0 : nb[d];
#pragma unroll
    for (int k = 0; k < K; ++k) t[d][k] = u.ld1(k, j, half);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0.0f;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] += nb[d] < 0 ? 0.0f : t[d][k];
  }
}

__device__ __forceinline__ void load_nb(const int* tab, int n, int i, int (&nb)[6]) {
#pragma unroll
  for (int d = 0; d < 6; ++d) nb[d] = tab[(size_t)d * n + i];
}

// ------------------------------------------------------------------ set-up
// Red voxels: the packed inverse of Q_nn = B_n + diag(alpha) deg_n.
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_setup_red(RbDev rb, const double* __restrict__ B64,
                                                       double* __restrict__ P64, float* __restrict__ P32,
                                                       int* __restrict__ bad) {
  constexpr int NB = Tri<K>::NB;
  const int j = blockIdx.x * TILE + threadIdx.x;
  if (j >= rb.NR) return;
  const int n = rb.red[j];
  int deg = 0;
  for (int d = 0; d < 6; ++d) deg += rb.nbR[(size_t)d * rb.NR + j] >= 0;
  double a[NB], inv[NB];
  load_soa(B64, rb.N, n, a);
#pragma unroll
  for (int k = 0; k < K; ++k) a[pk(k, k)] += rb.alpha64[k] * (double)deg;
  const bool ok = spd_inverse_any<K>(a, inv);
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    P64[(size_t)i * rb.NR + j] = inv[i];
    P32[(size_t)i * rb.NR + j] = (float)inv[i];
  }
  if (!ok) atomicMin(bad, n);
}

// Black voxels: Q_mm packed, and the packed inverse of the Schur block
// S_m = Q_mm - sum_{n ~ m} diag(alpha) Q_nn^{-1} diag(alpha) (reads the red
// inverses written by k_rb_setup_red).
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_setup_black(RbDev rb, const double* __restrict__ B64,
                                                         double* __restrict__ D64, float* __restrict__ D32,
                                                         double* __restrict__ S64, float* __restrict__ S32,
                                                         int* __restrict__ bad) {
  constexpr int NB = Tri<K>::NB;
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= rb.NB) return;
  const int m = rb.blk[i];
  int nb[6];
  load_nb(rb.nbB, rb.NB, i, nb);
  int deg = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) deg += nb[d] >= 0;
  double a[NB], inv[NB];
  load_soa(B64, rb.N, m, a);
#pragma unroll
  for (int k = 0; k < K; ++k) a[pk(k, k)] += rb.alpha64[k] * (double)deg;
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    D64[(size_t)e * rb.NB + i] = a[e];
    D32[(size_t)e * rb.NB + i] = (float)a[e];
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if (nb[d] < 0) continue;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int l = 0; l <= k; ++l)
        a[pk(k, l)] -= rb.alpha64[k] * rb.alpha64[l] * rb.P64[(size_t)pk(k, l) * rb.NR + nb[d]];
    }
  }
  const bool ok = spd_inverse_any<K>(a, inv);
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    S64[(size_t)e * rb.NB + i] = inv[e];
    S32[(size_t)e * rb.NB + i] = (float)inv[e];
  }
  if (!ok) atomicMin(bad, m);
}

// ------------------------------------------------------------------ solve
// Split, in voxel order (reads of b and x coalesced): red voxels t = Q_nn^{-1}
// b_n, black voxels c = b_m and x_B = x_m (x_B not written for a zero start
// value); the per-tile partials of ||b||^2 into bbpart[r][tile].
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_split_voxels(RbDev rb, int R, int rc, const double* __restrict__ b,
                                                          const double* __restrict__ x, int zero_guess,
                                                          double* __restrict__ t, double* __restrict__ c,
                                                          double* __restrict__ xB, double* __restrict__ bbpart) {
  const int n = blockIdx.x * TILE + threadIdx.x;
  const int r0 = blockIdx.y * rc, r1 = min(R, r0 + rc);
  const bool valid = n < rb.N;
  const int nn = valid ? n : rb.N - 1;   // lanes past the end compute on the last voxel and store nothing
  const unsigned on = (unsigned)nn * 8u;
  const int vp = rb.vpos[nn], pos = vp >> 1;
  const bool red = (vp & 1) == 0;
  const unsigned op = (unsigned)pos * 8u;
  // the red inverse, held across the work item's right-hand sides (black
  // lanes hold red block 0 and do not use it)
  const Packed<double, K, HoldRb<double, K, 1>::v> P(rb.P64, rb.NR, red ? op : 0u);
  ItemSums<1> sums;
#pragma unroll 1
  for (int r = r0; r < r1; ++r) {
    const size_t ur = (size_t)r * K * rb.N;
    const Slab<double> bs(b + ur, K, rb.N);
    double acc[1] = {0.0}, bv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      bv[k] = bs.ld(k, on);
      acc[0] += bv[k] * bv[k];
    }
    if (!valid) acc[0] = 0.0;
    if (red) {
      double tv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) tv[k] = 0.0;
      sym_apply<K>(P, bv, tv);
      if (valid) {
        const Slab<double> ts(t + (size_t)r * K * rb.NR, K, rb.NR);
#pragma unroll
        for (int k = 0; k < K; ++k) ts.st(k, op, tv[k]);
      }
    } else if (valid) {
      const Slab<double> cs(c + (size_t)r * K * rb.NB, K, rb.NB);
#pragma unroll
      for (int k = 0; k < K; ++k) cs.st(k, op, bv[k]);
      if (!zero_guess) {   // from a zero start value x_B is first written by x_B = d (+ a p)
        const Slab<double> xu(x + ur, K, rb.N), xs(xB + (size_t)r * K * rb.NB, K, rb.NB);
        double xv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) xv[k] = xu.ld(k, on);
#pragma unroll
        for (int k = 0; k < K; ++k) xs.st(k, op, xv[k]);
      }
    }
    sums.add(r - r0, acc);
  }
  sums.flush(bbpart, 0, r0, r1 - r0, rb.ntN, blockIdx.x);
}

// Black voxels: c += alpha .* sum_{n ~ m} t_n, which makes
// c = b_B - E' D_R^{-1} b_R.
template <int K, typename T>
__global__ __launch_bounds__(TILE) void k_rb_split_black(RbDev rb, int R, int rc, const double* __restrict__ t,
                                                         double* __restrict__ c, RbFirst<T> first) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  const int r0 = blockIdx.y * rc, r1 = min(R, r0 + rc);
  const bool valid = i < rb.NB;
  const int ii = valid ? i : 0;   // lanes past the end compute on voxel 0 and store nothing
  int nb[6];
  load_nb(rb.nbB, rb.NB, ii, nb);
  const unsigned oi = (unsigned)ii * 8u, oT = (unsigned)ii * (unsigned)sizeof(T);
  // the Schur inverse for the first refinement, held across the work item
  const Packed<T, K, HoldRb<T, K, 1>::v> S(RbT<T>::S(rb), rb.NB, oT);
  ItemSums<3> sums;
#pragma unroll 1
  for (int r = r0; r < r1; ++r) {
    const Slab<double> ts(t + (size_t)r * K * rb.NR, K, rb.NR), cs(c + (size_t)r * K * rb.NB, K, rb.NB);
    double s[K], cv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) cv[k] = cs.ld(k, oi);
    neighbour_sum<double, K>(nb, ts, s);
#pragma unroll
    for (int k = 0; k < K; ++k) cv[k] += rb.alpha64[k] * s[k];
    if (valid) {
#pragma unroll
      for (int k = 0; k < K; ++k) cs.st(k, oi, cv[k]);
    }
    if (first.r) {
      // the first refinement from x_B = 0: its residual is c itself
      double acc[3] = {0.0, 0.0, 0.0};
      T rt[K], zt[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        acc[0] += cv[k] * cv[k];
        rt[k] = (T)cv[k];
        zt[k] = 0;
      }
      sym_apply<K>(S, rt, zt);
#pragma unroll
      for (int k = 0; k < K; ++k) acc[2] += (double)rt[k] * (double)zt[k];
      if (valid) {
        RbVec<T, K>(first.r + (size_t)r * K * rb.NB, rb.NB).store(ii, rt);
        RbVec<T, K>(first.p + (size_t)r * K * rb.NB, rb.NB).store(ii, zt);
      } else {
        acc[0] = acc[2] = 0.0;
      }
      sums.add(r - r0, acc);
    }
  }
  if (first.r) sums.flush(first.part, first.vstride, first.r0 + r0, r1 - r0, first.pstride, blockIdx.x);
}

// Right-hand side r takes part in the red stage of phase `want` (nothing to do
// for the first refinement from a zero start value: S 0 = 0).
__device__ __forceinline__ bool red_active(const RbDev& rb, const RhsState& s, int want) {
  return s.phase == want && !(want == PH_OUTER && rb.zero_start && s.outer == 0);
}

// Red stage of S v: u_n = Q_nn^{-1} (alpha .* sum_{m ~ n} v_m) at the red voxels,
// for the right-hand sides of an inner step (v = p, u in the inner precision)
// or, with OUTER, of the FP64 refinement (v = x_B, u = u64; T = double).
template <typename T, int K, bool HOLD, bool OUTER>
__global__ __launch_bounds__(TILE) void k_rb_red(const RbProb* __restrict__ probs, int nprob) {
  static_assert(!OUTER || sizeof(T) == 8, "the refinement's red stage is FP64");
  const RbWork w = rb_item<RBW_RED>(probs, nprob);
  const RbProb& P = probs[w.p];
  const RbDev& rb = P.rb;
  const RhsState* st = P.pr.st;
  const int want = OUTER ? PH_OUTER : PH_INNER;
  const int j = w.tile * TILE + threadIdx.x;
  bool any = false;
  for (int r = w.r0; r < w.r1; ++r) any = any || red_active(rb, st[r], want);
  if (!any || j >= rb.NR) return;
  const T* v = OUTER ? (const T*)P.xB : (const T*)P.p;
  T* u = OUTER ? (T*)P.u64 : (T*)P.u;
  int nb[6];
  load_nb(rb.nbR, rb.NR, j, nb);
  const unsigned oj = (unsigned)j * (unsigned)sizeof(T);
  const Packed<T, K, HOLD> Pn(RbT<T>::P(rb), rb.NR, oj);
  // y = Q_nn^{-1} (alpha .* sum_{m ~ n} v_m) for right-hand side r
  auto stage = [&](int r, T (&y)[K]) {
#pragma clang fp contract(off)
    const RbVec<T, K> vs(v + (size_t)r * K * rb.NB, rb.NB);
    T s[K];
    neighbour_sum_v<T, K>(nb, vs, s);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s[k] *= RbT<T>::alpha(rb, k);
      y[k] = 0;
    }
    sym_apply<K>(Pn, s, y);
  };
  if constexpr (!OUTER && UPaired<T, K>::v) {
    // both right-hand sides of a pair in the item: one 8-byte store per row
    // (an inactive partner's half written as zero: no kernel reads it before
    // its next red stage)
#pragma unroll 1
    for (int r = w.r0; r < w.r1;) {
      const UPairs<K> up((const float*)u, r, rb.NR, P.uw);
      const int half = r & (P.uw - 1);
      if (P.uw == 2 && half == 0 && r + 1 < w.r1) {
        const bool a0 = red_active(rb, st[r], want), a1 = red_active(rb, st[r + 1], want);
        if (a0 || a1) {
          T y0[K], y1[K];
          if (a0) {
            stage(r, y0);
          } else {
#pragma unroll
            for (int k = 0; k < K; ++k) y0[k] = 0;
          }
          if (a1) {
            stage(r + 1, y1);
          } else {
#pragma unroll
            for (int k = 0; k < K; ++k) y1[k] = 0;
          }
#pragma unroll
          for (int k = 0; k < K; ++k) up.st2(k, j, y0[k], y1[k]);
        }
        r += 2;
      } else {
        if (red_active(rb, st[r], want)) {
          T y[K];
          stage(r, y);
#pragma unroll
          for (int k = 0; k < K; ++k) up.st1(k, j, half, y[k]);
        }
        r += 1;
      }
    }
  } else {
#pragma unroll 1
    for (int r = w.r0; r < w.r1; ++r) {
      if (!red_active(rb, st[r], want)) continue;
      T y[K];
      stage(r, y);
      RbVec<T, K>(u + (size_t)r * K * rb.NR, rb.NR).store(j, y);
    }
  }
}

// FP64 refinement at the black voxels of right-hand sides waiting on it:
// r64 = c - S x_B (u64 from the red stage on x_B), r = T(r64),
// p = blkdiag(S)^{-1} r in the inner precision (p only starts the next inner
// solve); partials ||r64||^2 (slot 0) and r'p (slot 2).
template <typename T, int K, bool HOLD>
__global__ __launch_bounds__(TILE) void k_rb_refine(const RbProb* __restrict__ probs, int nprob) {
  const RbWork w = rb_item<RBW_OUTER>(probs, nprob);
  const RbProb& P = probs[w.p];
  const RbDev& rb = P.rb;
  const RhsState* st = P.pr.st;
  if (rb.prof && w.first && threadIdx.x == 0) {
    bool act = false;
    for (int r = 0; r < P.pr.R; ++r) act = act || refine_active(rb, st[r]);
    if (act) atomicAdd((unsigned long long*)&rb.prof[PF_REFINE_ACT], 1ull);
  }
  bool any = false;
  for (int r = w.r0; r < w.r1; ++r) any = any || refine_active(rb, st[r]);
  if (!any) return;
  const int R = P.pr.R, pstride = P.pr.pstride;
  const int i = w.tile * TILE + threadIdx.x;
  const bool valid = i < rb.NB;
  const int ii = valid ? i : 0;   // lanes past the end compute on voxel 0 and contribute nothing
  int nb[6];
  load_nb(rb.nbB, rb.NB, ii, nb);
  const unsigned o8 = (unsigned)ii * 8u, oT = (unsigned)ii * (unsigned)sizeof(T);
  const Packed<double, K, HOLD> D(rb.D64, rb.NB, o8);
  const Packed<T, K, HOLD> S(RbT<T>::S(rb), rb.NB, oT);
  ItemSums<3> sums;
#pragma unroll 1
  for (int r = w.r0; r < w.r1; ++r) {
    const RhsState& sr = st[r];
    if (!refine_active(rb, sr)) continue;
    const size_t off = (size_t)r * K * rb.NB;
    const Slab<double> cs(P.c64 + off, K, rb.NB), xs(P.xB + off, K, rb.NB),
        us(P.u64 + (size_t)r * K * rb.NR, K, rb.NR);
    const RbVec<T, K> rs((T*)P.r + off, rb.NB), ps((T*)P.p + off, rb.NB);
    double r64[K];
    {
      double xv[K], y[K], s[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        xv[k] = xs.ld(k, o8);
        y[k] = 0.0;
      }
      sym_apply<K>(D, xv, y);
      neighbour_sum<double, K>(nb, us, s);
#pragma unroll
      for (int k = 0; k < K; ++k) r64[k] = cs.ld(k, o8) - (y[k] - rb.alpha64[k] * s[k]);
    }
    double acc[3] = {0.0, 0.0, 0.0};
    T rt[K], zt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[0] += r64[k] * r64[k];
      rt[k] = (T)r64[k];
      zt[k] = 0;
    }
    sym_apply<K>(S, rt, zt);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[2] += (double)rt[k] * (double)zt[k];
    if (valid) {
      rs.store(ii, rt);
      ps.store(ii, zt);
    } else {
      acc[0] = acc[2] = 0.0;
    }
    sums.add(r - w.r0, acc);
  }
  sums.flush(P.pr.part, (size_t)R * pstride, w.r0, w.r1 - w.r0, pstride, w.tile);
}

// The black stage at voxel ii for one right-hand side, given the neighbour sum
// s = sum_{n ~ m} u_n: q = Q_mm p - alpha .* s (stored), and the seven inner
// products of the one-reduction iteration with z = blkdiag(S)^{-1} r and
// t = blkdiag(S)^{-1} q at the voxel: p'q, r'z, q'z, q't, r'r, q'r, q'q.
template <typename T, int K, typename BD, typename BS>
__device__ __forceinline__ void black_stage(const RbDev& rb, const BD& D, const BS& S, const T (&p)[K],
                                            const T (&rr)[K], const T (&s)[K], bool valid, int ii,
                                            const RbVec<T, K>& qs, double (&acc)[7]) {
  // products and sums written out as fused multiply-adds, nothing contracted
  // by the compiler: the result is the same in every path that calls this
#pragma clang fp contract(off)
  T y[K], q[K], z[K], t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) y[k] = 0;
  sym_apply<K>(D, p, y);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    q[k] = fma_of(-RbT<T>::alpha(rb, k), s[k], y[k]);
    z[k] = t[k] = 0;
  }
  if (valid) qs.store(ii, q);
  sym_apply<K>(S, rr, z);
  sym_apply<K>(S, q, t);
  T a[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    a[0] = fma_of(p[k], q[k], a[0]);
    a[1] = fma_of(rr[k], z[k], a[1]);
    a[2] = fma_of(q[k], z[k], a[2]);
    a[3] = fma_of(q[k], t[k], a[3]);
    a[4] = fma_of(rr[k], rr[k], a[4]);
    a[5] = fma_of(q[k], rr[k], a[5]);
    a[6] = fma_of(q[k], q[k], a[6]);
  }
#pragma unroll
  for (int e = 0; e < 7; ++e) acc[e] = valid ? (double)a[e] : 0.0;
}

// Black stage of q = S p after a separate red stage (u read from memory).
// HOLD: the voxel blocks held in registers across the work item's
// right-hand sides, 2 = Q_mm and S_m^{-1}, 1 = S_m^{-1} only (it is applied
// twice per right-hand side), 0 = neither.  PAIRS: some member of the launch
// stores u in pairs (the pair and single paths; without, the fewer registers
// of the single path alone).
template <typename T, int K, int HOLD, bool PAIRS>
__global__ __launch_bounds__(TILE) void k_rb_matvec(const RbProb* __restrict__ probs, int nprob) {
  const RbWork w = rb_item<RBW_BLACK>(probs, nprob);
  const RbProb& P = probs[w.p];
  const RbDev& rb = P.rb;
  const RhsState* st = P.pr.st;
  count_launch(P, w, PH_INNER, PF_MATVEC_ACT);
  bool any = false;
  for (int r = w.r0; r < w.r1; ++r) any = any || st[r].phase == PH_INNER;
  if (!any) return;
  const int R = P.pr.R, pstride = P.pr.pstride;
  const int i = w.tile * TILE + threadIdx.x;
  const bool valid = i < rb.NB;
  const int ii = valid ? i : 0;
  int nb[6];
  load_nb(rb.nbB, rb.NB, ii, nb);
  const unsigned oT = (unsigned)ii * (unsigned)sizeof(T);
  const Packed<T, K, (HOLD >= 2)> D(RbT<T>::D(rb), rb.NB, oT);
  const Packed<T, K, (HOLD >= 1)> S(RbT<T>::S(rb), rb.NB, oT);
  ItemSums<7> sums;
  auto vec = [&](const void* base, int r) { return RbVec<T, K>((const T*)base + (size_t)r * K * rb.NB, rb.NB); };
  auto qvec = [&](int r) { return RbVec<T, K>((T*)P.q + (size_t)r * K * rb.NB, rb.NB); };
#pragma unroll 1
  for (int r = w.r0; r < w.r1;) {
    if constexpr (PAIRS) {
      // a pair with both right-hand sides in the item and in the inner phase
      // gathers u once for the two
      const int half = r & (P.uw - 1);
      const bool pair = P.uw == 2 && half == 0 && r + 1 < w.r1;
      const bool a0 = st[r].phase == PH_INNER, a1 = pair && st[r + 1].phase == PH_INNER;
      const UPairs<K> up((const float*)P.u, r, rb.NR, P.uw);
      if (a0 && a1) {
        T p0[K], r0[K], p1[K], r1[K], s0[K], s1[K];
        vec(P.p, r).load(ii, p0);
        vec(P.r, r).load(ii, r0);
        vec(P.p, r + 1).load(ii, p1);
        vec(P.r, r + 1).load(ii, r1);
        neighbour_sum_pair<K>(nb, up, s0, s1);
        double acc[7];
        black_stage<T, K>(rb, D, S, p0, r0, s0, valid, ii, qvec(r), acc);
        sums.add(r - w.r0, acc);
        black_stage<T, K>(rb, D, S, p1, r1, s1, valid, ii, qvec(r + 1), acc);
        sums.add(r + 1 - w.r0, acc);
      } else if (a0 || a1) {
        // the same in every lane (states are per right-hand side)
        const int ra = __builtin_amdgcn_readfirstlane(a0 ? r : r + 1);
        T p[K], rr[K], s[K];
        vec(P.p, ra).load(ii, p);
        vec(P.r, ra).load(ii, rr);
        neighbour_sum_half<K>(nb, up, ra & (P.uw - 1), s);
        double acc[7];
        black_stage<T, K>(rb, D, S, p, rr, s, valid, ii, qvec(ra), acc);
        sums.add(ra - w.r0, acc);
      }
      r += pair ? 2 : 1;
    } else {
      if (st[r].phase == PH_INNER) {
        const RbVec<T, K> us((const T*)P.u + (size_t)r * K * rb.NR, rb.NR);
        T p[K], rr[K], s[K];
        vec(P.p, r).load(ii, p);
        vec(P.r, r).load(ii, rr);
        neighbour_sum_v<T, K>(nb, us, s);
        double acc[7];
        black_stage<T, K>(rb, D, S, p, rr, s, valid, ii, qvec(r), acc);
        sums.add(r - w.r0, acc);
      }
      r += 1;
    }
  }
  sums.flush(P.pr.part, (size_t)R * pstride, w.r0, w.r1 - w.r0, pstride, w.tile);
}

// d += a p (d = a p on the first step), r -= a q, p = blkdiag(S)^{-1} r + beta p.
template <typename T, int K, bool HOLD>
__global__ __launch_bounds__(TILE) void k_rb_update(const RbProb* __restrict__ probs, int nprob) {
  const RbWork w = rb_item<RBW_BLACK>(probs, nprob);
  const RbProb& P = probs[w.p];
  const RbDev& rb = P.rb;
  const RhsState* st = P.pr.st;
  count_launch(P, w, PH_INNER, PF_UPDATE_ACT);
  const int i = w.tile * TILE + threadIdx.x;
  bool any = false;
  for (int r = w.r0; r < w.r1; ++r) any = any || st[r].phase == PH_INNER;
  if (!any || i >= rb.NB) return;
  const unsigned oT = (unsigned)i * (unsigned)sizeof(T);
  const Packed<T, K, HOLD> S(RbT<T>::S(rb), rb.NB, oT);
#pragma unroll 1
  for (int r = w.r0; r < w.r1; ++r) {
    const RhsState& s = st[r];
    if (s.phase != PH_INNER) continue;
    const T a = (T)s.a, beta = (T)s.beta;
    const bool fresh = s.inner_it == 1;
    const size_t off = (size_t)r * K * rb.NB;
    const RbVec<T, K> ds((T*)P.d + off, rb.NB), rs((T*)P.r + off, rb.NB), ps((T*)P.p + off, rb.NB),
        qs((T*)P.q + off, rb.NB);
    T p[K], dd[K], rn[K], q[K], z[K];
    ps.load(i, p);
    rs.load(i, rn);
    qs.load(i, q);
    if (fresh) {
#pragma unroll
      for (int k = 0; k < K; ++k) dd[k] = a * p[k];
    } else {
      ds.load(i, dd);
#pragma unroll
      for (int k = 0; k < K; ++k) dd[k] += a * p[k];
    }
    ds.store(i, dd);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      rn[k] -= a * q[k];
      z[k] = 0;
    }
    rs.store(i, rn);
    sym_apply<K>(S, rn, z);
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] += beta * p[k];
    ps.store(i, z);
  }
}

// x_B += d (when valid) + a p (when the last step is pending) for right-hand
// sides whose inner solve has ended.
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_rb_addsol(const RbProb* __restrict__ probs, int nprob) {
  const RbWork w = rb_item<RBW_OUTER>(probs, nprob);
  const RbProb& P = probs[w.p];
  const RbDev& rb = P.rb;
  const RhsState* st = P.pr.st;
  const int i = w.tile * TILE + threadIdx.x;
  if (i >= rb.NB) return;
  const unsigned o8 = (unsigned)i * 8u;
#pragma unroll 1
  for (int r = w.r0; r < w.r1; ++r) {
    const RhsState& s = st[r];
    // with a zero start value, the first x_B += d writes x_B without reading it
    const bool fresh = rb.zero_start && s.outer == 1;
    if (s.phase != PH_OUTER || !(s.has_d || s.pend || fresh)) continue;
    const bool hd = s.has_d != 0, hp = s.pend != 0;
    const double a = s.a;
    const Slab<double> xs(P.xB + (size_t)r * K * rb.NB, K, rb.NB);
    const RbVec<T, K> ds((const T*)P.d + (size_t)r * K * rb.NB, rb.NB), ps((const T*)P.p + (size_t)r * K * rb.NB, rb.NB);
    T dt[K], pt[K];
    double v[K];
    if (hd) ds.load(i, dt);
    if (hp) ps.load(i, pt);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = fresh ? 0.0 : xs.ld(k, o8);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (hd) v[k] += (double)dt[k];
      if (hp) v[k] += a * (double)pt[k];
      xs.st(k, o8, v[k]);
    }
  }
}

// Writes the solution in the caller's layout, in voxel order (writes of x
// coalesced): x_m = x_B at the black voxels, x_n = Q_nn^{-1} (b_n + alpha .*
// sum_{m ~ n} x_m) = t_n + u_n at the red ones, t = Q_nn^{-1} b_n from the
// split and u = Q_nn^{-1} (alpha .* sum x_m) from the red stage of the last
// outer step (which followed the last change of x_B); zero for b = 0.
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_recover(RbDev rb, const RhsState* __restrict__ st,
                                                     const double* __restrict__ t, const double* __restrict__ u64,
                                                     const double* __restrict__ xB, double* __restrict__ x) {
  const int r = blockIdx.y, n = blockIdx.x * TILE + threadIdx.x;
  if (n >= rb.N) return;
  const bool zero = st[r].zero_b != 0;
  // from a zero start value, x_B holds nothing (and u was not formed) until
  // the first x_B += d
  const bool xzero = rb.zero_start && st[r].outer <= 1;
  const Slab<double> xs(xB + (size_t)r * K * rb.NB, K, rb.NB), xu(x + (size_t)r * K * rb.N, K, rb.N);
  const unsigned on = (unsigned)n * 8u;
  const int vp = rb.vpos[n], pos = vp >> 1;
  const unsigned op = (unsigned)pos * 8u;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  if (zero) {
  } else if (vp & 1) {   // black
    if (!xzero) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = xs.ld(k, op);
    }
  } else {               // red
    const Slab<double> ts(t + (size_t)r * K * rb.NR, K, rb.NR), us(u64 + (size_t)r * K * rb.NR, K, rb.NR);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = ts.ld(k, op);
    if (!xzero) {
      double u[K];
#pragma unroll
      for (int k = 0; k < K; ++k) u[k] = us.ld(k, op);
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] += u[k];
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) xu.st(k, on, v[k]);
}

// One wavefront per right-hand side of a member: reduce its black tiles'
// partials in a fixed order and advance the state with the main solver's
// rules.  For the refinement the ||b||^2 slot comes from the split partials
// (ntN voxel tiles).
template <int KIND>
__global__ __launch_bounds__(FIN_WAVES * WAVE) void k_rb_finalize(const RbProb* __restrict__ probs, int nprob) {
  const int b = blockIdx.x;
  int p = 0;
  while (p + 1 < nprob && b >= probs[p + 1].pr.fin_begin) ++p;
  const RbProb& P = probs[p];
  const Prob& pr = P.pr;
  const int r = (b - pr.fin_begin) * FIN_WAVES + (int)(threadIdx.x / WAVE);
  if (r >= pr.R) return;
  if (pr.st[r].phase != (KIND == 0 ? PH_OUTER : PH_INNER)) return;
  const int lane = threadIdx.x % WAVE;
  const int ntB = P.rb.ntB, ntN = P.rb.ntN;
  if constexpr (KIND == 0) {
    double v[3], bb[1];
    sum_partials<3>(pr.part, pr.R, pr.pstride, ntB, r, v);
    sum_partials<1>(P.bb, 1, ntN, ntN, r, bb);
    v[1] = bb[0];
    if (lane == 0) finalize_refine(pr, r, v);
  } else {
    double v[7];
    sum_partials<7>(pr.part, pr.R, pr.pstride, ntB, r, v);
    if (lane == 0) finalize_matvec(pr, r, v);
  }
}

inline dim3 grid2(int tiles, int R) { return dim3((unsigned)tiles, (unsigned)R); }

}  // namespace

#define RB_K_SWITCH(K, X)                                                                            \
  switch (K) {                                                                                       \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) \
        X(19) X(20) X(21) X(22) X(23) X(24)                                                            \
    default: return hipErrorInvalidValue;                                                            \
  }

// Grouped launches over the nprob members (device descriptors) of one K
// group; W = the launch's work items.  Blocks are held in registers across a
// work item's right-hand sides where NBLK of them fit (HoldRb).
#define RB_HOLD_LAUNCH(KERN, KK, NBLK, TB, ...)                                  \
  do {                                                                           \
    if constexpr (HoldRb<TB, KK, NBLK>::v)                                       \
      GP_LAUNCH((KERN<T, KK, true>), __VA_ARGS__);                      \
    else                                                                         \
      GP_LAUNCH((KERN<T, KK, false>), __VA_ARGS__);                     \
  } while (0)

template <typename T>
hipError_t launch_rbg_red_t(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {
  if (W == 0) return hipSuccess;
#define X(KK)                                                                                                    \
  case KK:                                                                                                       \
    if constexpr (HoldRb<T, KK, 1>::v)                                                                           \
      GP_LAUNCH((k_rb_red<T, KK, true, false>), dim3(W), dim3(TILE), 0, s, probs, nprob);              \
    else                                                                                                         \
      GP_LAUNCH((k_rb_red<T, KK, false, false>), dim3(W), dim3(TILE), 0, s, probs, nprob);             \
    break;
  RB_K_SWITCH(K, X)
#undef X
  return hipGetLastError();
}

// The refinement reads its blocks where they are used: its work items are
// mostly one right-hand side, and holding the FP64 Q_mm and S_m^{-1} for the
// whole item cost occupancy (107 against 142 us per launch on the whole-brain
// 64-RHS solve).
template <typename T>
hipError_t launch_rbg_refine_t(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {
  if (W == 0) return hipSuccess;
#define X(KK) \
  case KK: GP_LAUNCH((k_rb_refine<T, KK, false>), dim3(W), dim3(TILE), 0, s, probs, nprob); break;
  RB_K_SWITCH(K, X)
#undef X
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rbg_matvec_t(hipStream_t s, int K, const RbProb* probs, int nprob, int W, bool pairs) {
  if (W == 0) return hipSuccess;
#define MV(KK, H)                                                                                \
  do {                                                                                           \
    if constexpr (UPaired<T, KK>::v) {                                                           \
      if (pairs) {                                                                               \
        GP_LAUNCH((k_rb_matvec<T, KK, H, true>), dim3(W), dim3(TILE), 0, s, probs, nprob);     \
        break;                                                                                   \
      }                                                                                          \
    }                                                                                            \
    GP_LAUNCH((k_rb_matvec<T, KK, H, false>), dim3(W), dim3(TILE), 0, s, probs, nprob);        \
  } while (0)
#define X(KK)                                                                                   \
  case KK:                                                                                      \
    if constexpr (HoldRb<T, KK, 2>::v)                                                          \
      MV(KK, 2);                                                                                \
    else if constexpr (HoldRb<T, KK, 1>::v)                                                     \
      MV(KK, 1);                                                                                \
    else                                                                                        \
      MV(KK, 0);                                                                                \
    break;
  RB_K_SWITCH(K, X)
#undef X
#undef MV
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rbg_update_t(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {
  if (W == 0) return hipSuccess;
#define X(KK) \
  case KK: RB_HOLD_LAUNCH(k_rb_update, KK, 1, T, dim3(W), dim3(TILE), 0, s, probs, nprob); break;
  RB_K_SWITCH(K, X)
#undef X
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rbg_addsol_t(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {
  if (W == 0) return hipSuccess;
#define X(KK) \
  case KK: GP_LAUNCH((k_rb_addsol<T, KK>), dim3(W), dim3(TILE), 0, s, probs, nprob); break;
  RB_K_SWITCH(K, X)
#undef X
  return hipGetLastError();
}

#define RB_INST(T)                                                                                          \
  template <>                                                                                               \
  hipError_t launch_rbg_red<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {              \
    return launch_rbg_red_t<T>(s, K, probs, nprob, W);                                                      \
  }                                                                                                         \
  template <>                                                                                               \
  hipError_t launch_rbg_refine<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {           \
    return launch_rbg_refine_t<T>(s, K, probs, nprob, W);                                                   \
  }                                                                                                         \
  template <>                                                                                               \
  hipError_t launch_rbg_matvec<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W, bool pairs) { \
    return launch_rbg_matvec_t<T>(s, K, probs, nprob, W, pairs);                                            \
  }                                                                                                         \
  template <>                                                                                               \
  hipError_t launch_rbg_update<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {           \
    return launch_rbg_update_t<T>(s, K, probs, nprob, W);                                                   \
  }                                                                                                         \
  template <>                                                                                               \
  hipError_t launch_rbg_addsol<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {           \
    return launch_rbg_addsol_t<T>(s, K, probs, nprob, W);                                                   \
  }
}  // namespace gp
