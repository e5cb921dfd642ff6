// Incomplete Cholesky preconditioning on the red-black voxel order (the
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
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i][wv] = v[i];
  }
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

// sum over the six neighbour slots of vector v (rows of one right-hand side),
// a missing neighbour (-1) contributing zero
template <typename T, int K>
__device__ __forceinline__ void neighbour_sum(const int (&nb)[6], const Slab<T>& v, T (&s)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if (nb[d] < 0) continue;
    const unsigned o = (unsigned)nb[d] * (unsigned)sizeof(T);
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] += v.ld(k, o);
  }
}

// While profiling: one count in `slot` per launch in which some right-hand
// side is in `phase` (the launches that move the blocks), taken by workgroup
// (0, 0) before any state can change.
__device__ inline void count_launch(const RbDev& rb, const RhsState* st, int phase, int slot) {
  if (rb.prof && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    for (int r = 0; r < (int)gridDim.y; ++r) {
      if (st[r].phase == phase) {
        atomicAdd((unsigned long long*)&rb.prof[slot], 1ull);
        break;
      }
    }
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
  const bool ok = spd_inverse<K>(a, inv);
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
  const bool ok = spd_inverse<K>(a, inv);
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    S64[(size_t)e * rb.NB + i] = inv[e];
    S32[(size_t)e * rb.NB + i] = (float)inv[e];
  }
  if (!ok) atomicMin(bad, m);
}

// ------------------------------------------------------------------ solve
// Red voxels: t = Q_nn^{-1} b_n, and the red part of ||b||^2 into
// bbpart[r][ntB + tile].
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_split_red(RbDev rb, const double* __restrict__ b,
                                                       double* __restrict__ t, double* __restrict__ bbpart) {
  const int r = blockIdx.y, j = blockIdx.x * TILE + threadIdx.x;
  double acc[1] = {0.0};
  if (j < rb.NR) {
    const int n = rb.red[j];
    const Slab<double> bs(b + (size_t)r * K * rb.N, K, rb.N), ts(t + (size_t)r * K * rb.NR, K, rb.NR);
    const Slab<double> Ps(rb.P64, Tri<K>::NB, rb.NR);
    const unsigned on = (unsigned)n * 8u, oj = (unsigned)j * 8u;
    double bv[K], tv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      bv[k] = bs.ld(k, on);
      acc[0] += bv[k] * bv[k];
    }
    packed_apply<double, K>(Ps, oj, bv, tv);
#pragma unroll
    for (int k = 0; k < K; ++k) ts.st(k, oj, tv[k]);
  }
  const int ntBR = rb.ntB + rb.ntR;
  block_sums<1>(acc, bbpart, 0, (size_t)r * ntBR + rb.ntB + blockIdx.x);
}

// Black voxels: c = b_m + alpha .* sum_{n ~ m} t_n, x_B = x_m (not written
// for a zero start value), and the black part of ||b||^2 into bbpart[r][tile].
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_split_black(RbDev rb, const double* __restrict__ b,
                                                         const double* __restrict__ x, int zero_guess,
                                                         const double* __restrict__ t, double* __restrict__ c,
                                                         double* __restrict__ xB, double* __restrict__ bbpart) {
  const int r = blockIdx.y, i = blockIdx.x * TILE + threadIdx.x;
  double acc[1] = {0.0};
  if (i < rb.NB) {
    const int m = rb.blk[i];
    int nb[6];
    load_nb(rb.nbB, rb.NB, i, nb);
    const size_t ur = (size_t)r * K * rb.N;
    const Slab<double> bs(b + ur, K, rb.N), ts(t + (size_t)r * K * rb.NR, K, rb.NR);
    const Slab<double> cs(c + (size_t)r * K * rb.NB, K, rb.NB), xs(xB + (size_t)r * K * rb.NB, K, rb.NB);
    const unsigned om = (unsigned)m * 8u, oi = (unsigned)i * 8u;
    double s[K];
    neighbour_sum<double, K>(nb, ts, s);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double bk = bs.ld(k, om);
      acc[0] += bk * bk;
      cs.st(k, oi, bk + rb.alpha64[k] * s[k]);
    }
    if (!zero_guess) {   // from a zero start value x_B is first written by x_B = d (+ a p)
      const Slab<double> xu(x + ur, K, rb.N);
#pragma unroll
      for (int k = 0; k < K; ++k) xs.st(k, oi, xu.ld(k, om));
    }
  }
  const int ntBR = rb.ntB + rb.ntR;
  block_sums<1>(acc, bbpart, 0, (size_t)r * ntBR + blockIdx.x);
}

// Red stage of S v for right-hand sides in phase `want`:
// u_n = Q_nn^{-1} (alpha .* sum_{m ~ n} v_m).
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_rb_red(const RbDev* __restrict__ rbp, const RhsState* __restrict__ st, int want,
                                                 const T* __restrict__ v, T* __restrict__ u) {
  const RbDev& rb = *rbp;
  const int r = blockIdx.y, j = blockIdx.x * TILE + threadIdx.x;
  if (st[r].phase != want || j >= rb.NR) return;
  if (want == PH_OUTER && rb.zero_start && st[r].outer == 0) return;   // x_B = 0: S x_B = 0
  int nb[6];
  load_nb(rb.nbR, rb.NR, j, nb);
  const Slab<T> vs(v + (size_t)r * K * rb.NB, K, rb.NB), us(u + (size_t)r * K * rb.NR, K, rb.NR);
  const Slab<T> Ps(RbT<T>::P(rb), Tri<K>::NB, rb.NR);
  const unsigned oj = (unsigned)j * (unsigned)sizeof(T);
  T s[K], y[K];
  neighbour_sum<T, K>(nb, vs, s);
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] *= RbT<T>::alpha(rb, k);
  packed_apply<T, K>(Ps, oj, s, y);
#pragma unroll
  for (int k = 0; k < K; ++k) us.st(k, oj, y[k]);
}

// FP64 refinement at the black voxels of right-hand sides waiting on it:
// r64 = c - S x_B (u64 from the red stage on x_B), r = T(r64),
// p = T(blkdiag(S)^{-1} r64); partials ||r64||^2 (slot 0) and r64' p (slot 2).
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_rb_refine(const RbDev* __restrict__ rbp, const RhsState* __restrict__ st,
                                                    const double* __restrict__ c, const double* __restrict__ xB,
                                                    const double* __restrict__ u64, T* __restrict__ rv,
                                                    T* __restrict__ pv, double* __restrict__ part, int R,
                                                    int pstride) {
  const RbDev& rb = *rbp;
  const int r = blockIdx.y, i = blockIdx.x * TILE + threadIdx.x;
  count_launch(rb, st, PH_OUTER, PF_REFINE_ACT);
  if (st[r].phase != PH_OUTER) return;
  double acc[3] = {0.0, 0.0, 0.0};
  if (i < rb.NB) {
    int nb[6];
    load_nb(rb.nbB, rb.NB, i, nb);
    const size_t off = (size_t)r * K * rb.NB;
    const Slab<double> cs(c + off, K, rb.NB), xs(xB + off, K, rb.NB), us(u64 + (size_t)r * K * rb.NR, K, rb.NR);
    const Slab<double> Ds(rb.D64, Tri<K>::NB, rb.NB), Ss(rb.S64, Tri<K>::NB, rb.NB);
    const Slab<T> rs(rv + off, K, rb.NB), ps(pv + off, K, rb.NB);
    const unsigned o8 = (unsigned)i * 8u, oT = (unsigned)i * (unsigned)sizeof(T);
    double r64[K], z[K];
    if (rb.zero_start && st[r].outer == 0) {   // x_B = 0: r = c
#pragma unroll
      for (int k = 0; k < K; ++k) r64[k] = cs.ld(k, o8);
    } else {
      double xv[K], y[K], s[K];
#pragma unroll
      for (int k = 0; k < K; ++k) xv[k] = xs.ld(k, o8);
      packed_apply<double, K>(Ds, o8, xv, y);
      neighbour_sum<double, K>(nb, us, s);
#pragma unroll
      for (int k = 0; k < K; ++k) r64[k] = cs.ld(k, o8) - (y[k] - rb.alpha64[k] * s[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) acc[0] += r64[k] * r64[k];
    packed_apply<double, K>(Ss, o8, r64, z);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[2] += r64[k] * z[k];
      rs.st(k, oT, (T)r64[k]);
      ps.st(k, oT, (T)z[k]);
    }
  }
  block_sums<3>(acc, part, (size_t)R * pstride, (size_t)r * pstride + blockIdx.x);
}

// Black stage of q = S p with the seven inner products of the one-reduction
// iteration, z = blkdiag(S)^{-1} r and t = blkdiag(S)^{-1} q at the voxel:
// p'q, r'z, q'z, q't, r'r, q'r, q'q.
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_rb_matvec(const RbDev* __restrict__ rbp, const RhsState* __restrict__ st,
                                                    const T* __restrict__ pv, const T* __restrict__ u,
                                                    const T* __restrict__ rv, T* __restrict__ qv,
                                                    double* __restrict__ part, int R, int pstride) {
  const RbDev& rb = *rbp;
  const int r = blockIdx.y, i = blockIdx.x * TILE + threadIdx.x;
  count_launch(rb, st, PH_INNER, PF_MATVEC_ACT);
  if (st[r].phase != PH_INNER) return;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < rb.NB) {
    int nb[6];
    load_nb(rb.nbB, rb.NB, i, nb);
    const size_t off = (size_t)r * K * rb.NB;
    const Slab<T> ps(pv + off, K, rb.NB), rs(rv + off, K, rb.NB), qs(qv + off, K, rb.NB);
    const Slab<T> us(u + (size_t)r * K * rb.NR, K, rb.NR);
    const Slab<T> Ds(RbT<T>::D(rb), Tri<K>::NB, rb.NB), Ss(RbT<T>::S(rb), Tri<K>::NB, rb.NB);
    const unsigned oT = (unsigned)i * (unsigned)sizeof(T);
    T p[K], y[K], s[K], q[K], rr[K], z[K], t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = ps.ld(k, oT);
    packed_apply<T, K>(Ds, oT, p, y);
    neighbour_sum<T, K>(nb, us, s);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      q[k] = y[k] - RbT<T>::alpha(rb, k) * s[k];
      qs.st(k, oT, q[k]);
      rr[k] = rs.ld(k, oT);
      z[k] = t[k] = 0;
    }
    sym_apply<K>([&](int e) { return Ss.ld(e, oT); }, rr, z);
    sym_apply<K>([&](int e) { return Ss.ld(e, oT); }, q, t);
    T a[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      a[0] += p[k] * q[k];
      a[1] += rr[k] * z[k];
      a[2] += q[k] * z[k];
      a[3] += q[k] * t[k];
      a[4] += rr[k] * rr[k];
      a[5] += q[k] * rr[k];
      a[6] += q[k] * q[k];
    }
#pragma unroll
    for (int e = 0; e < 7; ++e) acc[e] = (double)a[e];
  }
  block_sums<7>(acc, part, (size_t)R * pstride, (size_t)r * pstride + blockIdx.x);
}

// d += a p (d = a p on the first step), r -= a q, p = blkdiag(S)^{-1} r + beta p.
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_rb_update(const RbDev* __restrict__ rbp, const RhsState* __restrict__ st, T* __restrict__ dv,
                                                    T* __restrict__ rv, T* __restrict__ pv,
                                                    const T* __restrict__ qv) {
  const RbDev& rb = *rbp;
  const int r = blockIdx.y, i = blockIdx.x * TILE + threadIdx.x;
  count_launch(rb, st, PH_INNER, PF_UPDATE_ACT);
  const RhsState& s = st[r];
  if (s.phase != PH_INNER || i >= rb.NB) return;
  const T a = (T)s.a, beta = (T)s.beta;
  const bool fresh = s.inner_it == 1;
  const size_t off = (size_t)r * K * rb.NB;
  const Slab<T> ds(dv + off, K, rb.NB), rs(rv + off, K, rb.NB), ps(pv + off, K, rb.NB), qs(qv + off, K, rb.NB);
  const Slab<T> Ss(RbT<T>::S(rb), Tri<K>::NB, rb.NB);
  const unsigned oT = (unsigned)i * (unsigned)sizeof(T);
  T p[K], rn[K], z[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    p[k] = ps.ld(k, oT);
    ds.st(k, oT, fresh ? a * p[k] : ds.ld(k, oT) + a * p[k]);
    rn[k] = rs.ld(k, oT) - a * qs.ld(k, oT);
    rs.st(k, oT, rn[k]);
  }
  packed_apply<T, K>(Ss, oT, rn, z);
#pragma unroll
  for (int k = 0; k < K; ++k) ps.st(k, oT, z[k] + beta * p[k]);
}

// x_B += d (when valid) + a p (when the last step is pending) for right-hand
// sides whose inner solve has ended.
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_rb_addsol(const RbDev* __restrict__ rbp, const RhsState* __restrict__ st,
                                                    double* __restrict__ xB, const T* __restrict__ dv,
                                                    const T* __restrict__ pv) {
  const RbDev& rb = *rbp;
  const int r = blockIdx.y, i = blockIdx.x * TILE + threadIdx.x;
  const RhsState& s = st[r];
  // with a zero start value, the first x_B += d writes x_B without reading it
  const bool fresh = rb.zero_start && s.outer == 1;
  if (s.phase != PH_OUTER || !(s.has_d || s.pend || fresh) || i >= rb.NB) return;
  const bool hd = s.has_d != 0, hp = s.pend != 0;
  const double a = s.a;
  const size_t off = (size_t)r * K * rb.NB;
  const Slab<double> xs(xB + off, K, rb.NB);
  const Slab<T> ds(dv + off, K, rb.NB), ps(pv + off, K, rb.NB);
  const unsigned o8 = (unsigned)i * 8u, oT = (unsigned)i * (unsigned)sizeof(T);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = fresh ? 0.0 : xs.ld(k, o8);
    if (hd) v += (double)ds.ld(k, oT);
    if (hp) v += a * (double)ps.ld(k, oT);
    xs.st(k, o8, v);
  }
}

// Writes the solution in the caller's layout: x_m = x_B at the black voxels,
// x_n = Q_nn^{-1} (b_n + alpha .* sum_{m ~ n} x_m) at the red ones (zero for
// a right-hand side with b = 0).  Workgroups [0, ntR) take red tiles, the rest
// black tiles.
template <int K>
__global__ __launch_bounds__(TILE) void k_rb_recover(RbDev rb, const RhsState* __restrict__ st,
                                                     const double* __restrict__ b, const double* __restrict__ xB,
                                                     double* __restrict__ x) {
  const int r = blockIdx.y;
  const bool zero = st[r].zero_b != 0;
  // from a zero start value, x_B holds nothing until the first x_B += d
  const bool xzero = rb.zero_start && st[r].outer <= 1;
  const size_t ur = (size_t)r * K * rb.N;
  const Slab<double> xs(xB + (size_t)r * K * rb.NB, K, rb.NB), xu(x + ur, K, rb.N);
  if ((int)blockIdx.x < rb.ntR) {
    const int j = blockIdx.x * TILE + threadIdx.x;
    if (j >= rb.NR) return;
    const int n = rb.red[j];
    const unsigned on = (unsigned)n * 8u;
    double v[K];
    if (zero) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = 0.0;
    } else {
      int nb[6];
      load_nb(rb.nbR, rb.NR, j, nb);
      const Slab<double> bs(b + ur, K, rb.N), Ps(rb.P64, Tri<K>::NB, rb.NR);
      double s[K];
      if (xzero) {
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] = 0.0;
      } else {
        neighbour_sum<double, K>(nb, xs, s);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) s[k] = bs.ld(k, on) + rb.alpha64[k] * s[k];
      packed_apply<double, K>(Ps, (unsigned)j * 8u, s, v);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) xu.st(k, on, v[k]);
  } else {
    const int i = (blockIdx.x - rb.ntR) * TILE + threadIdx.x;
    if (i >= rb.NB) return;
    const unsigned om = (unsigned)rb.blk[i] * 8u, oi = (unsigned)i * 8u;
#pragma unroll
    for (int k = 0; k < K; ++k) xu.st(k, om, (zero || xzero) ? 0.0 : xs.ld(k, oi));
  }
}

// One wavefront per right-hand side: reduce the black tiles' partials in a
// fixed order and advance the state with the main solver's rules.  For the
// refinement the ||b||^2 slot comes from the split partials (both colours).
template <int KIND>
__global__ __launch_bounds__(FIN_WAVES * WAVE) void k_rb_finalize(const Prob* __restrict__ prp,
                                                                  const double* __restrict__ bbpart, int ntB,
                                                                  int ntBR) {
  const Prob& pr = *prp;
  const int r = blockIdx.x * FIN_WAVES + (int)(threadIdx.x / WAVE);
  if (r >= pr.R) return;
  if (pr.st[r].phase != (KIND == 0 ? PH_OUTER : PH_INNER)) return;
  const int lane = threadIdx.x % WAVE;
  if constexpr (KIND == 0) {
    double v[3], bb[1];
    sum_partials<3>(pr.part, pr.R, pr.pstride, ntB, r, v);
    sum_partials<1>(bbpart, 1, ntBR, ntBR, r, bb);
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
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)         \
    default: return hipErrorInvalidValue;                                                            \
  }

hipError_t launch_rb_setup(hipStream_t s, const RbDev& rb, const double* B64, double* P64, float* P32,
                           double* D64, float* D32, double* S64, float* S32, int* bad) {
  const int gr = (rb.NR + TILE - 1) / TILE, gb = (rb.NB + TILE - 1) / TILE;
#define X(KK)                                                                                         \
  case KK:                                                                                            \
    if (gr > 0) hipLaunchKernelGGL(k_rb_setup_red<KK>, dim3(gr), dim3(TILE), 0, s, rb, B64, P64, P32, bad); \
    if (gb > 0)                                                                                       \
      hipLaunchKernelGGL(k_rb_setup_black<KK>, dim3(gb), dim3(TILE), 0, s, rb, B64, D64, D32, S64, S32, bad); \
    break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_rb_split(hipStream_t s, const RbDev& rb, int R, const double* b, const double* x, int zero_guess,
                           double* t, double* c, double* xB, double* bbpart) {
#define X(KK)                                                                                        \
  case KK:                                                                                           \
    if (rb.ntR > 0) hipLaunchKernelGGL(k_rb_split_red<KK>, grid2(rb.ntR, R), dim3(TILE), 0, s, rb, b, t, bbpart); \
    if (rb.ntB > 0)                                                                                  \
      hipLaunchKernelGGL(k_rb_split_black<KK>, grid2(rb.ntB, R), dim3(TILE), 0, s, rb, b, x, zero_guess, t, c, \
                         xB, bbpart);                                                                \
    break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb_red_t(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, int want, const T* v, T* u) {
  if (rb.ntR == 0) return hipSuccess;
#define X(KK) \
  case KK: hipLaunchKernelGGL((k_rb_red<T, KK>), grid2(rb.ntR, R), dim3(TILE), 0, s, rbd, st, want, v, u); break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}
hipError_t launch_rb_red(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, int want,
                         const double* v, double* u) {
  return launch_rb_red_t<double>(s, rb, rbd, R, st, want, v, u);
}
hipError_t launch_rb_red(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, int want,
                         const float* v, float* u) {
  return launch_rb_red_t<float>(s, rb, rbd, R, st, want, v, u);
}

template <typename T>
hipError_t launch_rb_refine_t(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, const double* c,
                              const double* xB, const double* u64, T* r, T* p, double* part, int pstride) {
  if (rb.ntB == 0) return hipSuccess;
#define X(KK)                                                                                          \
  case KK:                                                                                             \
    hipLaunchKernelGGL((k_rb_refine<T, KK>), grid2(rb.ntB, R), dim3(TILE), 0, s, rbd, st, c, xB, u64, r, p, part, \
                       R, pstride);                                                                    \
    break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb_matvec_t(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, const T* p, const T* u,
                              const T* r, T* q, double* part, int pstride) {
  if (rb.ntB == 0) return hipSuccess;
#define X(KK)                                                                                              \
  case KK:                                                                                                 \
    hipLaunchKernelGGL((k_rb_matvec<T, KK>), grid2(rb.ntB, R), dim3(TILE), 0, s, rbd, st, p, u, r, q, part, R, \
                       pstride);                                                                           \
    break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb_update_t(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, T* d, T* r, T* p,
                              const T* q) {
  if (rb.ntB == 0) return hipSuccess;
#define X(KK) \
  case KK: hipLaunchKernelGGL((k_rb_update<T, KK>), grid2(rb.ntB, R), dim3(TILE), 0, s, rbd, st, d, r, p, q); break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb_addsol_t(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, double* xB, const T* d,
                              const T* p) {
  if (rb.ntB == 0) return hipSuccess;
#define X(KK) \
  case KK: hipLaunchKernelGGL((k_rb_addsol<T, KK>), grid2(rb.ntB, R), dim3(TILE), 0, s, rbd, st, xB, d, p); break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

#define RB_INST(T)                                                                                          \
  hipError_t launch_rb_refine(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, const double* c,    \
                              const double* xB, const double* u64, T* r, T* p, double* part, int pstride) {  \
    return launch_rb_refine_t<T>(s, rb, rbd, R, st, c, xB, u64, r, p, part, pstride);                           \
  }                                                                                                         \
  hipError_t launch_rb_matvec(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, const T* p,         \
                              const T* u, const T* r, T* q, double* part, int pstride) {                     \
    return launch_rb_matvec_t<T>(s, rb, rbd, R, st, p, u, r, q, part, pstride);                                  \
  }                                                                                                         \
  hipError_t launch_rb_update(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, T* d, T* r, T* p,   \
                              const T* q) {                                                                 \
    return launch_rb_update_t<T>(s, rb, rbd, R, st, d, r, p, q);                                                 \
  }                                                                                                         \
  hipError_t launch_rb_addsol(hipStream_t s, const RbDev& rb, const RbDev* rbd, int R, const RhsState* st, double* xB,         \
                              const T* d, const T* p) {                                                     \
    return launch_rb_addsol_t<T>(s, rb, rbd, R, st, xB, d, p);                                                   \
  }
RB_INST(double)
RB_INST(float)
#undef RB_INST

hipError_t launch_rb_recover(hipStream_t s, const RbDev& rb, int R, const RhsState* st, const double* b,
                             const double* xB, double* x) {
  const int tiles = rb.ntR + rb.ntB;
  if (tiles == 0) return hipSuccess;
#define X(KK) \
  case KK: hipLaunchKernelGGL(k_rb_recover<KK>, grid2(tiles, R), dim3(TILE), 0, s, rb, st, b, xB, x); break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_rb_finalize(hipStream_t s, int kind, int R, const Prob* prd, const double* bbpart, int ntB,
                              int ntBR) {
  const int g = (R + FIN_WAVES - 1) / FIN_WAVES;
  if (kind == 0)
    hipLaunchKernelGGL(k_rb_finalize<0>, dim3(g), dim3(FIN_WAVES * WAVE), 0, s, prd, bbpart, ntB, ntBR);
  else
    hipLaunchKernelGGL(k_rb_finalize<1>, dim3(g), dim3(FIN_WAVES * WAVE), 0, s, prd, bbpart, ntB, ntBR);
  return hipGetLastError();
}

}  // namespace gp
