// Preconditioned conjugate gradients with the posterior precision
//   Q = diag(alpha) (x) D_w + H' blkdiag_n(B_n) H
// for many right-hand sides and many operators per launch.
//
// Operator action at voxel n, regressor k (the k-major entry form of the
// precision of w_r = vec(W'), Section 3 and Appendix A.2):
//   (Q v)_{k,n} = alpha_k * sum_d (v_{k,n} - v_{k,nb_d(n)}) + sum_j B_n[k,j] v_{j,n}
// where nb_d(n) is the neighbour in direction d, or n itself when that
// neighbour lies outside the mask -- the term then vanishes, which gives the
// in-mask degree on the Laplacian diagonal (Section 2, free boundary).
//
// Iteration (Section 3.1: PCG until ||b - Qx|| / ||b|| <= delta), split into
// three kernels per step so that each global reduction ends a launch:
//   refine  (FP64)  : r64 = b - Q x, ||r64||^2, ||b||^2;  r = T(r64), z = M^{-1} r, r'z
//   matvec  (T)     : p = z + beta p_old (p = z at the first step), q = Q p, p'q
//   update  (T)     : d += a p, r -= a q, z = M^{-1} r, r'z, r'r
//   addsol  (FP64)  : x += d once an inner solve has ended
// Each of those kernels stores per-tile partial sums; a small finalising
// kernel then reduces them per right-hand side in a fixed order and advances
// that right-hand side's state, so no workgroup waits on another.
#pragma once
#include "device.hpp"

namespace gp {

template <typename T> struct OpT;
template <> struct OpT<double> {
  __device__ static const double* B(const OpDev& o) { return o.B64; }
  __device__ static const double* P(const OpDev& o) { return o.P64; }
  __device__ static double alpha(const OpDev& o, int k) { return o.alpha64[k]; }
};
template <> struct OpT<float> {
  __device__ static const float* B(const OpDev& o) { return o.B32; }
  __device__ static const float* P(const OpDev& o) { return o.P32; }
  __device__ static float alpha(const OpDev& o, int k) { return o.alpha32[k]; }
};

template <int K> struct Tri { static constexpr int NB = K * (K + 1) / 2; };

// Minimum resident waves per SIMD requested from the compiler (caps VGPRs):
// 4 (<= 128 VGPRs) while the per-voxel blocks fit, else 2.
template <int K> struct Occ { static constexpr int inner = K <= 10 ? 4 : 2; static constexpr int outer = 2; };
template <int PC, int K> struct PSize { static constexpr int n = PC == PC_BLOCK ? Tri<K>::NB : K; };

template <typename T, int NV>
__device__ inline void load_soa(const T* __restrict__ A, int N, int n, T (&a)[NV]) {
  const __attribute__((address_space(1))) T* g = (const __attribute__((address_space(1))) T*)A;
#pragma unroll
  for (int i = 0; i < NV; ++i) a[i] = g[(size_t)i * N + (unsigned)n];
}

template <typename T, int PC, int K>
__device__ inline void precond_apply(const T (&P)[PSize<PC, K>::n], const T (&r)[K], T (&z)[K]) {
  if constexpr (PC == PC_JACOBI) {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = P[k] * r[k];
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) s += P[pk(k, j)] * r[j];
      z[k] = s;
    }
  }
}

// Per-RHS sums held in LDS: s_red[(slot * NV + v) * nwaves + wave].
template <int NV>
__device__ inline void wave_deposit(double* s_red, int slot, const double (&acc)[NV]) {
  const int wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double s = wave_sum(acc[v]);
    if ((threadIdx.x % WAVE) == 0) s_red[(slot * NV + v) * nw + wv] = s;
  }
}

// After the right-hand-side loop: one store per (active RHS, value) of the
// workgroup's sum, waves added in order.
template <int NV>
__device__ inline void flush_partials(const Prob& pr, const double* s_red, int r0, int r1, int tile,
                                      int want_phase) {
  __syncthreads();
  const int nw = blockDim.x / WAVE;
  const int i = threadIdx.x;
  if (i < (r1 - r0) * NV) {
    const int slot = i / NV, v = i % NV, r = r0 + slot;
    if (pr.st[r].phase == want_phase) {
      double t = 0.0;
      for (int j = 0; j < nw; ++j) t += s_red[(slot * NV + v) * nw + j];
      pr.part[((size_t)v * pr.R + r) * pr.pstride + tile] = t;
    }
  }
  __syncthreads();   // s_red is reused by the next work item
}

struct Where {
  int p, tile, chunk, n, nn;
  bool valid;
};

// Persistent sweep over the W work items of a grouped launch.  Workgroups are
// dealt to the XCDs round-robin (workgroup b runs on XCD b % NXCD), so the
// items are split into NXCD contiguous ranges and the workgroups of one XCD
// walk their range in order with a stride of their count.  The items being
// processed at any moment on an XCD are then neighbours in the work order,
// which keeps the stencil's z-neighbour slices in that XCD's L2.
struct Sweep {
  int item, end, step;
};

__device__ inline Sweep sweep_begin(int W) {
  const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
  const int base = W / NXCD, rem = W % NXCD;
  const int start = xcd * base + (xcd < rem ? xcd : rem);
  const int cnt = base + (xcd < rem ? 1 : 0);
  return Sweep{start + slot, start + cnt, (int)(gridDim.x / NXCD)};
}

// Work items of a problem are ordered right-hand-side chunk major, tile minor.
__device__ inline Where locate(const Prob* __restrict__ probs, int nprob, int item) {
  Where w;
  w.p = find_prob(probs, nprob, item);
  const int local = item - probs[w.p].work_begin;
  const int nt = probs[w.p].op.ntiles;
  w.chunk = local / nt;
  w.tile = local - w.chunk * nt;
  const int N = probs[w.p].op.N;
  w.n = w.tile * TILE + (int)threadIdx.x;
  w.valid = w.n < N;
  w.nn = w.valid ? w.n : N - 1;
  return w;
}

__device__ inline bool finite(double v) { return v == v && v - v == 0.0; }

// Does any right-hand side in [r0, r1) sit in `phase`?  (uniform per workgroup)
__device__ inline bool any_in_phase(const Prob& pr, int r0, int r1, int phase) {
  for (int r = r0; r < r1; ++r)
    if (pr.st[r].phase == phase) return true;
  return false;
}

// --------------------------------------------------------------- finalisers
// Each finaliser advances one right-hand side from the per-tile partials of
// the launch that just ended; it runs on lane 0 of the wavefront that summed
// them.  Counters for the profiler are added with integer atomics.
__device__ inline void prof_add(const Prob& pr, int slot, long long v) {
  if (pr.prof && v) atomicAdd((unsigned long long*)&pr.prof[slot], (unsigned long long)v);
}

// Counts a launch in slot `act` when any right-hand side of the problem is in
// `phase`; called by the workgroup holding the problem's first work item
// while no finaliser can be changing the states.
__device__ inline void prof_launch(const Prob& pr, int act, int phase) {
  if (pr.prof && threadIdx.x == 0 && any_in_phase(pr, 0, pr.R, phase))
    atomicAdd((unsigned long long*)&pr.prof[act], 1ull);
}

__device__ inline void finalize_refine(const Prob& pr, int r, const double (&v)[3]) {
  RhsState& s = pr.st[r];
  const double rr = v[0], bb = v[1], rz = v[2];
  prof_add(pr, PF_REFINE_RHS, 1);
  prof_add(pr, PF_ADDSOL_RHS, s.has_d);
  if (s.outer == 0) s.bnorm2 = bb;
  s.has_d = 0;
  s.outer += 1;
  s.rr64 = rr;
  const double bn2 = s.bnorm2;
  if (!finite(bn2)) {
    s.status = ST_BREAKDOWN; s.phase = PH_DONE;
  } else if (bn2 == 0.0) {
    s.relres = 0.0; s.zero_b = 1; s.status = ST_OK; s.phase = PH_DONE;
  } else {
    const double rel = sqrt(rr / bn2);
    s.relres = rel;
    if (!finite(rel)) {
      s.status = ST_BREAKDOWN; s.phase = PH_DONE;
    } else if (rel <= pr.cfg.tol) {
      s.status = ST_OK; s.phase = PH_DONE;
    } else if (s.outer >= pr.cfg.max_outer || s.total_it >= pr.cfg.max_iter) {
      s.status = ST_NOT_CONVERGED; s.phase = PH_DONE;
    } else if (!(rz > 0.0) || !finite(rz)) {
      s.status = ST_BREAKDOWN; s.phase = PH_DONE;
    } else {
      const double it2 = pr.cfg.inner_tol * pr.cfg.inner_tol * rr;
      const double ot2 = 0.25 * pr.cfg.tol * pr.cfg.tol * bn2;
      s.target2 = it2 > ot2 ? it2 : ot2;
      s.rho = rz;
      s.first = 1;
      s.inner_it = 0;
      s.has_d = 1;
      s.phase = PH_INNER;
    }
  }
}

__device__ inline void finalize_matvec(const Prob& pr, int r, const double (&v)[1]) {
  RhsState& s = pr.st[r];
  prof_add(pr, PF_MATVEC_RHS, 1);
  prof_add(pr, PF_MATVEC_FIRST, s.first);
  const double sigma = v[0];
  if (!(sigma > 0.0) || !finite(sigma)) {
    if (s.inner_it == 0) {       // no usable correction yet
      s.has_d = 0; s.status = ST_BREAKDOWN; s.phase = PH_DONE;
    } else {                     // keep the correction so far; re-evaluate in FP64
      s.phase = PH_OUTER;
    }
  } else {
    s.a = s.rho / sigma;
    s.first = 0;
  }
}

__device__ inline void finalize_update(const Prob& pr, int r, const double (&v)[2]) {
  RhsState& s = pr.st[r];
  prof_add(pr, PF_UPDATE_RHS, 1);
  prof_add(pr, PF_UPDATE_FRESH, s.inner_it == 0);
  const double rz = v[0], rr = v[1];
  s.inner_it += 1;
  s.total_it += 1;
  if (!finite(rr) || !finite(rz)) {
    s.has_d = 0; s.status = ST_BREAKDOWN; s.phase = PH_DONE;
  } else if (rr <= s.target2 || s.total_it >= pr.cfg.max_iter || !(rz > 0.0)) {
    s.phase = PH_OUTER;
  } else {
    s.beta = rz / s.rho;
    s.rho = rz;
  }
}

constexpr int FIN_WAVES = 4;   // right-hand sides finalised per workgroup

// One wavefront per right-hand side of one problem: sum that right-hand side's
// partials over the tiles in a fixed order and advance its state.
template <int KIND>
__global__ __launch_bounds__(FIN_WAVES * WAVE) void k_finalize(const Prob* __restrict__ probs, int nprob) {
  const int b = blockIdx.x;
  int p = 0;
  while (p + 1 < nprob && b >= probs[p + 1].fin_begin) ++p;
  const Prob& pr = probs[p];
  const int r = (b - pr.fin_begin) * FIN_WAVES + (int)(threadIdx.x / WAVE);
  if (r >= pr.R) return;
  const int want = KIND == 0 ? PH_OUTER : PH_INNER;
  if (pr.st[r].phase != want) return;
  const int lane = threadIdx.x % WAVE;
  if constexpr (KIND == 0) {
    double v[3];
    sum_partials<3>(pr.part, pr.R, pr.pstride, pr.op.ntiles, r, v);
    if (lane == 0) finalize_refine(pr, r, v);
  } else if constexpr (KIND == 1) {
    double v[1];
    sum_partials<1>(pr.part, pr.R, pr.pstride, pr.mv_mode ? pr.mv_tiles : pr.op.ntiles, r, v);
    if (lane == 0) finalize_matvec(pr, r, v);
  } else {
    double v[2];
    sum_partials<2>(pr.part, pr.R, pr.pstride, pr.op.ntiles, r, v);
    if (lane == 0) finalize_update(pr, r, v);
  }
}

// ------------------------------------------------------------------ kernels
// Addressing: every vector access is a wave-uniform base pointer (the slab of
// one right-hand side and regressor) plus a 32-bit per-lane byte offset, so
// loads take the scalar-base form and no 64-bit address is kept per lane.
// Pointers held in the problem descriptors are generic; the casts to the
// global address space let the compiler emit global (not flat) accesses.
#define GP_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ldo(const T* base, unsigned off) {
  return *(const GP_GLOBAL T*)((const GP_GLOBAL char*)base + off);
}
template <typename T>
__device__ __forceinline__ void sto(T* base, unsigned off, T v) {
  *(GP_GLOBAL T*)((GP_GLOBAL char*)base + off) = v;
}

// Byte offsets of the voxel and its six neighbours for element size S.
template <int S>
__device__ __forceinline__ void voxel_offsets(const OpDev& op, int nn, unsigned& own, unsigned (&nb)[6]) {
  own = (unsigned)nn * S;
  const __attribute__((address_space(1))) int* g = (const __attribute__((address_space(1))) int*)op.nbr;
#pragma unroll
  for (int d = 0; d < 6; ++d) nb[d] = (unsigned)g[(size_t)d * op.N + (unsigned)nn] * S;
}

template <typename T, int PC, int K>
__global__ __launch_bounds__(TILE, Occ<K>::outer) void k_refine(const Prob* __restrict__ probs, int nprob, int W) {
  constexpr int NB = Tri<K>::NB, NP = PSize<PC, K>::n;
  __shared__ double s_red[RCMAX * 3 * (TILE / WAVE)];
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int N = op.N;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_REFINE_ACT, PH_OUTER);
    const int r0 = w.chunk * pr.Rc;
    const int r1 = min(pr.R, r0 + pr.Rc);
    if (!any_in_phase(pr, r0, r1, PH_OUTER)) continue;
    unsigned o8, nb8[6];
    voxel_offsets<8>(op, w.nn, o8, nb8);
    const unsigned oT = (unsigned)w.nn * sizeof(T);
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      if (pr.st[r].phase != PH_OUTER) continue;
      // the voxel's FP64 block and preconditioner are re-read per right-hand
      // side (cache hits) rather than held in registers across the loop
      double B[NB];
      load_soa(op.B64, N, w.nn, B);
      T P[NP];
      load_soa(OpT<T>::P(op), N, w.nn, P);
      const double* xr = pr.x + (size_t)r * K * N;
      const double* br = pr.b + (size_t)r * K * N;
      double xo[K], y[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const double* xk = xr + (size_t)k * N;
        const double xc = ldo(xk, o8);
        double s6 = 0.0;
  #pragma unroll
        for (int d = 0; d < 6; ++d) s6 += xc - ldo(xk, nb8[d]);
        xo[k] = xc;
        y[k] = op.alpha64[k] * s6;
      }
  #pragma unroll
      for (int k = 0; k < K; ++k) {
  #pragma unroll
        for (int j = 0; j < K; ++j) y[k] += B[pk(k, j)] * xo[j];
      }
      double acc[3] = {0.0, 0.0, 0.0};
      T rt[K], z[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const double bk = ldo(br + (size_t)k * N, o8);
        const double rk = bk - y[k];
        acc[0] += rk * rk;
        acc[1] += bk * bk;
        rt[k] = (T)rk;
      }
      precond_apply<T, PC, K>(P, rt, z);
  #pragma unroll
      for (int k = 0; k < K; ++k) acc[2] += (double)rt[k] * (double)z[k];
      if (w.valid) {
        T* rp = (T*)pr.r + (size_t)r * K * N;
        T* zp = (T*)pr.z + (size_t)r * K * N;
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          sto(rp + (size_t)k * N, oT, rt[k]);
          sto(zp + (size_t)k * N, oT, z[k]);
        }
      } else {
        acc[0] = acc[1] = acc[2] = 0.0;
      }
      wave_deposit<3>(s_red, r - r0, acc);
    }
    flush_partials<3>(pr, s_red, r0, r1, w.tile, PH_OUTER);
  }
}

template <typename T, int K>
__global__ __launch_bounds__(TILE, Occ<K>::inner) void k_matvec(const Prob* __restrict__ probs, int nprob, int W,
                                                                int parity) {
  constexpr int NB = Tri<K>::NB;
  __shared__ double s_red[RCMAX * 1 * (TILE / WAVE)];
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int N = op.N;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_MATVEC_ACT, PH_INNER);
    const int r0 = w.chunk * pr.Rc;
    const int r1 = min(pr.R, r0 + pr.Rc);
    if (!any_in_phase(pr, r0, r1, PH_INNER)) continue;
    unsigned o, nb[6];
    voxel_offsets<sizeof(T)>(op, w.nn, o, nb);
    T B[NB];
    load_soa(OpT<T>::B(op), N, w.nn, B);
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      const RhsState& s = pr.st[r];
      if (s.phase != PH_INNER) continue;
      const bool first = s.first != 0;
      const T beta = (T)s.beta;
      const size_t off = (size_t)r * K * N;
      const T* zr = (const T*)pr.z + off;
      const T* pin = (const T*)(parity ? pr.p1 : pr.p0) + off;
      T* pout = (T*)(parity ? pr.p0 : pr.p1) + off;
      T* qr = (T*)pr.q + off;
      T po[K], qv[K];
      if (first) {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          const T* zk = zr + (size_t)k * N;
          const T pc = ldo(zk, o);
          T s6 = 0;
  #pragma unroll
          for (int d = 0; d < 6; ++d) s6 += pc - ldo(zk, nb[d]);
          po[k] = pc;
          qv[k] = OpT<T>::alpha(op, k) * s6;
        }
      } else {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          const T* zk = zr + (size_t)k * N;
          const T* pk_ = pin + (size_t)k * N;
          const T pc = ldo(zk, o) + beta * ldo(pk_, o);
          T s6 = 0;
  #pragma unroll
          for (int d = 0; d < 6; ++d) s6 += pc - (ldo(zk, nb[d]) + beta * ldo(pk_, nb[d]));
          po[k] = pc;
          qv[k] = OpT<T>::alpha(op, k) * s6;
        }
      }
  #pragma unroll
      for (int k = 0; k < K; ++k) {
  #pragma unroll
        for (int j = 0; j < K; ++j) qv[k] += B[pk(k, j)] * po[j];
      }
      double acc[1] = {0.0};
      if (w.valid) {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          sto(pout + (size_t)k * N, o, po[k]);
          sto(qr + (size_t)k * N, o, qv[k]);
          acc[0] += (double)po[k] * (double)qv[k];
        }
      }
      wave_deposit<1>(s_red, r - r0, acc);
    }
    flush_partials<1>(pr, s_red, r0, r1, w.tile, PH_INNER);
  }
}

template <typename T, int PC, int K>
__global__ __launch_bounds__(TILE, Occ<K>::inner) void k_update(const Prob* __restrict__ probs, int nprob, int W,
                                                                int parity) {
  constexpr int NP = PSize<PC, K>::n;
  __shared__ double s_red[RCMAX * 2 * (TILE / WAVE)];
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int N = op.N;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_UPDATE_ACT, PH_INNER);
    const int r0 = w.chunk * pr.Rc;
    const int r1 = min(pr.R, r0 + pr.Rc);
    if (!any_in_phase(pr, r0, r1, PH_INNER)) continue;
    T P[NP];
    load_soa(OpT<T>::P(op), N, w.nn, P);
    const unsigned o = (unsigned)w.nn * sizeof(T);
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      const RhsState& s = pr.st[r];
      if (s.phase != PH_INNER) continue;
      const T a = (T)s.a;
      const bool fresh = s.inner_it == 0;
      const size_t off = (size_t)r * K * N;
      const T* pc = (const T*)(parity ? pr.p0 : pr.p1) + off;
      const T* qr = (const T*)pr.q + off;
      T* dr = (T*)pr.d + off;
      T* rr = (T*)pr.r + off;
      T* zr = (T*)pr.z + off;
      T rv[K], dv[K], z[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const size_t kb = (size_t)k * N;
        const T pk_ = ldo(pc + kb, o);
        dv[k] = fresh ? a * pk_ : ldo(dr + kb, o) + a * pk_;
        rv[k] = ldo(rr + kb, o) - a * ldo(qr + kb, o);
      }
      precond_apply<T, PC, K>(P, rv, z);
      double acc[2] = {0.0, 0.0};
      if (w.valid) {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          const size_t kb = (size_t)k * N;
          sto(dr + kb, o, dv[k]);
          sto(rr + kb, o, rv[k]);
          sto(zr + kb, o, z[k]);
          acc[0] += (double)rv[k] * (double)z[k];
          acc[1] += (double)rv[k] * (double)rv[k];
        }
      }
      wave_deposit<2>(s_red, r - r0, acc);
    }
    flush_partials<2>(pr, s_red, r0, r1, w.tile, PH_INNER);
  }
}

// x += d for right-hand sides whose inner solve has ended.
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_addsol(const Prob* __restrict__ probs, int nprob, int W) {
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    if (!w.valid) continue;
    const int N = pr.op.N;
    const int r0 = w.chunk * pr.Rc;
    const int r1 = min(pr.R, r0 + pr.Rc);
    const unsigned oT = (unsigned)w.n * sizeof(T), o8 = (unsigned)w.n * 8u;
    for (int r = r0; r < r1; ++r) {
      const RhsState& s = pr.st[r];
      if (s.phase != PH_OUTER || !s.has_d) continue;
      const size_t off = (size_t)r * K * N;
      const T* dr = (const T*)pr.d + off;
      double* xr = pr.x + off;
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const size_t kb = (size_t)k * N;
        sto(xr + kb, o8, ldo(xr + kb, o8) + (double)ldo(dr + kb, oT));
      }
    }
  }
}

}  // namespace gp
