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
// Iteration (Section 3.1: PCG until ||b - Qx|| / ||b|| <= delta), in the
// form that needs one global reduction per inner step: the next residual's
// norms come from three-term expansions in inner products that the matvec
// launch already forms (D'Azevedo, Eijkhout and Romine, LAPACK Working Note
// 56, 1993), so the direction p is built by the elementwise update and the
// stencil gathers p alone.
//   refine  (FP64)  : r64 = b - Q x, ||r64||^2, ||b||^2;  r = T(r64), p = M^{-1} r, r'p
//   matvec  (T)     : q = Q p;  with z = M^{-1} r and t = M^{-1} q at the voxel:
//                     p'q, r'z, q'z, q't, r'r, q'r, q'q
//   finalise        : a = r'z / p'q,
//                     rho' = r'z - 2a q'z + a^2 q't   (= r_new' M^{-1} r_new)
//                     rr'  = r'r - 2a q'r + a^2 q'q   (= ||r_new||^2)
//                     stop the inner solve on rr' or a cap, else beta = rho' / r'z
//   update  (T)     : d += a p,  r -= a q,  p = M^{-1} r + beta p   (no reduction)
//   addsol  (FP64)  : x += d (+ a p of a final step) once an inner solve has ended
// The matvec and refine kernels store per-tile partial sums; a small
// finalising kernel then reduces them per right-hand side in a fixed order and
// advances that right-hand side's state, so no workgroup waits on another.
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

// z = M^{-1} r at voxel n with the preconditioner's entries streamed from
// memory (for K too large to hold the block in registers).
template <typename T, int PC, int K>
__device__ inline void precond_apply_mem(const T* __restrict__ P, int N, int n, const T (&r)[K], T (&z)[K]) {
  const __attribute__((address_space(1))) T* g = (const __attribute__((address_space(1))) T*)P;
  if constexpr (PC == PC_JACOBI) {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = g[(size_t)k * N + (unsigned)n] * r[k];
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int j = 0; j <= k; ++j) {
        const T p = g[(size_t)pk(k, j) * N + (unsigned)n];
        z[k] += p * r[j];
        if (j != k) z[j] += p * r[k];
      }
    }
  }
}

// r'M^{-1}r, q'M^{-1}r and q'M^{-1}q at voxel n, with the preconditioner's
// entries streamed from memory (each used once, none held across the loop).
template <typename T, int PC, int K>
__device__ inline void precond_forms(const T* __restrict__ P, int N, int n, const T (&r)[K], const T (&q)[K],
                                     T& rr, T& qr, T& qq) {
  const __attribute__((address_space(1))) T* g = (const __attribute__((address_space(1))) T*)P;
  rr = qr = qq = 0;
  if constexpr (PC == PC_JACOBI) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T p = g[(size_t)k * N + (unsigned)n];
      rr += p * r[k] * r[k];
      qr += p * q[k] * r[k];
      qq += p * q[k] * q[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int j = 0; j <= k; ++j) {
        const T p = g[(size_t)pk(k, j) * N + (unsigned)n];
        if (j == k) {
          rr += p * r[k] * r[k];
          qr += p * q[k] * r[k];
          qq += p * q[k] * q[k];
        } else {
          rr += 2 * p * r[k] * r[j];
          qr += p * (q[k] * r[j] + q[j] * r[k]);
          qq += 2 * p * q[k] * q[j];
        }
      }
    }
  }
}

// Blocks held in registers across a work item's right-hand sides while they
// fit; larger K streams them per right-hand side (cache hits).
template <int K> struct HoldB { static constexpr bool v = K <= 6; };
// Regressors whose neighbour gathers may be in flight together in the matvec.
template <typename T, int K> struct GatherG { static constexpr int v = (sizeof(T) == 4 && K >= 12) ? 4 : K; };
// The update kernel holds the preconditioner in registers while it fits.
template <typename T, int PC, int K> struct HoldP {
  static constexpr bool v = PC == PC_JACOBI || (sizeof(T) == 4 ? K <= 12 : K <= 8);
};

// Resident-wave request of the matvec kernel: 4 per SIMD (<= 128 VGPRs) while
// its per-voxel vectors fit, else 2.
template <typename T, int K> struct OccMV { static constexpr int v = sizeof(T) == 4 ? (K <= 11 ? 4 : 2) : (K <= 5 ? 4 : 2); };

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
  prof_add(pr, PF_ADDSOL_D, s.has_d);
  prof_add(pr, PF_ADDSOL_P, s.pend);
  if (s.outer == 0) s.bnorm2 = bb;
  s.has_d = 0;
  s.pend = 0;
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
      s.inner_it = 0;
      s.phase = PH_INNER;
    }
  }
}

// v = (p'q, r'z, q'z, q't, r'r, q'r, q'q) of the step just taken.
__device__ inline void finalize_matvec(const Prob& pr, int r, const double (&v)[7]) {
  RhsState& s = pr.st[r];
  prof_add(pr, PF_MATVEC_RHS, 1);
  const double sigma = v[0], rz = v[1];
  if (!(sigma > 0.0) || !finite(sigma) || !(rz > 0.0) || !finite(rz)) {
    if (s.inner_it == 0) {
      s.has_d = 0; s.status = ST_BREAKDOWN; s.phase = PH_DONE;   // no usable correction
    } else {
      s.phase = PH_OUTER;   // keep the correction so far; re-evaluate in FP64
    }
    return;
  }
  const double a = rz / sigma;
  const double rho = rz - 2.0 * a * v[2] + a * a * v[3];
  const double rr = v[4] - 2.0 * a * v[5] + a * a * v[6];
  s.a = a;
  s.inner_it += 1;
  s.total_it += 1;
  if (!finite(rho) || !finite(rr) || !finite(a)) {
    s.has_d = 0; s.status = ST_BREAKDOWN; s.phase = PH_DONE;
  } else if (rr <= s.target2 || s.total_it >= pr.cfg.max_iter || !(rho > 0.0)) {
    s.pend = 1;             // the final step a p is added to x with d
    s.phase = PH_OUTER;
  } else {
    prof_add(pr, PF_UPDATE_RHS, 1);
    prof_add(pr, PF_UPDATE_FRESH, s.inner_it == 1);
    s.beta = rho / rz;
    s.rho = rho;
    s.has_d = 1;            // the update launch writes d
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
  } else {
    double v[7];
    sum_partials<7>(pr.part, pr.R, pr.pstride, pr.mv_mode ? pr.mv_tiles : pr.op.ntiles, r, v);
    if (lane == 0) finalize_matvec(pr, r, v);
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
        T* pp = (T*)pr.p + (size_t)r * K * N;   // first direction p = M^{-1} r
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          sto(rp + (size_t)k * N, oT, rt[k]);
          sto(pp + (size_t)k * N, oT, z[k]);
        }
      } else {
        acc[0] = acc[1] = acc[2] = 0.0;
      }
      wave_deposit<3>(s_red, r - r0, acc);
    }
    flush_partials<3>(pr, s_red, r0, r1, w.tile, PH_OUTER);
  }
}

// q = Q p and the seven inner products of the step (see the header comment).
template <typename T, int PC, int K>
__global__ __launch_bounds__(TILE, (OccMV<T, K>::v)) void k_matvec(const Prob* __restrict__ probs, int nprob, int W) {
  constexpr int NB = Tri<K>::NB;
  __shared__ double s_red[RCMAX * NPART * (TILE / WAVE)];
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
    T Bh[HoldB<K>::v ? NB : 1];
    if constexpr (HoldB<K>::v) load_soa(OpT<T>::B(op), N, w.nn, Bh);
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      if (pr.st[r].phase != PH_INNER) continue;
      const size_t off = (size_t)r * K * N;
      const T* pp = (const T*)pr.p + off;
      const T* rp = (const T*)pr.r + off;
      T* qp = (T*)pr.q + off;
      T pc[K], qv[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const T* pk_ = pp + (size_t)k * N;
        const T c = ldo(pk_, o);
        T s6 = 0;
  #pragma unroll
        for (int d = 0; d < 6; ++d) s6 += c - ldo(pk_, nb[d]);
        pc[k] = c;
        qv[k] = OpT<T>::alpha(op, k) * s6;
        // bound the gathers in flight (GatherG<T, K> regressors at a time)
        if constexpr (GatherG<T, K>::v < K)
          if ((k + 1) % GatherG<T, K>::v == 0) __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (HoldB<K>::v) {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
  #pragma unroll
          for (int j = 0; j < K; ++j) qv[k] += Bh[pk(k, j)] * pc[j];
        }
      } else {
        const __attribute__((address_space(1))) T* Bg = (const __attribute__((address_space(1))) T*)OpT<T>::B(op);
  #pragma unroll
        for (int k = 0; k < K; ++k) {
  #pragma unroll
          for (int j = 0; j <= k; ++j) {
            const T bkj = Bg[(size_t)pk(k, j) * N + (unsigned)w.nn];
            qv[k] += bkj * pc[j];
            if (j != k) qv[j] += bkj * pc[k];
          }
        }
      }
      T rv[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) rv[k] = ldo(rp + (size_t)k * N, o);
      T rPr, qPr, qPq;
      precond_forms<T, PC, K>(OpT<T>::P(op), N, w.nn, rv, qv, rPr, qPr, qPq);
      double acc[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (w.valid) {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
          sto(qp + (size_t)k * N, o, qv[k]);
          const double pd = pc[k], qd = qv[k], rd = rv[k];
          acc[0] += pd * qd;
          acc[4] += rd * rd;
          acc[5] += qd * rd;
          acc[6] += qd * qd;
        }
        acc[1] = rPr;
        acc[2] = qPr;
        acc[3] = qPq;
      }
      wave_deposit<NPART>(s_red, r - r0, acc);
    }
    flush_partials<NPART>(pr, s_red, r0, r1, w.tile, PH_INNER);
  }
}

// d += a p,  r -= a q,  p = M^{-1} r + beta p  for right-hand sides that go on.
template <typename T, int PC, int K>
__global__ __launch_bounds__(TILE, (OccMV<T, K>::v)) void k_update(const Prob* __restrict__ probs, int nprob, int W) {
  constexpr int NP = PSize<PC, K>::n;
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int N = op.N;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_UPDATE_ACT, PH_INNER);
    const int r0 = w.chunk * pr.Rc;
    const int r1 = min(pr.R, r0 + pr.Rc);
    if (!w.valid || !any_in_phase(pr, r0, r1, PH_INNER)) continue;
    constexpr bool hold = HoldP<T, PC, K>::v;
    T P[hold ? NP : 1];
    if constexpr (hold) load_soa(OpT<T>::P(op), N, w.n, P);
    const unsigned o = (unsigned)w.n * sizeof(T);
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      const RhsState& s = pr.st[r];
      if (s.phase != PH_INNER) continue;
      const T a = (T)s.a, beta = (T)s.beta;
      const bool fresh = s.inner_it == 1;
      const size_t off = (size_t)r * K * N;
      T* pp = (T*)pr.p + off;
      const T* qp = (const T*)pr.q + off;
      T* dp = (T*)pr.d + off;
      T* rp = (T*)pr.r + off;
      T pv[K], rv[K], z[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const size_t kb = (size_t)k * N;
        pv[k] = ldo(pp + kb, o);
        const T dv = fresh ? a * pv[k] : ldo(dp + kb, o) + a * pv[k];
        rv[k] = ldo(rp + kb, o) - a * ldo(qp + kb, o);
        sto(dp + kb, o, dv);
        sto(rp + kb, o, rv[k]);
      }
      if constexpr (hold)
        precond_apply<T, PC, K>(P, rv, z);
      else
        precond_apply_mem<T, PC, K>(OpT<T>::P(op), N, w.n, rv, z);
  #pragma unroll
      for (int k = 0; k < K; ++k) sto(pp + (size_t)k * N, o, z[k] + beta * pv[k]);
    }
  }
}

// x += d (when valid) + a p (when the last step is pending) for right-hand
// sides whose inner solve has ended.
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
      if (s.phase != PH_OUTER || !(s.has_d || s.pend)) continue;
      const bool hd = s.has_d != 0, hp = s.pend != 0;
      const double a = s.a;
      const size_t off = (size_t)r * K * N;
      const T* dr = (const T*)pr.d + off;
      const T* pp = (const T*)pr.p + off;
      double* xr = pr.x + off;
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const size_t kb = (size_t)k * N;
        double v = ldo(xr + kb, o8);
        if (hd) v += (double)ldo(dr + kb, oT);
        if (hp) v += a * (double)ldo(pp + kb, oT);
        sto(xr + kb, o8, v);
      }
    }
  }
}

}  // namespace gp
