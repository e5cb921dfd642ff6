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

template <typename T, int NV>
__device__ inline void load_soa(const Slab<T>& A, unsigned voff, T (&a)[NV]) {
#pragma unroll
  for (int i = 0; i < NV; ++i) a[i] = A.ld(i, voff);
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
__device__ inline void precond_apply_mem(const Slab<T>& P, unsigned voff, const T (&r)[K], T (&z)[K]) {
  if constexpr (PC == PC_JACOBI) {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = P.ld(k, voff) * r[k];
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int j = 0; j <= k; ++j) {
        const T p = P.ld(pk(k, j), voff);
        z[k] += p * r[j];
        if (j != k) z[j] += p * r[k];
      }
    }
  }
}

// r'M^{-1}r, q'M^{-1}r and q'M^{-1}q at voxel n, with the preconditioner's
// entries streamed from memory (each used once, none held across the loop).
template <typename T, int PC, int K>
__device__ inline void precond_forms(const Slab<T>& P, unsigned voff, const T (&r)[K], const T (&q)[K], T& rr,
                                     T& qr, T& qq) {
  rr = qr = qq = 0;
  if constexpr (PC == PC_JACOBI) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T p = P.ld(k, voff);
      rr += p * r[k] * r[k];
      qr += p * q[k] * r[k];
      qq += p * q[k] * q[k];
    }
  } else {
    // u = M^{-1} r and v = M^{-1} q from the packed symmetric block, each
    // entry loaded once; then r'u, q'u and q'v
    T u[K], v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = v[k] = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int j = 0; j <= k; ++j) {
        const T p = P.ld(pk(k, j), voff);
        u[k] += p * r[j];
        v[k] += p * q[j];
        if (j != k) {
          u[j] += p * r[k];
          v[j] += p * q[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      rr += r[k] * u[k];
      qr += q[k] * u[k];
      qq += q[k] * v[k];
    }
  }
}

// The same forms from a preconditioner block held in registers.
template <typename T, int PC, int K>
__device__ inline void precond_forms_reg(const T (&P)[PSize<PC, K>::n], const T (&r)[K], const T (&q)[K], T& rr,
                                         T& qr, T& qq) {
  T u[K], v[K];
  precond_apply<T, PC, K>(P, r, u);
  precond_apply<T, PC, K>(P, q, v);
  rr = qr = qq = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    rr += r[k] * u[k];
    qr += q[k] * u[k];
    qq += q[k] * v[k];
  }
}

// Blocks (and, in the matvec, the preconditioner) held in registers across a
// work item's right-hand sides while they fit; larger K streams them per
// right-hand side (cache hits).
template <typename T, int K> struct HoldB { static constexpr bool v = sizeof(T) == 4 ? K <= 10 : K <= 8; };
// Regressors whose neighbour gathers may be in flight together in the matvec.
template <typename T, int K> struct GatherG { static constexpr int v = (sizeof(T) == 4 && K >= 12) ? 4 : K; };
// The refine kernel holds the FP64 block and the preconditioner in registers
// across a work item's right-hand sides while they fit.
template <typename T, int K> struct HoldRefine { static constexpr bool v = K <= 6; };
// The update kernel holds the preconditioner in registers while it fits.
template <typename T, int PC, int K> struct HoldP {
  static constexpr bool v = PC == PC_JACOBI || (sizeof(T) == 4 ? K <= 12 : K <= 8);
};

// Resident-wave request of the matvec kernel: 4 per SIMD (<= 128 VGPRs) while
// its per-voxel vectors fit, else 2.
template <typename T, int K> struct OccMV { static constexpr int v = sizeof(T) == 4 ? (K <= 6 ? 4 : 2) : (K <= 5 ? 4 : 2); };

// Per-RHS sums held in LDS: s_red[(slot * NV + v) * nwaves + wave].
// The NV values are summed over the wavefront together: M halving exchanges
// (distances 32, 16, ... for the next power of two 2^M >= NV) leave every lane
// with a partial of value lane >> (6 - M), and a butterfly over the remaining
// distances completes it.  The order of the additions is fixed.
template <int NV>
__device__ inline void wave_deposit(double* s_red, int slot, const double (&acc)[NV]) {
  constexpr int M = NV <= 1 ? 0 : NV <= 2 ? 1 : NV <= 4 ? 2 : 3;
  constexpr int NP = 1 << M;
  static_assert(NV <= 8, "at most 8 values per deposit");
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  double a[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) a[i] = i < NV ? acc[i] : 0.0;
#pragma unroll
  for (int st = 0; st < M; ++st) {
    const int dist = 32 >> st;
    const int half = NP >> (st + 1);
    const bool hi = (lane & dist) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double keep = hi ? a[i + half] : a[i];
      const double send = hi ? a[i] : a[i + half];
      a[i] = keep + __shfl_xor(send, dist, WAVE);
    }
  }
  double e = a[0];
#pragma unroll
  for (int dist = 32 >> M; dist > 0; dist >>= 1) e += __shfl_xor(e, dist, WAVE);
  const int idx = lane >> (6 - M);
  if ((lane & ((64 >> M) - 1)) == 0 && idx < NV) s_red[(slot * NV + idx) * nw + wv] = e;
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
      *(__attribute__((address_space(1))) double*)&pr.part[((size_t)v * pr.R + r) * pr.pstride + tile] = t;
    }
  }
  __syncthreads();   // s_red is reused by the next work item
}

struct Where {
  int p, tile, chunk, n, nn;
  int r0, r1;   // right-hand sides [r0, r1) of the work item
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

// Work items of a problem: the voxel tiles are cut into NXCD contiguous
// blocks (slabs of slices, the voxels being numbered slice by slice); items
// run block major, then right-hand-side chunk, then tile.  With the sweep
// above, each XCD then owns about one block for every chunk: the block's
// matrices and preconditioner stay in that XCD's L2 across all chunks, and the
// stencil's z-neighbours lie in the same block except at its two faces.
// The refine and addsol kernels (OUTER) use their own right-hand-side chunks.
template <bool OUTER = false>
__device__ inline Where locate(const Prob* __restrict__ probs, int nprob, int item) {
  Where w;
  w.p = find_prob<OUTER>(probs, nprob, item);
  const Prob& pr = probs[w.p];
  const int local = item - (OUTER ? pr.work_begin_o : pr.work_begin);
  const int nt = pr.op.ntiles, nc = OUTER ? pr.nchunks_o : pr.nchunks;
  const int tb = (nt + NXCD - 1) / NXCD;          // tiles per block
  const int b = local / (nc * tb);
  const int j = local - b * nc * tb;
  const int ntb = min(tb, nt - b * tb);           // tiles in block b (the last may be short)
  w.chunk = j / ntb;
  w.tile = b * tb + (j - w.chunk * ntb);
  const int rc = OUTER ? pr.Rco : pr.Rc;
  w.r0 = w.chunk * rc;
  w.r1 = min(pr.R, w.r0 + rc);
  const int N = pr.op.N;
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
  prof_add(pr, PF_REFINE_X0, pr.cfg.zero_guess && s.outer == 0);
  prof_add(pr, PF_ADDSOL_FRESH, pr.cfg.zero_guess && s.outer == 1);
  s.slots |= 1ull << (s.total_it < 63 ? s.total_it : 63);
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
// Addressing: every array is read through a buffer descriptor (Slab): the
// voxel's byte offset is the per-lane operand, the regressor (or packed
// block entry) row is a wave-uniform scalar offset.

// Byte offsets of the six neighbours of voxel nn for element size S.
template <int S>
__device__ __forceinline__ void voxel_offsets(const OpDev& op, int nn, unsigned (&nb)[6]) {
  const Slab<int> nbr(op.nbr, 6, op.N);
#pragma unroll
  for (int d = 0; d < 6; ++d) nb[d] = (unsigned)nbr.ld(d, (unsigned)nn * 4u) * S;
}

// y += S x for a symmetric K x K block S given by its packed entries
// s(i) = S[k][j], i = pk(k, j), each read once.
// Every product-sum is one explicit fused multiply-add, so that the result
// does not depend on where the compiler inlines the block product.
template <int K, typename V, typename GetS>
__device__ __forceinline__ void sym_apply(const GetS& s, const V (&x)[K], V (&y)[K]) {
  #pragma unroll
  for (int k = 0; k < K; ++k) {
  #pragma unroll
    for (int j = 0; j <= k; ++j) {
      const V v = s(pk(k, j));
      y[k] = fma_of(v, x[j], y[k]);
      if (j != k) y[j] = fma_of(v, x[k], y[j]);
    }
  }
}

// Refinement of right-hand side r at voxel w.nn: r64 = b - Q x (Q x = 0 for a
// zero start value), r = T(r64), p = M^{-1} r; acc = (||r64||^2, ||b||^2, r'p).
// getB(i), getP(i): packed entry i of the voxel's FP64 block and preconditioner.
template <typename T, int PC, int K, typename GetB, typename GetP>
__device__ __forceinline__ void refine_rhs(const Prob& pr, const Where& w, int r, bool x0, const unsigned (&nb8)[6],
                                           const GetB& getB, const GetP& getP, double (&acc)[3]) {
  const OpDev& op = pr.op;
  const int N = op.N;
  const unsigned o8 = (unsigned)w.nn * 8u, oT = (unsigned)w.nn * sizeof(T);
  const size_t off = (size_t)r * K * N;
  const Slab<double> xs(pr.x + off, K, N), bs(pr.b + off, K, N);
  double y[K];
  #pragma unroll
  for (int k = 0; k < K; ++k) y[k] = 0.0;
  if (!x0) {
    double xo[K];
  #pragma unroll
    for (int k = 0; k < K; ++k) {
      const double xc = xs.ld(k, o8);
      double s6 = 0.0;
  #pragma unroll
      for (int d = 0; d < 6; ++d) s6 += xc - xs.ld(k, nb8[d]);
      xo[k] = xc;
      y[k] = op.alpha64[k] * s6;
    }
    sym_apply<K>(getB, xo, y);
  }
  acc[0] = acc[1] = acc[2] = 0.0;
  T rt[K], z[K];
  #pragma unroll
  for (int k = 0; k < K; ++k) {
    const double bk = bs.ld(k, o8);
    const double rk = bk - y[k];
    acc[0] += rk * rk;
    acc[1] += bk * bk;
    rt[k] = (T)rk;
    z[k] = 0;
  }
  if constexpr (PC == PC_JACOBI) {
  #pragma unroll
    for (int k = 0; k < K; ++k) z[k] = getP(k) * rt[k];
  } else {
    sym_apply<K>(getP, rt, z);
  }
  #pragma unroll
  for (int k = 0; k < K; ++k) acc[2] += (double)rt[k] * (double)z[k];
  if (w.valid) {
    const Slab<T> rs((T*)pr.r + off, K, N), ps((T*)pr.p + off, K, N);   // first direction p = M^{-1} r
  #pragma unroll
    for (int k = 0; k < K; ++k) {
      rs.st(k, oT, rt[k]);
      ps.st(k, oT, z[k]);
    }
  } else {
    acc[0] = acc[1] = acc[2] = 0.0;
  }
}

template <typename T, int PC, int K>
__global__ __launch_bounds__(TILE, Occ<K>::outer) void k_refine(const Prob* __restrict__ probs, int nprob, int W) {
  constexpr int NB = Tri<K>::NB, NP = PSize<PC, K>::n;
  __shared__ double s_red[RCMAX * 3 * (TILE / WAVE)];
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate<true>(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int N = op.N;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_REFINE_ACT, PH_OUTER);
    const int r0 = w.r0, r1 = w.r1;
    if (!any_in_phase(pr, r0, r1, PH_OUTER)) continue;
    unsigned nb8[6];
    voxel_offsets<8>(op, w.nn, nb8);
    const unsigned o8 = (unsigned)w.nn * 8u, oT = (unsigned)w.nn * sizeof(T);
    const Slab<double> Bs(op.B64, NB, N);
    const Slab<T> Ps(OpT<T>::P(op), NP, N);
    if constexpr (HoldRefine<T, K>::v) {
      // the voxel's FP64 block and preconditioner, in registers across the
      // work item's right-hand sides
      double B[NB];
      T P[NP];
      load_soa(Bs, o8, B);
      load_soa(Ps, oT, P);
      const auto getB = [&](int i) { return B[i]; };
      const auto getP = [&](int i) { return P[i]; };
  #pragma unroll 1
      for (int r = r0; r < r1; ++r) {
        if (pr.st[r].phase != PH_OUTER) continue;
        double acc[3];
        refine_rhs<T, PC, K>(pr, w, r, pr.cfg.zero_guess && pr.st[r].outer == 0, nb8, getB, getP, acc);
        wave_deposit<3>(s_red, r - r0, acc);
      }
    } else {
      // streamed per right-hand side (cache hits)
      const auto getB = [&](int i) { return Bs.ld(i, o8); };
      const auto getP = [&](int i) { return Ps.ld(i, oT); };
  #pragma unroll 1
      for (int r = r0; r < r1; ++r) {
        if (pr.st[r].phase != PH_OUTER) continue;
        double acc[3];
        refine_rhs<T, PC, K>(pr, w, r, pr.cfg.zero_guess && pr.st[r].outer == 0, nb8, getB, getP, acc);
        wave_deposit<3>(s_red, r - r0, acc);
      }
    }
    flush_partials<3>(pr, s_red, r0, r1, w.tile, PH_OUTER);
  }
}

// q = Q p and the seven inner products of the step (see the header comment).
template <typename T, int PC, int K>
__global__ __launch_bounds__(TILE, (OccMV<T, K>::v)) void k_matvec(const Prob* __restrict__ probs, int nprob, int W) {
  constexpr int NB = Tri<K>::NB, NP = PSize<PC, K>::n;
  __shared__ double s_red[RCMAX * NPART * (TILE / WAVE)];
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int N = op.N;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_MATVEC_ACT, PH_INNER);
    const int r0 = w.r0, r1 = w.r1;
    if (!any_in_phase(pr, r0, r1, PH_INNER)) continue;
    unsigned nb[6];
    voxel_offsets<sizeof(T)>(op, w.nn, nb);
    const unsigned o = (unsigned)w.nn * sizeof(T);
    const Slab<T> Bs(OpT<T>::B(op), NB, N), Ps(OpT<T>::P(op), NP, N);
    T Bh[HoldB<T, K>::v ? NB : 1], Ph[HoldB<T, K>::v ? NP : 1];
    if constexpr (HoldB<T, K>::v) {
      load_soa(Bs, o, Bh);
      load_soa(Ps, o, Ph);
    }
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      if (pr.st[r].phase != PH_INNER) continue;
      const size_t off = (size_t)r * K * N;
      const Slab<T> ps((const T*)pr.p + off, K, N), rs((const T*)pr.r + off, K, N), qs((T*)pr.q + off, K, N);
      T pc[K], qv[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        const T c = ps.ld(k, o);
        T s6 = 0;
  #pragma unroll
        for (int d = 0; d < 6; ++d) s6 += c - ps.ld(k, nb[d]);
        pc[k] = c;
        qv[k] = OpT<T>::alpha(op, k) * s6;
        // bound the gathers in flight (GatherG<T, K> regressors at a time)
        if constexpr (GatherG<T, K>::v < K)
          if ((k + 1) % GatherG<T, K>::v == 0) __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (HoldB<T, K>::v) {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
  #pragma unroll
          for (int j = 0; j < K; ++j) qv[k] += Bh[pk(k, j)] * pc[j];
        }
      } else {
  #pragma unroll
        for (int k = 0; k < K; ++k) {
  #pragma unroll
          for (int j = 0; j <= k; ++j) {
            const T bkj = Bs.ld(pk(k, j), o);
            qv[k] += bkj * pc[j];
            if (j != k) qv[j] += bkj * pc[k];
          }
        }
      }
      T rv[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) rv[k] = rs.ld(k, o);
      T rPr, qPr, qPq;
      if constexpr (HoldB<T, K>::v)
        precond_forms_reg<T, PC, K>(Ph, rv, qv, rPr, qPr, qPq);
      else
        precond_forms<T, PC, K>(Ps, o, rv, qv, rPr, qPr, qPq);
      // the voxel's terms of the seven sums, in T; added up in double
      T spq = 0, srr = 0, sqr = 0, sqq = 0;
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        spq += pc[k] * qv[k];
        srr += rv[k] * rv[k];
        sqr += qv[k] * rv[k];
        sqq += qv[k] * qv[k];
      }
      double acc[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (w.valid) {
  #pragma unroll
        for (int k = 0; k < K; ++k) qs.st(k, o, qv[k]);
        acc[0] = spq;
        acc[1] = rPr;
        acc[2] = qPr;
        acc[3] = qPq;
        acc[4] = srr;
        acc[5] = sqr;
        acc[6] = sqq;
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
    const int r0 = w.r0, r1 = w.r1;
    if (!w.valid || !any_in_phase(pr, r0, r1, PH_INNER)) continue;
    const unsigned o = (unsigned)w.n * sizeof(T);
    const Slab<T> Ps(OpT<T>::P(op), NP, N);
    constexpr bool hold = HoldP<T, PC, K>::v;
    T P[hold ? NP : 1];
    if constexpr (hold) load_soa(Ps, o, P);
  #pragma unroll 1
    for (int r = r0; r < r1; ++r) {
      const RhsState& s = pr.st[r];
      if (s.phase != PH_INNER) continue;
      const T a = (T)s.a, beta = (T)s.beta;
      const bool fresh = s.inner_it == 1;
      const size_t off = (size_t)r * K * N;
      const Slab<T> ps((T*)pr.p + off, K, N), qs((const T*)pr.q + off, K, N), ds((T*)pr.d + off, K, N),
          rs((T*)pr.r + off, K, N);
      // every load of the voxel ahead of its first store: a wait for a load
      // also waits for the stores issued before it (one counter for both)
      T pv[K], rv[K], qv[K], dv[K], z[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        pv[k] = ps.ld(k, o);
        rv[k] = rs.ld(k, o);
        qv[k] = qs.ld(k, o);
        dv[k] = fresh ? (T)0 : ds.ld(k, o);
      }
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        dv[k] += a * pv[k];
        rv[k] -= a * qv[k];
        ds.st(k, o, dv[k]);
        rs.st(k, o, rv[k]);
      }
      if constexpr (hold)
        precond_apply<T, PC, K>(P, rv, z);
      else
        precond_apply_mem<T, PC, K>(Ps, o, rv, z);
  #pragma unroll
      for (int k = 0; k < K; ++k) ps.st(k, o, z[k] + beta * pv[k]);
    }
  }
}

// x += d (when valid) + a p (when the last step is pending) for right-hand
// sides whose inner solve has ended; x = d + a p after the first inner solve
// from a zero start value.
template <typename T, int K>
__global__ __launch_bounds__(TILE) void k_addsol(const Prob* __restrict__ probs, int nprob, int W) {
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const Where w = locate<true>(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    if (!w.valid) continue;
    const int N = pr.op.N;
    const int r0 = w.r0, r1 = w.r1;
    const unsigned oT = (unsigned)w.n * sizeof(T), o8 = (unsigned)w.n * 8u;
    for (int r = r0; r < r1; ++r) {
      const RhsState& s = pr.st[r];
      // with a zero start value, the first x += d writes x without reading it
      const bool fresh = pr.cfg.zero_guess && s.outer == 1;
      if (s.phase != PH_OUTER || !(s.has_d || s.pend || fresh)) continue;
      const bool hd = s.has_d != 0, hp = s.pend != 0;
      const double a = s.a;
      const size_t off = (size_t)r * K * N;
      const Slab<T> ds((const T*)pr.d + off, K, N), ps((const T*)pr.p + off, K, N);
      const Slab<double> xs(pr.x + off, K, N);
      double v[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        v[k] = fresh ? 0.0 : xs.ld(k, o8);
        if (hd) v[k] += (double)ds.ld(k, oT);
        if (hp) v[k] += a * (double)ps.ld(k, oT);
      }
  #pragma unroll
      for (int k = 0; k < K; ++k) xs.st(k, o8, v[k]);
    }
  }
}

}  // namespace gp
