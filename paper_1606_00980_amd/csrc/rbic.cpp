// Host side of the red-black incomplete Cholesky preconditioner (the M of
// Algorithm 2, steps 6-7, as a zero-fill factor in K x K voxel blocks on the
// two-colour voxel order): the colour split of an operator, the set-up of the
// red inverses and black Schur blocks, and the driver of the half-size PCG on
// the black Schur complement that PCG with this M reduces to (the algebra is
// stated at the top of rbic.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "gmrf.h"
#include "launch.hpp"
#include "runtime.hpp"

namespace gp {
namespace rt {

struct RbData {
  int NB = 0, NR = 0, ntB = 0, ntR = 0, ntN = 0;
  int *blk = nullptr, *red = nullptr, *nbB = nullptr, *nbR = nullptr, *vpos = nullptr;
  double *D64 = nullptr, *S64 = nullptr, *P64 = nullptr;
  float *D32 = nullptr, *S32 = nullptr, *P32 = nullptr;
  // the descriptors a solver round reads, uploaded in one copy per solve
  struct Desc {
    RbDev desc;
    Prob prob;
  };
  Desc* d_blob = nullptr;
  RbDev* d_desc = nullptr;   // &d_blob->desc
  Prob* d_prob = nullptr;    // &d_blob->prob
  Desc h{};                  // host source
  // the set-up's positive-definiteness flag has not been read yet (it is read
  // with the first states of the next solve)
  bool check_bad = false;
  // pinned host copies of the states and of that flag: both readbacks are
  // asynchronous, so one wait covers them
  RhsState* h_sts = nullptr;
  size_t h_sts_cap = 0;
  int* h_bad = nullptr;
  // shape of the last solve in each inner precision (0 FP64, 1 FP32) at the
  // tolerances it had: the union over its right-hand sides of the iteration
  // counts after which they took an outer step, and the largest such count.
  // The first round of the next solve at the same settings replays it.
  uint64_t hist_mask[2] = {0, 0};
  int hist_len[2] = {0, 0};
  double hist_tol[2][2] = {{0, 0}, {0, 0}};
  std::vector<std::pair<void*, size_t>> allocs;
};

namespace {

template <typename P>
int rb_alloc(gp_ctx* c, RbData* d, size_t count, P** p) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(P);
  void* v = nullptr;
  if (int st = dev_alloc(c, bytes, &v)) return st;
  d->allocs.emplace_back(v, bytes);
  *p = (P*)v;
  return GP_OK;
}

RbDev rb_dev(const gp_op* op) {
  const RbData& d = *op->rb;
  RbDev v;
  std::memset(&v, 0, sizeof(v));
  v.blk = d.blk;
  v.red = d.red;
  v.nbB = d.nbB;
  v.nbR = d.nbR;
  v.vpos = d.vpos;
  v.D64 = d.D64;
  v.D32 = d.D32;
  v.S64 = d.S64;
  v.S32 = d.S32;
  v.P64 = d.P64;
  v.P32 = d.P32;
  v.NB = d.NB;
  v.NR = d.NR;
  v.ntB = d.ntB;
  v.ntR = d.ntR;
  v.ntN = d.ntN;
  v.N = op->N;
  v.K = op->K;
  for (int k = 0; k < op->K; ++k) {
    v.alpha64[k] = op->alpha[k];
    v.alpha32[k] = (float)op->alpha[k];
  }
  return v;
}

// Colour every voxel by the parity of x + y + z, number each colour in
// increasing voxel order, and tabulate each voxel's neighbours by their
// position in the other colour.
int build_lists(gp_op* op) {
  gp_ctx* c = op->ctx;
  const int N = op->N;
  std::vector<int> lin(N), nbr((size_t)6 * N);
  HIPTRY(hipMemcpyAsync(lin.data(), op->lin, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipMemcpyAsync(nbr.data(), op->nbr, (size_t)6 * N * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  std::vector<int> colour(N), pos(N), blk, red;
  const long nx = op->nx, ny = op->ny;
  for (int n = 0; n < N; ++n) {
    const long l = lin[n];
    const long x = l % nx, y = (l / nx) % ny, z = l / (nx * ny);
    colour[n] = (int)((x + y + z) & 1);
    std::vector<int>& list = colour[n] ? blk : red;
    pos[n] = (int)list.size();
    list.push_back(n);
  }
  RbData* d = new RbData();
  op->rb = d;
  d->NB = (int)blk.size();
  d->NR = (int)red.size();
  d->ntB = (d->NB + TILE - 1) / TILE;
  d->ntR = (d->NR + TILE - 1) / TILE;
  d->ntN = (N + TILE - 1) / TILE;
  std::vector<int> vpos(N);
  for (int n = 0; n < N; ++n) vpos[n] = 2 * pos[n] + colour[n];
  auto table = [&](const std::vector<int>& list, std::vector<int>& out) -> bool {
    const size_t n = list.size();
    out.assign(6 * n, -1);
    for (size_t i = 0; i < n; ++i) {
      const int v = list[i];
      for (int dd = 0; dd < 6; ++dd) {
        const int u = nbr[(size_t)dd * N + v];
        if (u == v) continue;
        if (colour[u] == colour[v]) return false;
        out[(size_t)dd * n + i] = pos[u];
      }
    }
    return true;
  };
  std::vector<int> nbB, nbR;
  if (!table(blk, nbB) || !table(red, nbR)) return fail(GP_ERR_INVALID_ARG, "voxel graph is not two-colourable");
  const size_t NBt = (size_t)op->K * (op->K + 1) / 2;
  int st = GP_OK;
  if ((st = rb_alloc(c, d, blk.size(), &d->blk)) || (st = rb_alloc(c, d, red.size(), &d->red)) ||
      (st = rb_alloc(c, d, nbB.size(), &d->nbB)) || (st = rb_alloc(c, d, nbR.size(), &d->nbR)) ||
      (st = rb_alloc(c, d, vpos.size(), &d->vpos)) ||
      (st = rb_alloc(c, d, NBt * d->NB, &d->D64)) || (st = rb_alloc(c, d, NBt * d->NB, &d->D32)) ||
      (st = rb_alloc(c, d, NBt * d->NB, &d->S64)) || (st = rb_alloc(c, d, NBt * d->NB, &d->S32)) ||
      (st = rb_alloc(c, d, NBt * d->NR, &d->P64)) || (st = rb_alloc(c, d, NBt * d->NR, &d->P32)) ||
      (st = rb_alloc(c, d, 1, &d->d_blob)))
    return st;
  d->d_desc = &d->d_blob->desc;
  d->d_prob = &d->d_blob->prob;
  auto up = [&](int* dst, const std::vector<int>& src) {
    return src.empty() ? hipSuccess
                       : hipMemcpyAsync(dst, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
  };
  HIPTRY(up(d->blk, blk));
  HIPTRY(up(d->red, red));
  HIPTRY(up(d->nbB, nbB));
  HIPTRY(up(d->nbR, nbR));
  HIPTRY(up(d->vpos, vpos));
  HIPTRY(hipStreamSynchronize(c->stream));
  return GP_OK;
}

// The launches of one solver round for inner precision T.
template <typename T>
struct Round {
  gp_ctx* c;
  const RbDev& h;
  const RbData& d;
  int R, Rc, Rco, pstride, ntN;   // Rco: right-hand sides per workgroup of the outer step
  RhsState* st;
  double *part, *bb, *c64, *xB, *u64;
  T *dv, *rv, *pv, *qv, *uv;

  // x_B += d, refinement r = c - S x_B, finalise (right-hand sides waiting on it)
  // the first outer step of a solve from a zero start value: the split has
  // done its refinement, so only the finalisation is left
  int outer_first(hipStream_t q) const {
    HIPTRY(launch_rb_finalize(q, 0, R, d.d_prob, bb, h.ntB, ntN));
    return GP_OK;
  }
  int outer(hipStream_t q) const {
    PROFILED(c, GP_KERNEL_RB_ADDSOL, launch_rb_addsol(q, h, d.d_desc, R, Rco, st, xB, dv, pv));
    PROFILED(c, GP_KERNEL_RB_RED64, launch_rb_red(q, h, d.d_desc, R, Rc, st, PH_OUTER, xB, u64));
    PROFILED(c, GP_KERNEL_RB_REFINE, launch_rb_refine(q, h, d.d_desc, R, Rco, st, c64, xB, u64, rv, pv, part, pstride));
    HIPTRY(launch_rb_finalize(q, 0, R, d.d_prob, bb, h.ntB, ntN));
    return GP_OK;
  }
  // q = S p with the seven inner products, finalise, update
  int inner(hipStream_t q) const {
    PROFILED(c, GP_KERNEL_RB_RED, launch_rb_red(q, h, d.d_desc, R, Rc, st, PH_INNER, pv, uv));
    PROFILED(c, GP_KERNEL_RB_MATVEC, launch_rb_matvec(q, h, d.d_desc, R, Rc, st, pv, uv, rv, qv, part, pstride));
    HIPTRY(launch_rb_finalize(q, 1, R, d.d_prob, bb, h.ntB, ntN));
    PROFILED(c, GP_KERNEL_RB_UPDATE, launch_rb_update(q, h, d.d_desc, R, Rc, st, dv, rv, pv, qv));
    return GP_OK;
  }
  // `len` iterations, iteration i preceded by the outer step when bit i of
  // `mask` is set, and with `tail` one more outer step after the last when bit
  // len is set; len = 0: the outer step alone.
  // With first (the solve's first round from a zero start value) the round's
  // first outer step is outer_first.
  int round(hipStream_t q, int len, uint64_t mask, bool tail = false, bool first = false) const {
    if (len == 0) return first ? outer_first(q) : outer(q);
    for (int i = 0; i < len; ++i) {
      if (i < 64 && ((mask >> i) & 1))
        if (int e = (first && i == 0) ? outer_first(q) : outer(q)) return e;
      if (int e = inner(q)) return e;
    }
    if (tail && len < 64 && ((mask >> len) & 1)) return outer(q);
    return GP_OK;
  }
};

// Algorithmic HBM bytes of the launches of one solve, from the work counters:
// every vector entry a launch needs read or written once (a gathered
// neighbour vector counted once), the blocks once per launch with work.
void rb_account(gp_ctx* c, const gp_op* op, int R, size_t tsz, bool zero_guess, const std::vector<long long>& pf) {
  const RbData& d = *op->rb;
  const double K = op->K, NB = d.NB, NR = d.NR, N = op->N, ts = (double)tsz, NBt = K * (K + 1) / 2;
  const double mv = (double)pf[PF_MATVEC_RHS], ref = (double)pf[PF_REFINE_RHS];
  // red stage: the black vector read, u written; the red inverses
  prof_add(c, GP_KERNEL_RB_RED, mv * NR, mv * K * (NB + NR) * ts + pf[PF_MATVEC_ACT] * NBt * NR * ts);
  // the same in FP64 on x_B for refinements from a non-zero x
  const double ref_x = ref - (double)pf[PF_REFINE_X0];
  prof_add(c, GP_KERNEL_RB_RED64, ref_x * NR, ref_x * K * (NB + NR) * 8 + pf[PF_REFINE_ACT] * NBt * NR * 8);
  // black stage: p, u, r read, q written; Q_mm and the Schur inverses
  prof_add(c, GP_KERNEL_RB_MATVEC, mv * NB, mv * K * (3 * NB + NR) * ts + pf[PF_MATVEC_ACT] * 2 * NBt * NB * ts);
  // p, q, r, d read (d not on the first step), d, r, p written; Schur inverses
  const double up = (double)pf[PF_UPDATE_RHS], fresh = (double)pf[PF_UPDATE_FRESH];
  prof_add(c, GP_KERNEL_RB_UPDATE, up * NB,
           (up - fresh) * 7 * K * NB * ts + fresh * 6 * K * NB * ts + pf[PF_UPDATE_ACT] * NBt * NB * ts);
  // c, x_B, u64 read, r and p written; FP64 Q_mm and the Schur inverses in
  // the inner precision (the first step from a zero start value is the
  // split's)
  const double x0 = (double)pf[PF_REFINE_X0];
  prof_add(c, GP_KERNEL_RB_REFINE, (ref - x0) * NB,
           (ref - x0) * K * (2 * NB * 8 + NR * 8 + 2 * NB * ts) + pf[PF_REFINE_ACT] * NBt * NB * (8 + ts));
  // x_B read (not on the first step from a zero start value) and written, d
  // and/or the pending step's p read
  const double ad = (double)pf[PF_ADDSOL_D], ap = (double)pf[PF_ADDSOL_P], af = (double)pf[PF_ADDSOL_FRESH];
  const double an = std::max(std::max(ad, ap), af);
  prof_add(c, GP_KERNEL_RB_ADDSOL, an * NB, an * K * NB * 16 - af * K * NB * 8 + (ad + ap) * K * NB * ts);
  // split: b read, t written and read, x read and x_B written (unless the start
  // value is zero), c written, the red inverses read, and from a zero start
  // value r and p of the first refinement written; recovery: x_B, t and u
  // read, x written
  prof_add(c, GP_KERNEL_RB_EDGE, 2.0 * R * N,
           R * K * 8 * (N + 2 * NR + (zero_guess ? 0 : 2 * NB) + NB) + x0 * K * 2 * NB * ts +
               R * K * 8 * (NB + 2 * NR + N) + NBt * NR * 8);
}

}  // namespace

void rb_release(gp_op* op) {
  if (!op->rb) return;
  for (auto& a : op->rb->allocs) dev_free(op->ctx, a.first, a.second);
  if (op->rb->h_sts) (void)hipHostFree(op->rb->h_sts);
  if (op->rb->h_bad) (void)hipHostFree(op->rb->h_bad);
  delete op->rb;
  op->rb = nullptr;
}

int rb_build(gp_op* op) {
  gp_ctx* c = op->ctx;
  if (!op->rb) {
    if (int st = build_lists(op)) {
      rb_release(op);
      return st;
    }
  }
  RbData& d = *op->rb;
  const RbDev h = rb_dev(op);
  if (int st = reset_bad(op)) return st;
  PROFILED(c, GP_KERNEL_PRECOND, launch_rb_setup(c->stream, h, op->B64, d.P64, d.P32, d.D64, d.D32, d.S64, d.S32,
                                                  op->d_bad));
  // the flag is read with the first states of the solve that follows (one
  // wait fewer); that solve then fails with GP_ERR_NOT_SPD
  d.check_bad = true;
  op->pc_built = GP_PRECOND_RB_IC0;
  return GP_OK;
}

int rb_solve(gp_ctx* c, gp_op* op, const std::vector<RbItem>& items, const gp_opts& o) {
  const auto t0 = std::chrono::steady_clock::now();
  long Rl = 0;
  for (const RbItem& it : items) Rl += it.R;
  if (Rl > 65535) return fail(GP_ERR_INVALID_ARG, "at most 65535 right-hand sides per operator with the red-black preconditioner");
  const int R = (int)Rl;
  if (R == 0) return GP_OK;
  if (!op->rb || op->pc_built != GP_PRECOND_RB_IC0) return fail(GP_ERR_INVALID_ARG, "preconditioner not built");
  RbData& d = *op->rb;
  const bool f32 = o.precision == GP_PREC_FP32_REFINE64;
  const size_t tsz = f32 ? sizeof(float) : sizeof(double);
  const int K = op->K, ntN = d.ntN, pstride = std::max(d.ntB, 1);
  const size_t nbv = (size_t)R * K * d.NB, nrv = (size_t)R * K * d.NR;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1), 256);
    return at;
  };
  const size_t o_st = take((size_t)R * sizeof(RhsState)), o_part = take((size_t)NPART * R * pstride * 8),
               o_bb = take((size_t)R * std::max(ntN, 1) * 8), o_c = take(nbv * 8), o_x = take(nbv * 8),
               o_u64 = take(nrv * 8), o_t = take(nrv * 8), o_d = take(nbv * tsz), o_r = take(nbv * tsz), o_p = take(nbv * tsz),
               o_q = take(nbv * tsz), o_u = take(nrv * tsz), o_prof = take(NPROF * sizeof(long long));
  if (int st = ensure_ws(c, off)) return st;
  char* ws = (char*)c->ws;
  hipStream_t s = c->stream;
  RhsState* sts = (RhsState*)(ws + o_st);
  double* part = (double*)(ws + o_part);
  double* bb = (double*)(ws + o_bb);
  double* c64 = (double*)(ws + o_c);
  double* xB = (double*)(ws + o_x);
  double* u64 = (double*)(ws + o_u64);
  double* t64 = (double*)(ws + o_t);   // t = Q_nn^{-1} b_n of the split, kept for the recovery

  long long* prof = c->prof_on ? (long long*)(ws + o_prof) : nullptr;
  d.h.desc = rb_dev(op);
  d.h.desc.prof = prof;
  d.h.desc.zero_start = o.zero_guess ? 1 : 0;
  std::memset(&d.h.prob, 0, sizeof(Prob));
  d.h.prob.prof = prof;
  d.h.prob.st = sts;
  d.h.prob.part = part;
  d.h.prob.R = R;
  d.h.prob.pstride = pstride;
  d.h.prob.cfg = SolveCfg{o.tol, f32 ? o.inner_tol : 0.0, o.max_iter, o.max_outer, o.zero_guess ? 1 : 0, 0};
  HIPTRY(hipMemcpyAsync(d.d_blob, &d.h, sizeof(RbData::Desc), hipMemcpyHostToDevice, s));
  HIPTRY(hipMemsetAsync(sts, 0, (size_t)R * sizeof(RhsState), s));
  if (prof) HIPTRY(hipMemsetAsync(prof, 0, NPROF * sizeof(long long), s));
  // per item: c = b_B - E' D_R^{-1} b_R, x_B, ||b||^2 partials, t = D_R^{-1} b_R;
  // from a zero start value also the first refinement (r = c, p = S_m^{-1} r)
  {
    size_t r0 = 0;
    for (const RbItem& it : items) {
      RbSplitFirst first{nullptr, nullptr, part, (size_t)R * pstride, pstride, (int)r0, f32};
      if (o.zero_guess) {
        first.r = ws + o_r + r0 * K * d.NB * tsz;
        first.p = ws + o_p + r0 * K * d.NB * tsz;
      }
      if (it.R > 0)
        PROFILED(c, GP_KERNEL_RB_EDGE,
                 launch_rb_split(s, d.h.desc, it.R, it.b, it.x, o.zero_guess ? 1 : 0, t64 + r0 * K * d.NR,
                                 c64 + r0 * K * d.NB, xB + r0 * K * d.NB, bb + r0 * ntN, first));
      r0 += (size_t)it.R;
    }
  }

  const int chunk = o.chunk > 0 ? o.chunk : 8;
  // right-hand sides per workgroup: the largest of 8, 4, 2 that still leaves
  // at least 1024 workgroups (four per compute unit), else 1
  int Rc = o.rhs_tile > 0 ? std::min(o.rhs_tile, RCMAX) : 1;
  if (o.rhs_tile <= 0)
    for (int cand : {8, 4, 2})
      if ((long)d.ntB * ((R + cand - 1) / cand) >= 1024) {
        Rc = cand;
        break;
      }
  Rc = std::max(1, std::min(Rc, R));
  // the FP64 refinement and x_B += d take one right-hand side per workgroup
  // (holding the FP64 blocks across several costs the refinement occupancy);
  // the FP64 red stage takes the inner chunks
  const int Rco = 1;
  const bool graphs = c->use_graphs && !c->prof_on;
  const std::string key = "rb|" + std::to_string((uintptr_t)d.d_desc) + "|" + std::to_string((uintptr_t)ws) + "|" +
                          std::to_string(K) + "," + std::to_string(d.NB) + "," + std::to_string(d.NR) + "," +
                          std::to_string(R) + "," + (f32 ? "f" : "d") + std::to_string(Rc);
  auto run_round = [&](int len, uint64_t mask, bool tail, bool first) -> int {
    auto enq = [&](hipStream_t q) -> int {
      if (f32) {
        const Round<float> rd{c, d.h.desc, d, R, Rc, Rco, pstride, ntN, sts, part, bb, c64, xB, u64,
                              (float*)(ws + o_d), (float*)(ws + o_r), (float*)(ws + o_p), (float*)(ws + o_q),
                              (float*)(ws + o_u)};
        return rd.round(q, len, mask, tail, first);
      }
      const Round<double> rd{c, d.h.desc, d, R, Rc, Rco, pstride, ntN, sts, part, bb, c64, xB, u64,
                             (double*)(ws + o_d), (double*)(ws + o_r), (double*)(ws + o_p), (double*)(ws + o_q),
                             (double*)(ws + o_u)};
      return rd.round(q, len, mask, tail, first);
    };
    if (!graphs) return enq(s);
    return graph_replay(c, key + "|" + std::to_string(len) + "/" + std::to_string(mask) + (tail ? "t" : "") +
                               (first ? "f" : ""),
                        enq);
  };

  // rounds planned as for the main solver: the outer step first, then
  // iterations with the outer step where inner solves are expected to end
  std::vector<RhsState> hs(R);
  if (d.h_sts_cap < (size_t)R) {
    if (d.h_sts) HIPTRY(hipHostFree(d.h_sts));
    d.h_sts = nullptr;
    d.h_sts_cap = 0;
    HIPTRY(hipHostMalloc((void**)&d.h_sts, (size_t)R * sizeof(RhsState), hipHostMallocDefault));
    d.h_sts_cap = (size_t)R;
  }
  if (!d.h_bad) HIPTRY(hipHostMalloc((void**)&d.h_bad, sizeof(int), hipHostMallocDefault));
  int n_outer = R, n_inner = 0;
  int round_len = chunk;
  uint64_t round_mask = f32 && o.chunk > 0 ? ~0ull : 1ull;
  bool tail = false;
  const int hp = f32 ? 1 : 0;
  if (o.chunk <= 0 && d.hist_mask[hp] && d.hist_tol[hp][0] == o.tol && d.hist_tol[hp][1] == o.inner_tol) {
    // the previous solve's shape: its outer steps where they were taken, and
    // the last of them (the final refinement) after the round's iterations
    round_len = d.hist_len[hp];
    round_mask = d.hist_mask[hp];
    tail = true;
  }
  const long max_rounds = (long)o.max_iter + 4L * o.max_outer + 8;
  long rounds = 0;
  // x in the caller's layout (repeated if a later round changes x_B)
  auto recover = [&]() -> int {
    size_t r0 = 0;
    for (const RbItem& it : items) {
      if (it.R > 0)
        PROFILED(c, GP_KERNEL_RB_EDGE,
                 launch_rb_recover(s, d.h.desc, it.R, sts + r0, t64 + r0 * K * d.NR, u64 + r0 * K * d.NR,
                                   xB + r0 * K * d.NB, it.x));
      r0 += (size_t)it.R;
    }
    return GP_OK;
  };
  bool recovered = false;
  int bad = INT_MAX;
  while (n_outer > 0 || n_inner > 0) {
    if (++rounds > max_rounds) return fail(GP_ERR_DEVICE, "solver driver made no progress");
    // the first round's first outer step (mask bit 0, set in every first round)
    // is the finalisation alone when the split took the refinement
    const bool first = rounds == 1 && o.zero_guess;
    if (int st = (!f32 && n_inner == 0 && !tail) ? run_round(0, 1, false, first)
                                                 : run_round(round_len, round_mask, tail, first))
      return st;
    // a replayed shape usually ends the solve: recover before waiting
    if (tail)
      if (int st = recover()) return st;
    recovered = tail;
    tail = false;
    HIPTRY(hipMemcpyAsync(d.h_sts, sts, (size_t)R * sizeof(RhsState), hipMemcpyDeviceToHost, s));
    const bool check = d.check_bad;
    if (check) HIPTRY(hipMemcpyAsync(d.h_bad, op->d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    std::memcpy(hs.data(), d.h_sts, (size_t)R * sizeof(RhsState));
    if (check) bad = *d.h_bad;
    if (check) {
      d.check_bad = false;
      if (bad != INT_MAX) {
        op->pc_built = -1;
        return fail(GP_ERR_NOT_SPD, "preconditioner block of voxel " + std::to_string(bad) + " is not positive definite");
      }
    }
    n_outer = n_inner = 0;
    for (const RhsState& h : hs) {
      n_outer += h.phase == PH_OUTER;
      n_inner += h.phase == PH_INNER;
    }
    if (n_outer > 0 || n_inner > 0) recovered = false;
    plan_round(hs, o, f32, chunk, &round_len, &round_mask);
  }
  if (!recovered)
    if (int st = recover()) return st;
  HIPTRY(hipStreamSynchronize(s));
  if (prof) {
    std::vector<long long> pf(NPROF);
    HIPTRY(hipMemcpy(pf.data(), prof, NPROF * sizeof(long long), hipMemcpyDeviceToHost));
    rb_account(c, op, R, tsz, o.zero_guess != 0, pf);
    if (int e = prof_resolve(c)) return e;
  }
  {
    uint64_t m = 0;
    for (const RhsState& h : hs) m |= h.slots;
    int len = 0;
    while (len < 63 && (m >> (len + 1)) != 0) ++len;
    // a shape that reaches the last bit (outer steps after 63 or more
    // iterations) is not replayed
    d.hist_mask[hp] = len < 63 ? m : 0;
    d.hist_len[hp] = len;
    d.hist_tol[hp][0] = o.tol;
    d.hist_tol[hp][1] = o.inner_tol;
  }
  const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  int ret = GP_OK;
  size_t r0 = 0;
  for (const RbItem& it : items) {
    for (int r = 0; r < it.R; ++r) {
      const RhsState& h = hs[r0 + r];
      const int status = h.phase == PH_DONE ? h.status : GP_ERR_NOT_CONVERGED;
      if (it.stats) it.stats[r] = gp_stats{status, h.total_it, h.outer, 0, h.relres, us};
      if (status != GP_OK && ret == GP_OK) ret = status;
    }
    r0 += (size_t)it.R;
  }
  if (ret == GP_ERR_NOT_CONVERGED) return fail(ret, "some right-hand sides did not reach the tolerance");
  if (ret == GP_ERR_BREAKDOWN) return fail(ret, "PCG breakdown (non-finite value or loss of definiteness)");
  return ret;
}

}  // namespace rt
}  // namespace gp
