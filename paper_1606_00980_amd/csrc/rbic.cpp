// Host side of the red-black incomplete Cholesky preconditioner (the M of
// Algorithm 2, steps 6-7, as a zero-fill factor in K x K voxel blocks on the
// two-colour voxel order): the colour split of an operator, the set-up of the
// red inverses and black Schur blocks, and the driver of the half-size PCG on
// the black Schur complement that PCG with this M reduces to (the algebra is
// stated at the top of rbic.hpp).  Several operators are solved together: the
// members of one solve are grouped by K and every solver-round kernel is one
// launch per group over the members' descriptors.
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
  // the set-up's positive-definiteness flag has not been read yet (it is read
  // with the first states of the next solve)
  bool check_bad = false;
  int* h_bad = nullptr;   // pinned host copy of that flag
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
      (st = rb_alloc(c, d, NBt * d->NR, &d->P64)) || (st = rb_alloc(c, d, NBt * d->NR, &d->P32)))
    return st;
  HIPTRY(hipHostMalloc((void**)&d->h_bad, sizeof(int), hipHostMallocDefault));
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

}  // namespace

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
  // Work items run block by block: within a block of tiles, every chunk of
  // right-hand sides sweeps the block's tiles before the next chunk starts,
  // so that a tile's z-neighbours (one plane of colour positions away) were
  // just gathered for the same chunk and are still in L2, and the block's
  // voxel blocks stay there across the chunks.  A block spans two planes
  // and two tiles, and its voxel blocks at most 1.5 MB.
  const size_t tile_blocks = (size_t)2 * (op->K * (op->K + 1) / 2) * 256 * sizeof(float);
  const int cap = std::max<int>(4, (int)(((size_t)1536 << 10) / tile_blocks));
  auto per_block = [&](int npos, int ntiles) {
    const int reach = (npos / std::max(op->nz, 1) + 255) / 256;   // tiles per z-plane of positions
    return std::max(1, std::min({2 * reach + 2, cap, std::max(ntiles, 1)}));
  };
  v.tbB = per_block(d.NB, d.ntB);
  v.tbR = per_block(d.NR, d.ntR);
  for (int k = 0; k < op->K; ++k) {
    v.alpha64[k] = op->alpha[k];
    v.alpha32[k] = (float)op->alpha[k];
  }
  return v;
}

void rb_release(gp_op* op) {
  if (!op->rb) return;
  for (auto& a : op->rb->allocs) dev_free(op->ctx, a.first, a.second);
  if (op->rb->h_bad) (void)hipHostFree(op->rb->h_bad);
  delete op->rb;
  op->rb = nullptr;
}

namespace {

int rb_lists(gp_op* op) {
  if (op->rb) return GP_OK;
  if (int st = build_lists(op)) {
    rb_release(op);
    return st;
  }
  return GP_OK;
}

// The blocks of op's preconditioner, enqueued on q (the colour lists built).
int rb_setup_on(gp_op* op, hipStream_t q) {
  gp_ctx* c = op->ctx;
  RbData& d = *op->rb;
  const RbDev h = rb_dev(op);
  HIPTRY(hipMemsetD32Async((hipDeviceptr_t)op->d_bad, INT_MAX, 1, q));
  PROFILED(c, GP_KERNEL_PRECOND, launch_rb_setup(q, h, op->B64, d.P64, d.P32, d.D64, d.D32, d.S64, d.S32, op->d_bad));
  // the flag is read with the first states of the solve that follows (one
  // wait fewer); that solve then fails with GP_ERR_NOT_SPD
  d.check_bad = true;
  op->pc_built = GP_PRECOND_RB_IC0;
  return GP_OK;
}

template <typename F>
int fork_items(gp_ctx* c, hipStream_t s, int n, F&& launch);

}  // namespace

int rb_build(gp_op* op) {
  if (int st = rb_lists(op)) return st;
  return rb_setup_on(op, op->ctx->stream);
}

int rb_build_ops(gp_ctx* c, const std::vector<gp_op*>& ops) {
  for (gp_op* op : ops)
    if (int st = rb_lists(op)) return st;
  return fork_items(c, c->stream, (int)ops.size(), [&](hipStream_t q, int i) { return rb_setup_on(ops[i], q); });
}

int rb_check_built(gp_op* op) {
  RbData& d = *op->rb;
  if (!d.check_bad) return GP_OK;
  HIPTRY(hipMemcpyAsync(d.h_bad, op->d_bad, sizeof(int), hipMemcpyDeviceToHost, op->ctx->stream));
  HIPTRY(hipStreamSynchronize(op->ctx->stream));
  d.check_bad = false;
  if (*d.h_bad != INT_MAX) {
    op->pc_built = -1;
    return fail(GP_ERR_NOT_SPD, "preconditioner block of voxel " + std::to_string(*d.h_bad) + " is not positive definite");
  }
  return GP_OK;
}

// ------------------------------------------------------------ members
namespace {
// bytes of one workspace slot (every slot at least 256, also an empty one)
size_t slot_bytes(size_t bytes) { return align_up(std::max<size_t>(bytes, 1), 256); }
// right-hand sides per row set of the red-stage vector u: pairs for an FP32
// solve of two or more with K <= UPAIR_KMAX, else one
int u_width(const gp_op* op, int R, bool f32) { return f32 && op->K <= UPAIR_KMAX && R >= 2 ? 2 : 1; }
// entries of u (an odd R takes a pair's worth for its last one)
size_t u_entries(const gp_op* op, int R, bool f32) {
  const int w = u_width(op, R, f32);
  return (size_t)((R + w - 1) / w * w) * op->K * op->rb->NR;
}
}  // namespace

size_t rb_member_bytes(const gp_op* op, int R, bool f32) {
  const RbData& d = *op->rb;
  const size_t tsz = f32 ? sizeof(float) : sizeof(double);
  const size_t nbv = (size_t)R * op->K * d.NB, nrv = (size_t)R * op->K * d.NR;
  const int pstride = std::max(d.ntB, 1);
  size_t b = 0;
  b += slot_bytes((size_t)NPART * R * pstride * 8);       // partials
  b += slot_bytes((size_t)R * std::max(d.ntN, 1) * 8);    // ||b||^2 partials
  b += 2 * slot_bytes(nbv * 8);                           // c64, xB
  b += 2 * slot_bytes(nrv * 8);                           // u64, t64
  b += 4 * slot_bytes(nbv * tsz);                         // d, r, p, q
  b += slot_bytes(u_entries(op, R, f32) * tsz);           // u of the red stage
  b += slot_bytes(NPROF * sizeof(long long));             // work counters
  return b;
}

void rb_member(gp_op* op, int R, bool f32, char* mem, RhsState* st, const SolveCfg& cfg, bool prof, RbMember* out) {
  const RbData& d = *op->rb;
  const size_t tsz = f32 ? sizeof(float) : sizeof(double);
  const size_t nbv = (size_t)R * op->K * d.NB, nrv = (size_t)R * op->K * d.NR;
  const int pstride = std::max(d.ntB, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* at = mem + off;
    off += slot_bytes(bytes);
    return at;
  };
  RbProb& P = out->desc;
  std::memset(&P, 0, sizeof(P));
  P.rb = rb_dev(op);
  P.pr.part = (double*)take((size_t)NPART * R * pstride * 8);
  P.bb = (double*)take((size_t)R * std::max(d.ntN, 1) * 8);
  P.c64 = (double*)take(nbv * 8);
  P.xB = (double*)take(nbv * 8);
  P.u64 = (double*)take(nrv * 8);
  out->t64 = (double*)take(nrv * 8);
  P.d = take(nbv * tsz);
  P.r = take(nbv * tsz);
  P.p = take(nbv * tsz);
  P.q = take(nbv * tsz);
  P.u = take(u_entries(op, R, f32) * tsz);
  P.uw = u_width(op, R, f32);
  long long* pf = (long long*)take(NPROF * sizeof(long long));
  out->prof = prof ? pf : nullptr;
  P.rb.prof = out->prof;
  P.rb.zero_start = cfg.zero_guess;
  P.pr.prof = out->prof;
  P.pr.st = st;
  P.pr.R = R;
  P.pr.pstride = pstride;
  P.pr.cfg = cfg;
  out->op = op;
  out->R = R;
}

std::vector<RbGroup> rb_groups(RbProb* h, int n, int rhs_tile, bool outer_chunks) {
  std::vector<RbGroup> gs;
  const int fpb = finalize_rhs_per_block();
  for (int j = 0; j < n; ++j) {
    if (gs.empty() || gs.back().K != h[j].rb.K) gs.push_back(RbGroup{h[j].rb.K, j, 0, 0, 0, 0, 0, 1});
    gs.back().count += 1;
  }
  for (RbGroup& g : gs) {
    // right-hand sides per inner work item: the tuned or requested value, else
    // the largest of 8, 4, 2 that still leaves at least 1024 workgroups in the
    // group's launch (four per compute unit)
    int Rc = rhs_tile > 0 ? std::min(rhs_tile, RCMAX) : 1;
    if (rhs_tile <= 0)
      for (int cand : {8, 4, 2}) {
        long items = 0;
        for (int j = g.first; j < g.first + g.count; ++j)
          items += (long)h[j].rb.ntB * ((h[j].pr.R + cand - 1) / cand);
        if (items >= 1024) {
          Rc = cand;
          break;
        }
      }
    int F = 0;
    for (int j = g.first; j < g.first + g.count; ++j) {
      RbProb& P = h[j];
      P.Rc = std::max(1, std::min(Rc, P.pr.R));
      P.nch = (P.pr.R + P.Rc - 1) / P.Rc;
      // pairs only where work items hold them: with one right-hand side per
      // item u keeps one per row (its gathers contiguous; the memory carved
      // for pairs holds that layout too)
      if (P.Rc < 2) P.uw = 1;
      g.uw = std::max(g.uw, P.uw);
      P.wB = g.WB;
      g.WB += P.rb.ntB * P.nch;
      P.wR = g.WR;
      g.WR += P.rb.ntR * P.nch;
      // the FP64 refinement and x_B += d: one right-hand side per work item
      // (holding the FP64 blocks across several costs the refinement
      // occupancy), or the inner chunks when most right-hand sides of a launch
      // are not in the outer phase (the serving loop), so that the launch does
      // not consist of empty workgroups
      P.Rco = outer_chunks ? P.Rc : 1;
      P.ncho = (P.pr.R + P.Rco - 1) / P.Rco;
      P.wO = g.WO;
      g.WO += P.rb.ntB * P.ncho;
      P.pr.fin_begin = F;
      F += (P.pr.R + fpb - 1) / fpb;
    }
    g.F = F;
  }
  return gs;
}

// ------------------------------------------------------------ rounds
namespace {

template <typename T>
int outer_step(gp_ctx* c, hipStream_t q, const RbGroup& g, const RbProb* dp, bool pf) {
  PROFILED_IF(pf, c, GP_KERNEL_RB_ADDSOL, launch_rbg_addsol<T>(q, g.K, dp, g.count, g.WO));
  PROFILED_IF(pf, c, GP_KERNEL_RB_RED64, launch_rbg_red64(q, g.K, dp, g.count, g.WR));
  PROFILED_IF(pf, c, GP_KERNEL_RB_REFINE, launch_rbg_refine<T>(q, g.K, dp, g.count, g.WO));
  HIPTRY(launch_rbg_finalize(q, 0, dp, g.count, g.F));
  return GP_OK;
}

template <typename T>
int inner_step(gp_ctx* c, hipStream_t q, const RbGroup& g, const RbProb* dp, bool pf) {
  PROFILED_IF(pf, c, GP_KERNEL_RB_RED, launch_rbg_red<T>(q, g.K, dp, g.count, g.WR));
  PROFILED_IF(pf, c, GP_KERNEL_RB_MATVEC, launch_rbg_matvec<T>(q, g.K, dp, g.count, g.WB, g.uw == 2));
  HIPTRY(launch_rbg_finalize(q, 1, dp, g.count, g.F));
  PROFILED_IF(pf, c, GP_KERNEL_RB_UPDATE, launch_rbg_update<T>(q, g.K, dp, g.count, g.WB));
  return GP_OK;
}

// One group's round: `len` iterations, iteration i preceded by the outer step
// when bit i of `mask` is set, and with `tail` one more outer step after the
// last when bit len is set; len = 0: the outer step alone.  With `first` (the
// solve's first round from a zero start value) the round's first outer step
// is the finalisation alone: the split has taken the first refinement.
template <typename T>
int group_round(gp_ctx* c, hipStream_t q, const RbGroup& g, const RbProb* dp, int len, uint64_t mask, bool tail,
                bool first, bool pf) {
  if (len == 0) {
    if (first) {
      HIPTRY(launch_rbg_finalize(q, 0, dp, g.count, g.F));
      return GP_OK;
    }
    return outer_step<T>(c, q, g, dp, pf);
  }
  for (int i = 0; i < len; ++i) {
    if (i < 64 && ((mask >> i) & 1)) {
      if (first && i == 0) {
        HIPTRY(launch_rbg_finalize(q, 0, dp, g.count, g.F));
      } else if (int e = outer_step<T>(c, q, g, dp, pf)) {
        return e;
      }
    }
    if (int e = inner_step<T>(c, q, g, dp, pf)) return e;
  }
  if (tail && len < 64 && ((mask >> len) & 1)) return outer_step<T>(c, q, g, dp, pf);
  return GP_OK;
}

// Enqueues launch(q, i) for n independent launches: in order on s for fewer
// than FORK_MIN (or while profiling, so that each launch is timed alone), else
// dealt over four branch streams forked from s and joined back into it.  The
// fork and join cost more than they save for a few launches (the whole-brain
// step's two items: 1.85 against 1.75 ms per step forked) and less for many
// (16 uneven operators, 32 items: 17.0 against 17.35 ms).
constexpr int FORK_MIN = 8;
template <typename F>
int fork_items(gp_ctx* c, hipStream_t s, int n, F&& launch) {
  if (n < FORK_MIN || c->prof_on) {
    for (int i = 0; i < n; ++i)
      if (int st = launch(s, i)) return st;
    return GP_OK;
  }
  const int nb = std::min(n, 4);
  if (int e = ensure_branches(c, (size_t)nb)) return e;
  HIPTRY(hipEventRecord(c->branch_ev[0], s));
  for (int b = 0; b < nb; ++b) HIPTRY(hipStreamWaitEvent(c->branch[b], c->branch_ev[0], 0));
  int st = GP_OK;
  for (int i = 0; i < n && st == GP_OK; ++i) st = launch(c->branch[i % nb], i);
  // joined also after a failed launch: s then orders after everything enqueued
  for (int b = 0; b < nb; ++b) {
    HIPTRY(hipEventRecord(c->branch_ev[1 + b], c->branch[b]));
    HIPTRY(hipStreamWaitEvent(s, c->branch_ev[1 + b], 0));
  }
  return st;
}

}  // namespace

int rb_enqueue_round(gp_ctx* c, hipStream_t q, bool f32, const std::vector<RbGroup>& gs, const RbProb* d_probs,
                     int len, uint64_t mask, bool tail, bool first, bool profiled, bool branched) {
  const bool pf = profiled && c->prof_on;
  auto one = [&](hipStream_t s, const RbGroup& g) -> int {
    const RbProb* dp = d_probs + g.first;
    return f32 ? group_round<float>(c, s, g, dp, len, mask, tail, first, pf)
               : group_round<double>(c, s, g, dp, len, mask, tail, first, pf);
  };
  if (!branched || gs.size() <= 1) {
    for (const RbGroup& g : gs)
      if (int e = one(q, g)) return e;
    return GP_OK;
  }
  // each group on a branch stream forked from q and joined back into it, so
  // that a captured round runs the groups as parallel graph branches
  if (int e = ensure_branches(c, gs.size())) return e;
  HIPTRY(hipEventRecord(c->branch_ev[0], q));
  for (size_t g = 0; g < gs.size(); ++g) {
    hipStream_t b = c->branch[g];
    HIPTRY(hipStreamWaitEvent(b, c->branch_ev[0], 0));
    if (int e = one(b, gs[g])) return e;
    HIPTRY(hipEventRecord(c->branch_ev[1 + g], b));
  }
  for (size_t g = 0; g < gs.size(); ++g) HIPTRY(hipStreamWaitEvent(q, c->branch_ev[1 + g], 0));
  return GP_OK;
}

int rb_split_member(gp_ctx* c, hipStream_t s, const RbMember& m, int r0, int R, const double* b, const double* x,
                    bool zero_guess, bool profiled) {
  const RbProb& P = m.desc;
  const int K = m.op->K, NB = P.rb.NB, NR = P.rb.NR;
  const bool f32 = m.f32;
  const size_t tsz = f32 ? sizeof(float) : sizeof(double);
  RbSplitFirst first{nullptr, nullptr, P.pr.part, (size_t)P.pr.R * P.pr.pstride, P.pr.pstride, r0, f32};
  if (zero_guess) {
    first.r = (char*)P.r + (size_t)r0 * K * NB * tsz;
    first.p = (char*)P.p + (size_t)r0 * K * NB * tsz;
  }
  if (R > 0)
    PROFILED_IF(profiled && c->prof_on, c, GP_KERNEL_RB_EDGE,
                launch_rb_split(s, P.rb, R, b, x, zero_guess ? 1 : 0, m.t64 + (size_t)r0 * K * NR,
                                (double*)P.c64 + (size_t)r0 * K * NB, P.xB + (size_t)r0 * K * NB,
                                (double*)P.bb + (size_t)r0 * P.rb.ntN, first));
  return GP_OK;
}

int rb_recover_member(gp_ctx* c, hipStream_t s, const RbMember& m, int r0, int R, double* x, bool profiled) {
  const RbProb& P = m.desc;
  const int K = m.op->K, NB = P.rb.NB, NR = P.rb.NR;
  if (R > 0)
    PROFILED_IF(profiled && c->prof_on, c, GP_KERNEL_RB_EDGE,
                launch_rb_recover(s, P.rb, R, P.pr.st + r0, m.t64 + (size_t)r0 * K * NR,
                                  P.u64 + (size_t)r0 * K * NR, P.xB + (size_t)r0 * K * NB, x));
  return GP_OK;
}

// Algorithmic HBM bytes of a member's launches, from its work counters: every
// vector entry a launch needs read or written once (a gathered neighbour
// vector counted once), the blocks once per launch with work.
void rb_account(gp_ctx* c, const RbMember& m, size_t tsz, bool zero_guess, const std::vector<long long>& pf) {
  const gp_op* op = m.op;
  const RbData& d = *op->rb;
  const int R = m.R;
  const double K = op->K, NB = d.NB, NR = d.NR, N = op->N, ts = (double)tsz, NBt = K * (K + 1) / 2;
  const double mv = (double)pf[PF_MATVEC_RHS], ref = (double)pf[PF_REFINE_RHS];
  // red stage: the black vector read, u written; the red inverses
  prof_add(c, GP_KERNEL_RB_RED, mv * NR, mv * K * (NB + NR) * ts + pf[PF_MATVEC_ACT] * NBt * NR * ts);
  // black stage: p, u, r read, q written; Q_mm and the Schur inverses
  prof_add(c, GP_KERNEL_RB_MATVEC, mv * NB, mv * K * (3 * NB + NR) * ts + pf[PF_MATVEC_ACT] * 2 * NBt * NB * ts);
  // the FP64 red stage on x_B for refinements from a non-zero x
  const double ref_x = ref - (double)pf[PF_REFINE_X0];
  prof_add(c, GP_KERNEL_RB_RED64, ref_x * NR, ref_x * K * (NB + NR) * 8 + pf[PF_REFINE_ACT] * NBt * NR * 8);
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

// ------------------------------------------------------------ grouped solve
int rb_solve_group(gp_ctx* c, const std::vector<RbOpItems>& ops_in, const gp_opts& o) {
  const auto t0 = std::chrono::steady_clock::now();
  // members ordered by K (one launch group per K)
  std::vector<const RbOpItems*> ops;
  for (const RbOpItems& oi : ops_in) {
    long Rl = 0;
    for (const RbItem& it : oi.items) Rl += it.R;
    if (Rl > 65535)
      return fail(GP_ERR_INVALID_ARG, "at most 65535 right-hand sides per operator with the red-black preconditioner");
    if (Rl > 0) ops.push_back(&oi);
  }
  if (ops.empty()) return GP_OK;
  std::stable_sort(ops.begin(), ops.end(), [](const RbOpItems* a, const RbOpItems* b) { return a->op->K < b->op->K; });
  for (const RbOpItems* oi : ops)
    if (!oi->op->rb || oi->op->pc_built != GP_PRECOND_RB_IC0) return fail(GP_ERR_INVALID_ARG, "preconditioner not built");
  const int n = (int)ops.size();
  const bool f32 = o.precision == GP_PREC_FP32_REFINE64;
  const size_t tsz = f32 ? sizeof(float) : sizeof(double);
  std::vector<int> Rm(n);
  long totalR = 0;
  for (int j = 0; j < n; ++j) {
    int R = 0;
    for (const RbItem& it : ops[j]->items) R += it.R;
    Rm[j] = R;
    totalR += R;
  }
  // a lone operator takes its tuned right-hand sides per work item, if any
  const gp_opts ot = n == 1 ? tuned_opts(c, ops[0]->op, Rm[0], o) : o;
  // workspace: every member's states contiguous (one copy brings them all to
  // the host), then each member's vectors
  std::vector<size_t> at(n);
  size_t off = align_up((size_t)totalR * sizeof(RhsState), 256);
  for (int j = 0; j < n; ++j) {
    at[j] = off;
    off += rb_member_bytes(ops[j]->op, Rm[j], f32);
  }
  if (int st = ensure_ws(c, off)) return st;
  if (int st = ensure_rb_probs(c, n)) return st;
  char* ws = (char*)c->ws;
  hipStream_t s = c->stream;
  RhsState* sts = (RhsState*)ws;
  const SolveCfg cfg{o.tol, f32 ? o.inner_tol : 0.0, o.max_iter, o.max_outer, o.zero_guess ? 1 : 0, 0};
  std::vector<RbMember> mem(n);
  {
    long r0 = 0;
    for (int j = 0; j < n; ++j) {
      rb_member(ops[j]->op, Rm[j], f32, ws + at[j], sts + r0, cfg, c->prof_on, &mem[j]);
      mem[j].f32 = f32;
      c->h_rbp[j] = mem[j].desc;
      r0 += Rm[j];
    }
  }
  std::vector<RbGroup> groups = rb_groups(c->h_rbp, n, ot.rhs_tile, false);
  for (int j = 0; j < n; ++j) mem[j].desc = c->h_rbp[j];
  HIPTRY(hipMemcpyAsync(c->d_rbp, c->h_rbp, n * sizeof(RbProb), hipMemcpyHostToDevice, s));
  HIPTRY(hipMemsetAsync(sts, 0, (size_t)totalR * sizeof(RhsState), s));
  for (int j = 0; j < n; ++j)
    if (mem[j].prof) HIPTRY(hipMemsetAsync(mem[j].prof, 0, NPROF * sizeof(long long), s));
  // the items (member, first right-hand side, item): their split and recovery
  // launches write disjoint memory and run on branch streams side by side
  struct ItemAt {
    int j, r0;
    const RbItem* it;
  };
  std::vector<ItemAt> items;
  for (int j = 0; j < n; ++j) {
    int r0 = 0;
    for (const RbItem& it : ops[j]->items) {
      items.push_back({j, r0, &it});
      r0 += it.R;
    }
  }
  // per item: c = b_B - E' D_R^{-1} b_R, x_B, ||b||^2 partials, t = D_R^{-1} b_R;
  // from a zero start value also the first refinement (r = c, p = S_m^{-1} r)
  if (int st = fork_items(c, s, (int)items.size(), [&](hipStream_t q, int i) {
        const ItemAt& a = items[i];
        return rb_split_member(c, q, mem[a.j], a.r0, a.it->R, a.it->b, a.it->x, o.zero_guess != 0, true);
      }))
    return st;

  const int chunk = o.chunk > 0 ? o.chunk : 8;
  const bool graphs = c->use_graphs && !c->prof_on;
  std::string key = "rb|" + std::to_string((uintptr_t)c->d_rbp) + "|" + std::to_string((uintptr_t)ws) + "|" +
                    (f32 ? "f" : "d");
  for (const RbGroup& g : groups)
    key += "|" + std::to_string(g.K) + "," + std::to_string(g.count) + "," + std::to_string(g.WB) + "," +
           std::to_string(g.WR) + "," + std::to_string(g.WO) + "," + std::to_string(g.F) + "," + std::to_string(g.uw);
  auto run_round = [&](int len, uint64_t mask, bool tail, bool first) -> int {
    if (!graphs) return rb_enqueue_round(c, s, f32, groups, c->d_rbp, len, mask, tail, first, true, false);
    return graph_replay(c,
                        key + "|" + std::to_string(len) + "/" + std::to_string(mask) + (tail ? "t" : "") +
                            (first ? "f" : ""),
                        [&](hipStream_t q) {
                          return rb_enqueue_round(c, q, f32, groups, c->d_rbp, len, mask, tail, first, false, true);
                        });
  };

  // rounds planned as for the main solver: the outer step first, then
  // iterations with the outer step where inner solves are expected to end
  std::vector<RhsState> hs(totalR);
  if (int st = ensure_rb_states(c, (size_t)totalR)) return st;
  int n_outer = (int)totalR, n_inner = 0;
  int round_len = chunk;
  uint64_t round_mask = f32 && o.chunk > 0 ? ~0ull : 1ull;
  bool tail = false;
  const int hp = f32 ? 1 : 0;
  if (o.chunk <= 0) {
    // every member's previous solve at these settings: their outer steps where
    // they were taken, and the last of them (the final refinement) after the
    // round's iterations
    bool have = true;
    uint64_t m = 0;
    int len = 0;
    for (const RbOpItems* oi : ops) {
      const RbData& d = *oi->op->rb;
      if (!d.hist_mask[hp] || d.hist_tol[hp][0] != o.tol || d.hist_tol[hp][1] != o.inner_tol) have = false;
      m |= d.hist_mask[hp];
      len = std::max(len, d.hist_len[hp]);
    }
    if (have) {
      round_len = len;
      round_mask = m;
      tail = true;
    }
  }
  const long max_rounds = (long)o.max_iter + 4L * o.max_outer + 8;
  long rounds = 0;
  // x in the caller's layout (repeated if a later round changes x_B)
  auto recover = [&]() -> int {
    return fork_items(c, s, (int)items.size(), [&](hipStream_t q, int i) {
      const ItemAt& a = items[i];
      return rb_recover_member(c, q, mem[a.j], a.r0, a.it->R, a.it->x, true);
    });
  };
  bool recovered = false;
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
    HIPTRY(hipMemcpyAsync(c->h_rbst, sts, (size_t)totalR * sizeof(RhsState), hipMemcpyDeviceToHost, s));
    std::vector<int> checking;
    for (int j = 0; j < n; ++j) {
      RbData& d = *ops[j]->op->rb;
      if (d.check_bad) {
        HIPTRY(hipMemcpyAsync(d.h_bad, ops[j]->op->d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
        checking.push_back(j);
      }
    }
    HIPTRY(hipStreamSynchronize(s));
    std::memcpy(hs.data(), c->h_rbst, (size_t)totalR * sizeof(RhsState));
    for (int j : checking) {
      RbData& d = *ops[j]->op->rb;
      d.check_bad = false;
      if (*d.h_bad != INT_MAX) {
        ops[j]->op->pc_built = -1;
        return fail(GP_ERR_NOT_SPD,
                    "preconditioner block of voxel " + std::to_string(*d.h_bad) + " is not positive definite");
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
  if (c->prof_on) {
    for (int j = 0; j < n; ++j) {
      std::vector<long long> pf(NPROF);
      HIPTRY(hipMemcpy(pf.data(), mem[j].prof, NPROF * sizeof(long long), hipMemcpyDeviceToHost));
      rb_account(c, mem[j], tsz, o.zero_guess != 0, pf);
    }
    if (int e = prof_resolve(c)) return e;
  }
  {
    long r0 = 0;
    for (int j = 0; j < n; ++j) {
      uint64_t m = 0;
      for (int r = 0; r < Rm[j]; ++r) m |= hs[r0 + r].slots;
      r0 += Rm[j];
      int len = 0;
      while (len < 63 && (m >> (len + 1)) != 0) ++len;
      // a shape that reaches the last bit (outer steps after 63 or more
      // iterations) is not replayed
      RbData& d = *ops[j]->op->rb;
      d.hist_mask[hp] = len < 63 ? m : 0;
      d.hist_len[hp] = len;
      d.hist_tol[hp][0] = o.tol;
      d.hist_tol[hp][1] = o.inner_tol;
    }
  }
  const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  int ret = GP_OK;
  long r0 = 0;
  for (int j = 0; j < n; ++j) {
    for (const RbItem& it : ops[j]->items) {
      for (int r = 0; r < it.R; ++r) {
        const RhsState& h = hs[r0 + r];
        const int status = h.phase == PH_DONE ? h.status : GP_ERR_NOT_CONVERGED;
        if (it.stats) it.stats[r] = gp_stats{status, h.total_it, h.outer, 0, h.relres, us};
        if (status != GP_OK && ret == GP_OK) ret = status;
      }
      r0 += it.R;
    }
  }
  if (ret == GP_ERR_NOT_CONVERGED) return fail(ret, "some right-hand sides did not reach the tolerance");
  if (ret == GP_ERR_BREAKDOWN) return fail(ret, "PCG breakdown (non-finite value or loss of definiteness)");
  return ret;
}

}  // namespace rt
}  // namespace gp
