// Serving loop: resident operators, admission by HBM budget, continuous
// batching of solve / sample / trace requests into the grouped PCG launches,
// per-request deadlines and cancellation, per-request latency.
//
// The worker thread repeats rounds.  A round retires waiting requests that
// were cancelled or passed their deadline, admits waiting requests (FIFO,
// while the byte budget and the right-hand-side slot table allow), prepares
// their right-hand sides on the device, retires running requests that were
// cancelled or passed their deadline, rebuilds the grouped-launch descriptors
// when the active set changed, runs one solver round (about `chunk`
// iterations, with the refinement step where it is expected to be needed) for
// every active right-hand side, copies
// the state table to the host and retires every request whose right-hand
// sides are all done.  Requests therefore join and leave the running batch at
// round boundaries, and the kernels' batch-invariant reductions make a
// request's result independent of its company.  A failing request (its own
// breakdown or iteration cap, deadline, cancellation, or an allocation
// failure at admission) retires alone with its status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <map>
#include <thread>
#include <vector>

#include "gmrf.h"
#include "launch.hpp"
#include "runtime.hpp"

using namespace gp;
using namespace gp::rt;

static_assert(KMAX == GP_KMAX, "gp_result holds one trace entry per regressor");

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  gp_request r{};
  gp_op* op = nullptr;
  const double* bw = nullptr;
  int R = 1;
  int slot0 = -1;
  char* mem = nullptr;      // one allocation holding every buffer below
  size_t bytes = 0;
  double *b = nullptr, *x = nullptr, *part = nullptr, *tr = nullptr;
  void* vec[NVEC] = {};     // inner vectors (Jacobi / block Jacobi)
  RbMember rbm;             // red-black member (GP_PRECOND_RB_IC0)
  int8_t* probes = nullptr;
  Clock::time_point t_submit, t_admit, deadline;
  bool has_deadline = false;
  std::atomic<bool> cancel{false};
  int64_t admit_round = -1;
};

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

}  // namespace

struct gp_server {
  gp_ctx* ctx = nullptr;
  std::vector<gp_op*> ops;
  std::vector<const double*> bw;
  gp_server_cfg cfg{};
  bool f32 = true, rb = false;
  size_t tsz = 4;
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_step;
  std::deque<Req*> pending;
  std::vector<Req*> active;
  std::deque<gp_result> finished;
  bool stop = false;
  int fatal = GP_OK;
  std::string fatal_msg;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, failed = 0, rhs_solved = 0, peak_active = 0;
  int64_t rounds = 0;       // solver rounds run
  int64_t credits = 0;      // manual mode: rounds granted and not yet run
  size_t bytes_in_use = 0;
  // Request workspaces come from slabs of device memory taken up to the byte
  // budget and kept until the server is destroyed, carved best-fit and
  // coalesced on release (worker thread only): once the slabs cover the
  // working set, admission and retirement make no allocator call.
  std::vector<std::pair<char*, size_t>> slabs;
  size_t slab_bytes = 0;
  std::map<char*, size_t> free_at;         // free ranges by address
  std::multimap<size_t, char*> free_len;   // the same ranges by length
  std::vector<double> latencies;
  Clock::time_point t_first{}, t_last{};
  bool any_submitted = false;
  // device state table, one RhsState per right-hand-side slot, and its pinned
  // host copy (the slots up to the highest in use are copied each round)
  RhsState* d_states = nullptr;
  RhsState* h_states = nullptr;
  double* h_trace = nullptr;        // pinned: the trace totals of the requests retiring in a round
  std::vector<char> slot_used;
  std::vector<RhsState> plan_buf;   // the active right-hand sides' states, for the round plan
  // grouped-launch descriptors (Jacobi / block Jacobi: Prob; red-black: RbProb)
  Prob* d_probs = nullptr;
  Prob* h_probs = nullptr;
  RbProb* d_rbp = nullptr;
  RbProb* h_rbp = nullptr;
  int probs_cap = 0;
  bool layout_dirty = true;
  std::vector<LaunchGroup> groups;
  std::vector<RbGroup> rgroups;
  std::vector<Req*> order;   // active requests in descriptor order
};

namespace {

int find_slots(gp_server* s, int R) {
  const int cap = (int)s->slot_used.size();
  int run = 0;
  for (int i = 0; i < cap; ++i) {
    run = s->slot_used[i] ? 0 : run + 1;
    if (run == R) return i - R + 1;
  }
  return -1;
}

size_t trace_scratch(const gp_op* op, int R) {
  return ((size_t)2 * R * op->K * op->ntiles + 2 * (size_t)R * op->K + 1 + 2 * KMAX) * sizeof(double);
}

size_t request_bytes(const gp_server* s, const gp_op* op, int R, int kind) {
  const size_t nv = (size_t)R * op->K * op->N;
  size_t b = 0;
  b += align_up(2 * nv * sizeof(double), 256);                                     // b, x
  if (s->rb) {
    b += rb_member_bytes(op, R, s->f32);                                           // red-black member
  } else {
    const Plan pl = plan_problem(op, R, s->cfg.opts, s->ctx->cus);
    b += NVEC * align_up(nv * s->tsz, 256);                                        // inner vectors
    b += align_up((size_t)NPART * R * pl.pstride * sizeof(double), 256);            // partials
  }
  if (kind == GP_REQ_SAMPLE) b += align_up((size_t)(op->dirs + 1) * op->K * op->N * sizeof(double), 256);
  if (kind == GP_REQ_TRACE) {
    b += align_up(nv, 256);                                                         // probes
    b += align_up(trace_scratch(op, R), 256);
  }
  return b;
}

constexpr size_t SLAB_BYTES = size_t(1) << 30;

bool slab_start(const gp_server* s, const char* p) {
  for (const auto& sl : s->slabs)
    if (sl.first == p) return true;
  return false;
}

void free_erase(gp_server* s, std::map<char*, size_t>::iterator it) {
  auto r = s->free_len.equal_range(it->second);
  for (auto k = r.first; k != r.second; ++k)
    if (k->second == it->first) {
      s->free_len.erase(k);
      break;
    }
  s->free_at.erase(it);
}

void free_insert(gp_server* s, char* p, size_t n) {
  s->free_at[p] = n;
  s->free_len.emplace(n, p);
}

// Returns [p, p + n) to the free ranges, merged with free neighbours in the
// same slab.
void arena_release(gp_server* s, char* p, size_t n) {
  auto next = s->free_at.find(p + n);
  if (next != s->free_at.end() && !slab_start(s, p + n)) {
    n += next->second;
    free_erase(s, next);
  }
  auto prev = s->free_at.lower_bound(p);
  if (prev != s->free_at.begin() && !slab_start(s, p)) {
    --prev;
    if (prev->first + prev->second == p) {
      p = prev->first;
      n += prev->second;
      free_erase(s, prev);
    }
  }
  free_insert(s, p, n);
}

// Best-fit range of n bytes; a new slab (1 GiB, or n if larger, within the
// budget) when no free range fits.  nullptr: nothing fits now.
char* arena_take(gp_server* s, size_t n) {
  auto it = s->free_len.lower_bound(n);
  if (it == s->free_len.end()) {
    if (s->slab_bytes + n > s->cfg.hbm_budget) return nullptr;
    size_t want = std::max(n, std::min(SLAB_BYTES, s->cfg.hbm_budget - s->slab_bytes));
    char* m = nullptr;
    if (hipMalloc((void**)&m, want) != hipSuccess) {
      (void)hipGetLastError();
      want = n;
      if (hipMalloc((void**)&m, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    s->slabs.emplace_back(m, want);
    s->slab_bytes += want;
    free_insert(s, m, want);
    it = s->free_len.lower_bound(n);
  }
  char* p = it->second;
  const size_t have = it->first;
  free_erase(s, s->free_at.find(p));
  if (have > n) free_insert(s, p + n, have - n);
  return p;
}

// With no workspace in use: gives every slab back to the device.
int arena_reset(gp_server* s) {
  HIPTRY(hipStreamSynchronize(s->stream));
  for (const auto& sl : s->slabs) HIPTRY(hipFree(sl.first));
  s->slabs.clear();
  s->slab_bytes = 0;
  s->free_at.clear();
  s->free_len.clear();
  return GP_OK;
}

// Lays out a request's buffers in its workspace and prepares its right-hand
// sides.
int admit(gp_server* s, Req* q) {
  hipStream_t st = s->stream;
  gp_op* op = q->op;
  const size_t nv = (size_t)q->R * op->K * op->N;
  char* p = q->mem;
  auto take = [&](size_t n) {
    char* r = p;
    p += align_up(n, 256);
    return r;
  };
  q->b = (double*)take(2 * nv * sizeof(double));
  q->x = q->b + nv;
  const gp_opts& o = s->cfg.opts;
  if (s->rb) {
    char* m = p;
    p += rb_member_bytes(op, q->R, s->f32);
    const SolveCfg cfg{o.tol, s->f32 ? o.inner_tol : 0.0, o.max_iter, o.max_outer, 1, 0};   // x starts at zero
    rb_member(op, q->R, s->f32, m, s->d_states + q->slot0, cfg, false, &q->rbm);
    q->rbm.f32 = s->f32;
  } else {
    for (int v = 0; v < NVEC; ++v) q->vec[v] = take(nv * s->tsz);
    q->part = (double*)take((size_t)NPART * q->R * plan_problem(op, q->R, o, s->ctx->cus).pstride * sizeof(double));
  }
  double* z = nullptr;
  if (q->r.kind == GP_REQ_SAMPLE) z = (double*)take((size_t)(op->dirs + 1) * op->K * op->N * sizeof(double));
  if (q->r.kind == GP_REQ_TRACE) {
    q->probes = (int8_t*)take(nv);
    q->tr = (double*)take(trace_scratch(op, q->R));
  }
  const OpDev d = op_dev(op);
  const size_t kn = (size_t)op->K * op->N;
  switch (q->r.kind) {
    case GP_REQ_SOLVE:
      HIPTRY(launch_rng_normal(st, q->r.seed, 4, kn, q->b));
      HIPTRY(launch_add_broadcast(st, 1, (long)kn, q->bw, q->b));
      break;
    case GP_REQ_SAMPLE: {
      const size_t n1 = (size_t)op->dirs * kn;
      HIPTRY(launch_rng_normal(st, q->r.seed, 1, n1, z));
      HIPTRY(launch_rng_normal(st, q->r.seed, 2, kn, z + n1));
      HIPTRY(launch_perturb(st, d, 1, q->bw, z, z + n1, q->b));
      break;
    }
    default:
      HIPTRY(launch_rng_rademacher(st, q->r.seed, 3, nv, q->probes));
      HIPTRY(launch_probe_rhs(st, (long)nv, q->probes, q->b));
      break;
  }
  HIPTRY(hipMemsetAsync(s->d_states + q->slot0, 0, (size_t)q->R * sizeof(RhsState), st));
  // red-black: c = b_B - E' D_R^{-1} b_R, t, and the first refinement from zero
  if (s->rb)
    if (int e = rb_split_member(s->ctx, st, q->rbm, 0, q->R, q->b, nullptr, true, false)) return e;
  return GP_OK;
}

int ensure_descriptors(gp_server* s, int n) {
  if (n <= s->probs_cap) return GP_OK;
  HIPTRY(hipStreamSynchronize(s->stream));
  if (s->d_probs) (void)hipFree(s->d_probs);
  if (s->h_probs) (void)hipHostFree(s->h_probs);
  if (s->d_rbp) (void)hipFree(s->d_rbp);
  if (s->h_rbp) (void)hipHostFree(s->h_rbp);
  s->d_probs = nullptr;
  s->h_probs = nullptr;
  s->d_rbp = nullptr;
  s->h_rbp = nullptr;
  s->probs_cap = std::max(n, 2 * s->probs_cap);
  if (s->rb) {
    HIPTRY(hipMalloc((void**)&s->d_rbp, (size_t)s->probs_cap * sizeof(RbProb)));
    HIPTRY(hipHostMalloc((void**)&s->h_rbp, (size_t)s->probs_cap * sizeof(RbProb), hipHostMallocDefault));
  } else {
    HIPTRY(hipMalloc((void**)&s->d_probs, (size_t)s->probs_cap * sizeof(Prob)));
    HIPTRY(hipHostMalloc((void**)&s->h_probs, (size_t)s->probs_cap * sizeof(Prob), hipHostMallocDefault));
  }
  return GP_OK;
}

int rebuild_layout(gp_server* s) {
  s->order = s->active;
  std::stable_sort(s->order.begin(), s->order.end(), [](Req* a, Req* b) { return a->op->K < b->op->K; });
  if (int st = ensure_descriptors(s, (int)s->order.size())) return st;
  const gp_opts& o = s->cfg.opts;
  const int n = (int)s->order.size();
  if (s->rb) {
    for (int j = 0; j < n; ++j) s->h_rbp[j] = s->order[j]->rbm.desc;
    s->rgroups = rb_groups(s->h_rbp, n, o.rhs_tile, true);
    HIPTRY(hipMemcpyAsync(s->d_rbp, s->h_rbp, (size_t)n * sizeof(RbProb), hipMemcpyHostToDevice, s->stream));
    s->layout_dirty = false;
    return GP_OK;
  }
  s->groups.clear();
  const SolveCfg cfg{o.tol, s->f32 ? o.inner_tol : 0.0, o.max_iter, o.max_outer, 1, 0};   // x starts at zero
  const int fpb = finalize_rhs_per_block();
  for (int j = 0; j < n; ++j) {
    Req* q = s->order[j];
    Prob& p = s->h_probs[j];
    std::memset(&p, 0, sizeof(Prob));
    p.op = op_dev(q->op);
    p.b = q->b;
    p.x = q->x;
    p.d = q->vec[0];
    p.r = q->vec[1];
    p.p = q->vec[2];
    p.q = q->vec[3];
    p.st = s->d_states + q->slot0;
    p.part = q->part;
    p.prof = nullptr;
    p.R = q->R;
    const Plan pl = plan_problem(q->op, q->R, o, s->ctx->cus);
    apply_plan(p, pl);
    p.cfg = cfg;
    if (s->groups.empty() || s->groups.back().K != q->op->K)
      s->groups.push_back(LaunchGroup{q->op->K, j, 0, 0, 0, 0, 0, 0, pl.mv_mode, o.wg_per_cu, 0, 0});
    auto& g = s->groups.back();
    p.work_begin = g.W;
    g.W += p.work_count;
    p.work_begin_o = g.Wo;
    g.Wo += p.work_count_o;
    p.mv_begin = g.Wmv;
    g.Wmv += p.mv_count;
    p.fin_begin = g.F;
    g.F += (q->R + fpb - 1) / fpb;
    g.count += 1;
  }
  size_groups(s->groups, s->ctx->cus);
  HIPTRY(hipMemcpyAsync(s->d_probs, s->h_probs, (size_t)n * sizeof(Prob), hipMemcpyHostToDevice, s->stream));
  s->layout_dirty = false;
  return GP_OK;
}

int run_round(gp_server* s) {
  hipStream_t st = s->stream;
  const int pc = s->cfg.opts.precond;
  // The round's plan from the active right-hand sides' states: with FP32
  // inner solves the outer step is placed where inner solves are expected to
  // end (and first, for requests just admitted), as in the solver's own
  // rounds; with FP64 inner solves it opens the round.  The launch groups
  // (one per K) run on branch streams forked from the server's stream.
  int len = s->cfg.chunk;
  uint64_t mask = 1;
  int top = 0;
  if (s->f32) {
    s->plan_buf.clear();
    for (Req* q : s->active)
      for (int r = 0; r < q->R; ++r) s->plan_buf.push_back(s->h_states[q->slot0 + r]);
    gp_opts po = s->cfg.opts;
    po.chunk = 0;
    plan_round(s->plan_buf, po, true, s->cfg.chunk, &len, &mask);
  }
  for (Req* q : s->active) top = std::max(top, q->slot0 + q->R);
  if (s->rb) {
    if (int e = rb_enqueue_round(s->ctx, st, s->f32, s->rgroups, s->d_rbp, len, mask, false, false, false, true))
      return e;
  } else if (int e = enqueue_round_branched(s->ctx, st, s->f32, pc, s->groups, s->d_probs, len, mask)) {
    return e;
  }
  HIPTRY(hipMemcpyAsync(s->h_states, s->d_states, (size_t)top * sizeof(RhsState), hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  s->rounds += 1;
  return GP_OK;
}

void base_result(const gp_server* s, const Req* q, gp_result* res) {
  std::memset(res, 0, sizeof(*res));
  res->ticket = q->ticket;
  res->kind = q->r.kind;
  res->op_index = q->r.op_index;
  res->rhs = q->R;
  res->admit_round = q->admit_round;
  res->retire_round = s->rounds;
}

// Returns a request's workspace to the arena (its pending work and the next
// user's are ordered on the server stream) and frees its slots.
int release(gp_server* s, Req* q) {
  if (q->mem) arena_release(s, q->mem, q->bytes);
  q->mem = nullptr;
  if (q->slot0 >= 0)
    for (int r = 0; r < q->R; ++r) s->slot_used[q->slot0 + r] = 0;
  return GP_OK;
}

// Finishes request q without a result (cancelled, deadline passed, or its
// admission failed): status only, nothing is written to its output.
int retire_failed(gp_server* s, Req* q, int status, gp_result* res) {
  base_result(s, q, res);
  res->status = status;
  if (int e = release(s, q)) return e;
  const auto now = Clock::now();
  res->latency_us = us_between(q->t_submit, now);
  res->queue_us = q->admit_round >= 0 ? us_between(q->t_submit, q->t_admit) : 0.0;
  return GP_OK;
}

// Enqueues the retirement of request q (all its right-hand sides are done):
// recovery of the red-black solution, trace reduction (its 1 + 2K totals
// copied to the pinned slot `trace_host`), result copy, release of its memory
// and slots.  The result's trace entries and latency are filled by
// retire_finish once the stream has been waited for.
int retire_enqueue(gp_server* s, Req* q, gp_result* res, double* trace_host) {
  hipStream_t st = s->stream;
  gp_op* op = q->op;
  base_result(s, q, res);
  res->status = GP_OK;
  for (int r = 0; r < q->R; ++r) {
    const RhsState& h = s->h_states[q->slot0 + r];
    if (h.status != GP_OK && res->status == GP_OK) res->status = h.status;
    res->iters_max = std::max(res->iters_max, h.total_it);
    res->relres_max = std::max(res->relres_max, h.relres);
  }
  const size_t nv = (size_t)q->R * op->K * op->N;
  if (res->status == GP_OK) {
    if (s->rb) {
      // x from x_B and the red rows (zeros for b = 0 or a solve that ended
      // at its first refinement)
      if (int e = rb_recover_member(s->ctx, st, q->rbm, 0, q->R, q->x, false)) return e;
    } else {
      // x starts at zero and is first written by the first x += d: right-hand
      // sides that ended at their first refinement (b = 0 among them) get zeros
      const size_t nr = (size_t)op->K * op->N;
      for (int r = 0; r < q->R; ++r) {
        const RhsState& h = s->h_states[q->slot0 + r];
        if (h.zero_b || h.outer <= 1) HIPTRY(hipMemsetAsync(q->x + r * nr, 0, nr * sizeof(double), st));
      }
    }
    if (q->r.kind == GP_REQ_TRACE) {
      double* part = q->tr;
      double* pairbuf = part + (size_t)2 * q->R * op->K * op->ntiles;
      double* out = pairbuf + (size_t)2 * q->R * op->K;
      HIPTRY(launch_trace(st, op_dev(op), q->R, q->probes, q->x, part, pairbuf, out));
      HIPTRY(hipMemcpyAsync(trace_host, out, (1 + 2 * (size_t)op->K) * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    if (q->r.out) HIPTRY(hipMemcpyAsync(q->r.out, q->x, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  return release(s, q);
}

void retire_finish(const Req* q, gp_result* res, const double* trace_host) {
  if (res->status == GP_OK && q->r.kind == GP_REQ_TRACE) {
    const int K = q->op->K;
    res->trace_total = trace_host[0];
    for (int k = 0; k < K; ++k) {
      res->trace_kk[k] = trace_host[1 + k];
      res->trace_Gkk[k] = trace_host[1 + K + k];
    }
  }
  const auto now = Clock::now();
  res->latency_us = us_between(q->t_submit, now);
  res->queue_us = us_between(q->t_submit, q->t_admit);
}

bool expired(const Req* q, Clock::time_point now) { return q->has_deadline && now >= q->deadline; }

void worker_main(gp_server* s) {
  if (hipSetDevice(s->ctx->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->fatal = GP_ERR_DEVICE;
    s->fatal_msg = "server thread could not select the device";
    s->cv_done.notify_all();
    s->cv_step.notify_all();
    return;
  }
  for (;;) {
    std::vector<Req*> admitted;
    std::vector<std::pair<Req*, int>> dropped;   // requests that never ran, with their status
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->cfg.manual)
        s->cv_work.wait(lk, [&] { return s->stop || s->credits > 0; });
      else if (s->active.empty())
        s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
      if (s->stop && (s->cfg.manual || (s->pending.empty() && s->active.empty()))) return;
      const auto now = Clock::now();
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        Req* q = *it;
        if (q->cancel.load() || expired(q, now)) {
          dropped.emplace_back(q, q->cancel.load() ? GP_ERR_CANCELLED : GP_ERR_TIMEOUT);
          it = s->pending.erase(it);
        } else {
          ++it;
        }
      }
      while (!s->pending.empty()) {
        Req* q = s->pending.front();
        if (s->bytes_in_use + q->bytes > s->cfg.hbm_budget) break;
        const int slot = find_slots(s, q->R);
        if (slot < 0) break;
        q->mem = arena_take(s, q->bytes);
        if (!q->mem && s->active.empty() && admitted.empty()) {
          // nothing holds a workspace: fresh slabs, then out of memory
          if (int e = arena_reset(s)) {
            s->fatal = e;
            s->fatal_msg = gp_last_error();
            s->stop = true;
            s->cv_done.notify_all();
            s->cv_step.notify_all();
            return;
          }
          q->mem = arena_take(s, q->bytes);
          if (!q->mem) {
            (void)fail(GP_ERR_OOM, "request workspace could not be allocated");
            dropped.emplace_back(q, GP_ERR_OOM);
            s->pending.pop_front();
            continue;
          }
        }
        if (!q->mem) break;   // waits for running requests to release theirs
        for (int r = 0; r < q->R; ++r) s->slot_used[slot + r] = 1;
        q->slot0 = slot;
        s->bytes_in_use += q->bytes;
        s->pending.pop_front();
        admitted.push_back(q);
      }
    }
    int err = GP_OK;
    std::vector<gp_result> done;
    for (auto& qd : dropped) {
      gp_result res;
      if ((err = retire_failed(s, qd.first, qd.second, &res)) != GP_OK) break;
      done.push_back(res);
      delete qd.first;
    }
    std::vector<Req*> freed;   // requests whose bytes leave the budget
    for (size_t i = 0; i < admitted.size() && err == GP_OK; ++i) {
      Req* q = admitted[i];
      q->t_admit = Clock::now();
      q->admit_round = s->rounds;
      const int st = admit(s, q);
      if (st == GP_OK) {
        // the host copy of its states starts as the device's (zero) until the
        // round reads them back
        std::memset(s->h_states + q->slot0, 0, (size_t)q->R * sizeof(RhsState));
        s->active.push_back(q);
        s->layout_dirty = true;
      } else {
        err = st;
      }
    }
    // running requests cancelled or past their deadline leave at this boundary
    if (err == GP_OK) {
      const auto now = Clock::now();
      std::vector<Req*> keep;
      for (Req* q : s->active) {
        if (err == GP_OK && (q->cancel.load() || expired(q, now))) {
          gp_result res;
          if ((err = retire_failed(s, q, q->cancel.load() ? GP_ERR_CANCELLED : GP_ERR_TIMEOUT, &res)) != GP_OK) break;
          done.push_back(res);
          freed.push_back(q);
          s->layout_dirty = true;
        } else {
          keep.push_back(q);
        }
      }
      if (err == GP_OK) s->active.swap(keep);
    }
    int64_t live = 0;
    for (Req* q : s->active) live += q->R;
    s->peak_active = std::max(s->peak_active, live);
    if (err == GP_OK && !s->active.empty()) {
      if (s->layout_dirty) err = rebuild_layout(s);
      if (err == GP_OK) err = run_round(s);
    }
    if (err == GP_OK) {
      // every finished request's retirement is enqueued, then one wait
      std::vector<Req*> still, leaving;
      std::vector<gp_result> out;
      for (Req* q : s->active) {
        bool all = true;
        for (int r = 0; r < q->R && all; ++r) all = s->h_states[q->slot0 + r].phase == PH_DONE;
        if (!all) {
          still.push_back(q);
          continue;
        }
        out.emplace_back();
        if ((err = retire_enqueue(s, q, &out.back(), s->h_trace + leaving.size() * (1 + 2 * KMAX))) != GP_OK)
          break;
        leaving.push_back(q);
        s->layout_dirty = true;
      }
      if (err == GP_OK && !leaving.empty()) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) err = fail(GP_ERR_DEVICE, "server stream failed");
        for (size_t i = 0; i < leaving.size() && err == GP_OK; ++i) {
          retire_finish(leaving[i], &out[i], s->h_trace + i * (1 + 2 * KMAX));
          done.push_back(out[i]);
          freed.push_back(leaving[i]);
        }
      }
      if (err == GP_OK) s->active.swap(still);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    for (Req* q : freed) {
      s->bytes_in_use -= q->bytes;
      delete q;
    }
    if (s->cfg.manual && s->credits > 0) s->credits -= 1;
    s->cv_step.notify_all();
    if (err != GP_OK) {
      s->fatal = err;
      s->fatal_msg = gp_last_error();
      s->stop = true;
      s->cv_done.notify_all();
      return;
    }
    for (gp_result& r : done) {
      if (r.status == GP_OK) {
        s->latencies.push_back(r.latency_us);
        s->rhs_solved += r.rhs;
      } else {
        s->failed += 1;
      }
      s->completed += 1;
      s->finished.push_back(r);
      s->t_last = Clock::now();
    }
    if (!done.empty()) s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

void gp_server_cfg_default(gp_server_cfg* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->hbm_budget = (size_t)16 << 30;
  c->max_active_rhs = 1024;
  c->chunk = 4;
  c->probes = 16;
  gp_opts_default(&c->opts);
}

int gp_server_create(gp_ctx* ctx, int nops, gp_op* const* ops, const double* const* bw, const gp_server_cfg* cfg,
                     gp_server** out) {
  if (!out) return fail(GP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx || nops < 1 || !ops || !bw) return fail(GP_ERR_INVALID_ARG, "ctx, ops or bw missing");
  gp_server_cfg c;
  if (cfg) c = *cfg; else gp_server_cfg_default(&c);
  std::string why;
  if (!valid_opts(c.opts, &why)) return fail(GP_ERR_INVALID_ARG, why);
  if (c.max_active_rhs < 1 || c.chunk < 1 || c.probes < 1 || c.probes > c.max_active_rhs)
    return fail(GP_ERR_INVALID_ARG, "max_active_rhs >= 1, chunk >= 1 and 1 <= probes <= max_active_rhs required");
  if (c.opts.precond == GP_PRECOND_RB_IC0 && c.probes > 65535)
    return fail(GP_ERR_INVALID_ARG, "at most 65535 probes per trace request with the red-black preconditioner");
  if (c.manual != 0 && c.manual != 1) return fail(GP_ERR_INVALID_ARG, "manual must be 0 or 1");
  for (int i = 0; i < nops; ++i) {
    if (!ops[i] || ops[i]->ctx != ctx || !bw[i]) return fail(GP_ERR_INVALID_ARG, "operator or b_w missing");
    if (!ops[i]->have_blocks || !ops[i]->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
    if (ops[i]->K < 1 || ops[i]->K > KMAX) return fail(GP_ERR_INVALID_ARG, "operator K out of range");
  }
  int expect = 0;
  if (!ctx->busy.compare_exchange_strong(expect, 1)) return fail(GP_ERR_BUSY, "context busy");
  gp_server* s = new gp_server();
  s->ctx = ctx;
  s->cfg = c;
  s->f32 = c.opts.precision == GP_PREC_FP32_REFINE64;
  s->rb = c.opts.precond == GP_PRECOND_RB_IC0;
  s->tsz = s->f32 ? sizeof(float) : sizeof(double);
  s->ops.assign(ops, ops + nops);
  s->bw.assign(bw, bw + nops);
  s->slot_used.assign(c.max_active_rhs, 0);
  auto bail = [&](int st) {
    if (s->d_states) (void)hipFree(s->d_states);
    if (s->h_states) (void)hipHostFree(s->h_states);
    if (s->h_trace) (void)hipHostFree(s->h_trace);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    ctx->busy.store(0);
    return st;
  };
  if (int st = set_device(ctx)) return bail(st);
  for (gp_op* op : s->ops) {
    if (op->pc_built != c.opts.precond)
      if (int st = build_precond(op, c.opts.precond)) return bail(st);
    if (s->rb)
      if (int st = rb_check_built(op)) return bail(st);
  }
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(GP_ERR_DEVICE, "could not create the server stream"));
  if (hipMalloc((void**)&s->d_states, (size_t)c.max_active_rhs * sizeof(RhsState)) != hipSuccess)
    return bail(fail(GP_ERR_OOM, "could not allocate the state table"));
  if (hipHostMalloc((void**)&s->h_states, (size_t)c.max_active_rhs * sizeof(RhsState), hipHostMallocDefault) !=
      hipSuccess)
    return bail(fail(GP_ERR_OOM, "could not allocate the host state table"));
  std::memset(s->h_states, 0, (size_t)c.max_active_rhs * sizeof(RhsState));
  if (hipHostMalloc((void**)&s->h_trace, (size_t)c.max_active_rhs * (1 + 2 * KMAX) * sizeof(double),
                    hipHostMallocDefault) != hipSuccess)
    return bail(fail(GP_ERR_OOM, "could not allocate the host trace table"));
  (void)hipGetLastError();
  s->worker = std::thread(worker_main, s);
  *out = s;
  return GP_OK;
}

int gp_server_submit(gp_server* s, const gp_request* req, uint64_t* ticket) {
  if (!s || !req) return fail(GP_ERR_INVALID_ARG, "server or request is NULL");
  if (req->kind < GP_REQ_SOLVE || req->kind > GP_REQ_TRACE) return fail(GP_ERR_INVALID_ARG, "unknown request kind");
  if (req->op_index < 0 || req->op_index >= (int)s->ops.size()) return fail(GP_ERR_INVALID_ARG, "op_index out of range");
  if (!(req->timeout_ms >= 0.0)) return fail(GP_ERR_INVALID_ARG, "timeout_ms must be >= 0");
  Req* q = new Req();
  q->r = *req;
  q->op = s->ops[req->op_index];
  q->bw = s->bw[req->op_index];
  q->R = req->kind == GP_REQ_TRACE ? s->cfg.probes : 1;
  q->bytes = request_bytes(s, q->op, q->R, req->kind);
  if (q->bytes > s->cfg.hbm_budget) {
    delete q;
    return fail(GP_ERR_OOM, "request needs more memory than the server's budget");
  }
  q->t_submit = Clock::now();
  if (req->timeout_ms > 0.0) {
    q->has_deadline = true;
    q->deadline = q->t_submit + std::chrono::duration_cast<Clock::duration>(
                                    std::chrono::duration<double, std::milli>(req->timeout_ms));
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal != GP_OK) {
    delete q;
    return fail(s->fatal, "server stopped: " + s->fatal_msg);
  }
  if (s->stop) {
    delete q;
    return fail(GP_ERR_INVALID_ARG, "server is stopping");
  }
  q->ticket = s->next_ticket++;
  if (!s->any_submitted) {
    s->any_submitted = true;
    s->t_first = q->t_submit;
  }
  s->submitted += 1;
  s->pending.push_back(q);
  if (ticket) *ticket = q->ticket;
  s->cv_work.notify_one();
  return GP_OK;
}

int gp_server_cancel(gp_server* s, uint64_t ticket) {
  if (!s) return fail(GP_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  for (Req* q : s->pending)
    if (q->ticket == ticket) {
      q->cancel.store(true);
      s->cv_work.notify_one();
      return GP_OK;
    }
  // the active list is the worker's; a flag set under the lock is read at the
  // next round boundary
  for (Req* q : s->active)
    if (q->ticket == ticket) {
      q->cancel.store(true);
      return GP_OK;
    }
  return fail(GP_ERR_INVALID_ARG, "unknown or finished ticket");
}

int gp_server_step(gp_server* s, int rounds) {
  if (!s) return fail(GP_ERR_INVALID_ARG, "server is NULL");
  if (!s->cfg.manual) return fail(GP_ERR_INVALID_ARG, "gp_server_step needs a server created with manual = 1");
  if (rounds < 0) return fail(GP_ERR_INVALID_ARG, "rounds must be >= 0");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->fatal != GP_OK) return fail(s->fatal, "server stopped: " + s->fatal_msg);
  s->credits += rounds;
  s->cv_work.notify_one();
  s->cv_step.wait(lk, [&] { return s->credits == 0 || s->fatal != GP_OK || s->stop; });
  if (s->fatal != GP_OK) return fail(s->fatal, "server stopped: " + s->fatal_msg);
  return GP_OK;
}

int gp_server_poll(gp_server* s, gp_result* out, int max, int* n) {
  if (!s || !n || (max > 0 && !out)) return fail(GP_ERR_INVALID_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  int k = 0;
  while (k < max && !s->finished.empty()) {
    out[k++] = s->finished.front();
    s->finished.pop_front();
  }
  *n = k;
  if (s->fatal != GP_OK && k == 0) return fail(s->fatal, "server stopped: " + s->fatal_msg);
  return GP_OK;
}

int gp_server_drain(gp_server* s, int timeout_ms) {
  if (!s) return fail(GP_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return s->fatal != GP_OK || s->completed == s->submitted; };
  if (s->cfg.manual) {
    if (!ready()) return fail(GP_ERR_BUSY, "requests still waiting for rounds (manual mode)");
  } else if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return fail(GP_ERR_BUSY, "requests still running");
  }
  if (s->fatal != GP_OK) return fail(s->fatal, "server stopped: " + s->fatal_msg);
  return GP_OK;
}

int gp_server_get_stats(gp_server* s, gp_server_stats* out) {
  if (!s || !out) return fail(GP_ERR_INVALID_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->rounds = s->rounds;
  out->rhs_solved = s->rhs_solved;
  out->peak_active_rhs = s->peak_active;
  if (!s->latencies.empty()) {
    std::vector<double> v = s->latencies;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const size_t i = (size_t)std::min<double>(v.size() - 1, std::max(0.0, std::ceil(p * v.size()) - 1));
      return v[i];
    };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / v.size();
    out->max_us = v.back();
  }
  if (s->completed > 0) {
    out->elapsed_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
    if (out->elapsed_s > 0) {
      out->solves_per_s = s->rhs_solved / out->elapsed_s;
      out->requests_per_s = s->completed / out->elapsed_s;
    }
  }
  return GP_OK;
}

int gp_server_destroy(gp_server* s) {
  if (!s) return GP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_step.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);
  (void)hipStreamSynchronize(s->stream);
  for (Req* q : s->active) delete q;
  for (Req* q : s->pending) delete q;
  (void)hipStreamSynchronize(s->stream);
  for (const auto& sl : s->slabs) (void)hipFree(sl.first);
  if (s->d_probs) (void)hipFree(s->d_probs);
  if (s->h_probs) (void)hipHostFree(s->h_probs);
  if (s->d_rbp) (void)hipFree(s->d_rbp);
  if (s->h_rbp) (void)hipHostFree(s->h_rbp);
  if (s->d_states) (void)hipFree(s->d_states);
  if (s->h_states) (void)hipHostFree(s->h_states);
  if (s->h_trace) (void)hipHostFree(s->h_trace);
  (void)hipStreamDestroy(s->stream);
  s->ctx->busy.store(0);
  delete s;
  return GP_OK;
}

}  // extern "C"
