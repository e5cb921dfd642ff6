// Host runtime behind the C ABI of gmrf.h: contexts with an HBM budget,
// operator construction, preconditioner set-up and the PCG driver that
// advances grouped launches of the kernels in pcg.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gmrf.h"
#include "launch.hpp"
#include "runtime.hpp"

using namespace gp;
using namespace gp::rt;

// Device scratch of the allocation-free trace reduction
// (gp_trace_reduce_static): a fixed array in every GPU's memory, held until
// the process ends.  Host code never passes `scratch` itself (its name is a
// host-side stand-in); it uses the address hipGetSymbolAddress returns for the
// current device, looked up once per device by gp_ctx_create.
constexpr size_t TRACE_SCRATCH_DOUBLES = ((size_t)16 << 20) / sizeof(double);   // 16 MiB
static __device__ __align__(256) double scratch[TRACE_SCRATCH_DOUBLES];

namespace gp {
namespace rt {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};   // device address of `scratch`, per device
}  // namespace

// The device address of `scratch` on device `dev` (which must be current),
// looked up on the first call for that device.
int scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(GP_ERR_INVALID_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(GP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return GP_OK;
}

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int set_device(gp_ctx* c) {
  HIPTRY(hipSetDevice(c->device));
  return GP_OK;
}

int dev_alloc(gp_ctx* c, size_t bytes, void** p) {
  bytes = align_up(std::max<size_t>(bytes, 1), 256);
  if (c->budget && c->used + bytes > c->budget)
    return fail(GP_ERR_OOM, "HBM budget exceeded: need " + std::to_string(bytes) + " more bytes, " +
                                std::to_string(c->budget - c->used) + " left");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GP_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  c->used += bytes;
  return GP_OK;
}

void dev_free(gp_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  bytes = align_up(std::max<size_t>(bytes, 1), 256);
  c->used -= std::min(c->used, bytes);
}

template <typename T>
int op_alloc(gp_op* op, size_t count, T** p) {
  const size_t bytes = count * sizeof(T);
  int st = dev_alloc(op->ctx, bytes, (void**)p);
  if (st == GP_OK) op->bytes += align_up(std::max<size_t>(bytes, 1), 256);
  return st;
}

template <typename T>
void op_free(gp_op* op, T*& p, size_t count) {
  if (!p) return;
  dev_free(op->ctx, p, count * sizeof(T));
  p = nullptr;
}

int ensure_ws(gp_ctx* c, size_t bytes) {
  if (bytes <= c->ws_cap) return GP_OK;
  if (c->ws) {
    HIPTRY(hipStreamSynchronize(c->stream));
    dev_free(c, c->ws, c->ws_cap);
    c->ws = nullptr;
    c->ws_cap = 0;
  }
  const size_t want = align_up(bytes + bytes / 4, 1 << 20);
  int st = dev_alloc(c, want, &c->ws);
  if (st != GP_OK) {
    st = dev_alloc(c, bytes, &c->ws);
    if (st != GP_OK) return st;
    c->ws_cap = align_up(bytes, 256);
    return GP_OK;
  }
  c->ws_cap = want;
  return GP_OK;
}

int ensure_rhs(gp_ctx* c, size_t count) {
  if (count <= c->rhs_cap) return GP_OK;
  if (c->rhs) {
    HIPTRY(hipStreamSynchronize(c->stream));
    dev_free(c, c->rhs, c->rhs_cap * sizeof(double));
    c->rhs = nullptr;
    c->rhs_cap = 0;
  }
  int st = dev_alloc(c, count * sizeof(double), (void**)&c->rhs);
  if (st != GP_OK) return st;
  c->rhs_cap = count;
  return GP_OK;
}

template <typename T>
int ensure_buf(gp_ctx* c, T*& buf, size_t& cap, size_t count) {
  if (count <= cap) return GP_OK;
  if (buf) {
    HIPTRY(hipStreamSynchronize(c->stream));
    dev_free(c, buf, cap * sizeof(T));
    buf = nullptr;
    cap = 0;
  }
  int st = dev_alloc(c, count * sizeof(T), (void**)&buf);
  if (st != GP_OK) return st;
  cap = count;
  return GP_OK;
}

int ensure_probs(gp_ctx* c, size_t n) {
  if (n <= c->probs_cap) return GP_OK;
  if (c->d_probs) {
    HIPTRY(hipStreamSynchronize(c->stream));
    dev_free(c, c->d_probs, c->probs_cap * sizeof(Prob));
    (void)hipHostFree(c->h_probs);
    c->d_probs = nullptr;
    c->h_probs = nullptr;
  }
  const size_t cap = std::max<size_t>(n, 16);
  int st = dev_alloc(c, cap * sizeof(Prob), (void**)&c->d_probs);
  if (st != GP_OK) return st;
  HIPTRY(hipHostMalloc((void**)&c->h_probs, cap * sizeof(Prob), hipHostMallocDefault));
  c->probs_cap = cap;
  return GP_OK;
}

// ------------------------------------------------------------ profiling
}  // namespace rt

LaunchTiming& launch_timing() {
  static thread_local LaunchTiming t;
  return t;
}

namespace rt {

// The launches between prof_begin and prof_end take the slot's two events in
// their dispatch packets (GP_LAUNCH); a span without a kernel records them
// back to back.
int prof_begin(gp_ctx* c, size_t* slot) {
  if (c->ev_used + 2 > c->evpool.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      HIPTRY(hipEventCreate(&e));
      c->evpool.push_back(e);
    }
  }
  *slot = c->ev_used;
  c->ev_used += 2;
  LaunchTiming& lt = launch_timing();
  lt.start = c->evpool[*slot];
  lt.stop = c->evpool[*slot + 1];
  lt.first = true;
  return GP_OK;
}

int prof_end(gp_ctx* c, int kind, size_t slot) {
  LaunchTiming& lt = launch_timing();
  const bool none = lt.first;
  lt = LaunchTiming{};
  if (none) {
    HIPTRY(hipEventRecord(c->evpool[slot], c->stream));
    HIPTRY(hipEventRecord(c->evpool[slot + 1], c->stream));
  }
  c->pending.push_back({kind, slot});
  return GP_OK;
}

// Waits for the stream and folds the recorded launch durations into acc.
int prof_resolve(gp_ctx* c) {
  if (c->pending.empty()) return GP_OK;
  HIPTRY(hipStreamSynchronize(c->stream));
  for (auto& pe : c->pending) {
    float ms = 0.f;
    HIPTRY(hipEventElapsedTime(&ms, c->evpool[pe.second], c->evpool[pe.second + 1]));
    c->acc[pe.first].ms += ms;
    c->acc[pe.first].launches += 1;
  }
  c->pending.clear();
  c->ev_used = 0;
  return GP_OK;
}

void prof_add(gp_ctx* c, int kind, double units, double bytes) {
  if (!c->prof_on) return;
  c->acc[kind].units += (int64_t)units;
  c->acc[kind].bytes += bytes;
}


OpDev op_dev(const gp_op* op) {
  OpDev d;
  std::memset(&d, 0, sizeof(d));
  d.nbr = op->nbr;
  d.B64 = op->B64;
  d.B32 = op->B32;
  d.P64 = op->P64;
  d.P32 = op->P32;
  d.L64 = op->L64;
  d.gmap = op->gmap;
  d.nx = op->nx;
  d.ny = op->ny;
  d.nz = op->nz;
  d.N = op->N;
  d.K = op->K;
  d.ntiles = op->ntiles;
  d.dirs = op->dirs;
  for (int k = 0; k < op->K; ++k) {
    d.alpha64[k] = op->alpha[k];
    d.alpha32[k] = (float)op->alpha[k];
  }
  return d;
}

int read_bad(gp_op* op, int* bad) {
  if (!op->h_bad) HIPTRY(hipHostMalloc((void**)&op->h_bad, sizeof(int), hipHostMallocDefault));
  HIPTRY(hipMemcpyAsync(op->h_bad, op->d_bad, sizeof(int), hipMemcpyDeviceToHost, op->ctx->stream));
  HIPTRY(hipStreamSynchronize(op->ctx->stream));
  *bad = *op->h_bad;
  return GP_OK;
}

int reset_bad(gp_op* op) {
  HIPTRY(hipMemsetD32Async((hipDeviceptr_t)op->d_bad, INT_MAX, 1, op->ctx->stream));
  return GP_OK;
}

int build_precond(gp_op* op, int pc) {
  if (pc == GP_PRECOND_RB_IC0) return rb_build(op);
  if (!op->have_blocks || !op->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
  int st = reset_bad(op);
  if (st) return st;
  const OpDev d = op_dev(op);
  PROFILED(op->ctx, GP_KERNEL_PRECOND,
           launch_precond(op->ctx->stream, d, pc == GP_PRECOND_JACOBI ? PC_JACOBI : PC_BLOCK, op->P64, op->P32,
                          op->d_bad));
  {
    const double NB = op->K * (op->K + 1) / 2.0, NP = pc == GP_PRECOND_JACOBI ? op->K : NB;
    prof_add(op->ctx, GP_KERNEL_PRECOND, op->N, (double)op->N * (NB * 8 + NP * 12));
  }
  int bad = INT_MAX;
  st = read_bad(op, &bad);
  if (st) return st;
  if (bad != INT_MAX) {
    op->pc_built = -1;
    return fail(GP_ERR_NOT_SPD, "preconditioner block of voxel " + std::to_string(bad) + " is not positive definite");
  }
  op->pc_built = pc;
  return GP_OK;
}

bool valid_opts(const gp_opts& o, std::string* why) {
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return *why = "tol must be positive", false;
  if (o.precision == GP_PREC_FP32_REFINE64 && !(o.inner_tol > 0.0 && o.inner_tol < 1.0))
    return *why = "inner_tol must lie in (0, 1)", false;
  if (o.max_iter < 1) return *why = "max_iter must be >= 1", false;
  if (o.max_outer < 1) return *why = "max_outer must be >= 1", false;
  if (o.precond != GP_PRECOND_JACOBI && o.precond != GP_PRECOND_BLOCK_JACOBI && o.precond != GP_PRECOND_RB_IC0)
    return *why = "unknown preconditioner", false;
  if (o.precision != GP_PREC_FP64 && o.precision != GP_PREC_FP32_REFINE64) return *why = "unknown precision", false;
  if (o.matvec < GP_MATVEC_AUTO || o.matvec > GP_MATVEC_ZMARCH) return *why = "unknown matvec kernel", false;
  if (o.rhs_tile < 0 || o.chunk < 0 || o.wg_per_cu < 0) return *why = "rhs_tile, chunk and wg_per_cu must be >= 0", false;
  return true;
}

Plan plan_problem(const gp_op* op, int R, const gp_opts& o, int cus) {
  Plan pl{};
  int rc = o.rhs_tile > 0 ? o.rhs_tile : 4;
  rc = std::max(1, std::min(std::min(rc, RCMAX), R));
  pl.Rc = rc;
  pl.nchunks = (R + rc - 1) / rc;
  pl.work_count = op->ntiles * pl.nchunks;
  pl.Rco = std::min(rc, 4);
  pl.nchunks_o = (R + pl.Rco - 1) / pl.Rco;
  pl.work_count_o = op->ntiles * pl.nchunks_o;
  pl.mv_mode = o.matvec == GP_MATVEC_ZMARCH ? 1 : 0;
  if (pl.mv_mode) {
    const int nxt = (op->nx + 63) / 64;
    pl.nyt = (op->ny + 3) / 4;
    const int zr = zm_rhs_per_block(op->K);
    pl.mv_nchunks = (R + zr - 1) / zr;
    // enough footprint x segment x chunk items to fill the device, segments of >= 4 slices
    const long base = (long)nxt * pl.nyt * pl.mv_nchunks;
    const long target = 8L * cus;
    const int nseg_want = (int)std::max<long>(1, (target + base - 1) / base);
    pl.zs = std::max(4, (op->nz + nseg_want - 1) / nseg_want);
    if (const char* e = getenv("GMRF_ZSLICES")) pl.zs = std::max(1, atoi(e));
    pl.nseg = (op->nz + pl.zs - 1) / pl.zs;
    pl.mv_tiles = nxt * pl.nyt * pl.nseg;
    pl.mv_count = pl.mv_tiles * pl.mv_nchunks;
  }
  pl.pstride = std::max(op->ntiles, pl.mv_tiles);
  return pl;
}

void apply_plan(Prob& p, const Plan& pl) {
  p.Rc = pl.Rc;
  p.nchunks = pl.nchunks;
  p.work_count = pl.work_count;
  p.Rco = pl.Rco;
  p.nchunks_o = pl.nchunks_o;
  p.work_count_o = pl.work_count_o;
  p.pstride = pl.pstride;
  p.mv_mode = pl.mv_mode;
  p.zs = pl.zs;
  p.nseg = pl.nseg;
  p.nyt = pl.nyt;
  p.mv_tiles = pl.mv_tiles;
  p.mv_nchunks = pl.mv_nchunks;
  p.mv_count = pl.mv_count;
}

void size_groups(std::vector<LaunchGroup>& gs, int cus) {
  for (LaunchGroup& g : gs) {
    const int wpc = g.wpc > 0 ? g.wpc : 8;
    const int cap = std::max(8, cus * wpc / 8 * 8);
    g.nblk = std::min(cap, (g.W + 7) / 8 * 8);
    g.nblk_mv = std::min(cap, (g.Wmv + 7) / 8 * 8);
    g.nblk_o = std::min(cap, (g.Wo + 7) / 8 * 8);
  }
}

int enqueue_outer(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                  const Prob* d_probs, bool profiled) {
  const bool pf = profiled && c->prof_on;
  for (const LaunchGroup& g : gs) {
    const Prob* dp = d_probs + g.first;
    PROFILED_IF(pf, c, GP_KERNEL_ADDSOL,
                f32 ? launch_addsol_f32(q, g.K, dp, g.count, g.Wo, g.nblk_o)
                    : launch_addsol_f64(q, g.K, dp, g.count, g.Wo, g.nblk_o));
    PROFILED_IF(pf, c, GP_KERNEL_REFINE,
                f32 ? launch_refine_f32(q, pc, g.K, dp, g.count, g.Wo, g.nblk_o)
                    : launch_refine_f64(q, pc, g.K, dp, g.count, g.Wo, g.nblk_o));
    HIPTRY(launch_finalize(q, 0, dp, g.count, g.F));
  }
  return GP_OK;
}

int enqueue_inner(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                  const Prob* d_probs, int iters, bool profiled) {
  const bool pf = profiled && c->prof_on;
  for (int i = 0; i < iters; ++i) {
    for (const LaunchGroup& g : gs) {
      const Prob* dp = d_probs + g.first;
      if (g.mv_mode)
        PROFILED_IF(pf, c, GP_KERNEL_MATVEC,
                    f32 ? launch_matvec_zm_f32(q, pc, g.K, dp, g.count, g.Wmv, g.nblk_mv)
                        : launch_matvec_zm_f64(q, pc, g.K, dp, g.count, g.Wmv, g.nblk_mv));
      else
        PROFILED_IF(pf, c, GP_KERNEL_MATVEC,
                    f32 ? launch_matvec_f32(q, pc, g.K, dp, g.count, g.W, g.nblk)
                        : launch_matvec_f64(q, pc, g.K, dp, g.count, g.W, g.nblk));
      HIPTRY(launch_finalize(q, 1, dp, g.count, g.F));
      PROFILED_IF(pf, c, GP_KERNEL_UPDATE,
                  f32 ? launch_update_f32(q, pc, g.K, dp, g.count, g.W, g.nblk)
                      : launch_update_f64(q, pc, g.K, dp, g.count, g.W, g.nblk));
    }
  }
  return GP_OK;
}

int enqueue_round(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                  const Prob* d_probs, int chunk, uint64_t outer_mask, bool profiled) {
  if (chunk == 0)   // the outer step alone
    return (outer_mask & 1) ? enqueue_outer(c, q, f32, pc, gs, d_probs, profiled) : GP_OK;
  for (int i = 0; i < chunk; ++i) {
    if (i < 64 && ((outer_mask >> i) & 1))
      if (int e = enqueue_outer(c, q, f32, pc, gs, d_probs, profiled)) return e;
    if (int e = enqueue_inner(c, q, f32, pc, gs, d_probs, 1, profiled)) return e;
  }
  return GP_OK;
}

int ensure_branches(gp_ctx* c, size_t n) {
  while (c->branch.size() < n) {
    hipStream_t b = nullptr;
    HIPTRY(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    c->branch.push_back(b);
  }
  while (c->branch_ev.size() < n + 1) {
    hipEvent_t e = nullptr;
    HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->branch_ev.push_back(e);
  }
  return GP_OK;
}

int ensure_rb_probs(gp_ctx* c, size_t n) {
  if (n <= c->rbp_cap) return GP_OK;
  if (c->d_rbp) {
    HIPTRY(hipStreamSynchronize(c->stream));
    dev_free(c, c->d_rbp, c->rbp_cap * sizeof(RbProb));
    (void)hipHostFree(c->h_rbp);
    c->d_rbp = nullptr;
    c->h_rbp = nullptr;
    c->rbp_cap = 0;
  }
  const size_t cap = std::max<size_t>(n, 16);
  if (int st = dev_alloc(c, cap * sizeof(RbProb), (void**)&c->d_rbp)) return st;
  HIPTRY(hipHostMalloc((void**)&c->h_rbp, cap * sizeof(RbProb), hipHostMallocDefault));
  c->rbp_cap = cap;
  return GP_OK;
}

int ensure_rb_states(gp_ctx* c, size_t n) {
  if (n <= c->rbst_cap) return GP_OK;
  if (c->h_rbst) {
    HIPTRY(hipStreamSynchronize(c->stream));
    (void)hipHostFree(c->h_rbst);
    c->h_rbst = nullptr;
    c->rbst_cap = 0;
  }
  HIPTRY(hipHostMalloc((void**)&c->h_rbst, n * sizeof(RhsState), hipHostMallocDefault));
  c->rbst_cap = n;
  return GP_OK;
}

int enqueue_round_branched(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                           const Prob* d_probs, int chunk, uint64_t outer_mask) {
  if (gs.size() <= 1) return enqueue_round(c, q, f32, pc, gs, d_probs, chunk, outer_mask, false);
  if (int e = ensure_branches(c, gs.size())) return e;
  HIPTRY(hipEventRecord(c->branch_ev[0], q));
  for (size_t g = 0; g < gs.size(); ++g) {
    hipStream_t b = c->branch[g];
    HIPTRY(hipStreamWaitEvent(b, c->branch_ev[0], 0));
    const std::vector<LaunchGroup> one{gs[g]};
    if (int e = enqueue_round(c, b, f32, pc, one, d_probs, chunk, outer_mask, false)) return e;
    HIPTRY(hipEventRecord(c->branch_ev[1 + g], b));
  }
  for (size_t g = 0; g < gs.size(); ++g) HIPTRY(hipStreamWaitEvent(q, c->branch_ev[1 + g], 0));
  return GP_OK;
}

struct Item {
  gp_op* op;
  int R;
  const double* b;
  double* x;
};

// ------------------------------------------------------------- PCG driver
// With FP32 inner solves and an automatic chunk, the next round is planned
// from each right-hand side's completed inner solves (their mean length est):
// the slot in which its current inner solve should end, the refinement in the
// slot after it, one more inner solve when the residual after this one (about
// relres * inner_tol) is still above tol.  The round lasts until the last
// expected refinement; the outer step is placed in the first slot and around
// every expected refinement.  Before any history: `chunk` slots, the outer
// step first.  A fixed chunk places the outer step in every slot (FP32) or the
// first (FP64).
void plan_round(const std::vector<RhsState>& hs, const gp_opts& o, bool f32, int chunk, int* round_len,
                uint64_t* round_mask) {
  *round_len = chunk;
  *round_mask = 1;
  if (!f32 || o.chunk > 0) {
    *round_mask = f32 ? ~0ull : 1ull;
    return;
  }
  int need = 1;
  uint64_t mask = 1;
  auto mark = [&](int slot) {   // 1-based slot that should carry the outer step
    for (int t = slot - 1; t <= slot + 1; ++t)
      if (t >= 1 && t <= 64) mask |= 1ull << (t - 1);
  };
  for (const RhsState& h : hs) {
    if (h.phase == PH_DONE) continue;
    const bool inner = h.phase == PH_INNER;
    const int done_solves = inner ? h.outer - 1 : h.outer;
    if (done_solves <= 0) {   // no history yet
      need = std::max(need, chunk);
      continue;
    }
    const int est = std::max(1, (h.total_it - (inner ? h.inner_it : 0) + done_solves - 1) / done_solves);
    int refine_slot = inner ? std::max(1, est - h.inner_it) + 1 : 1;
    mark(refine_slot);
    if (h.relres * o.inner_tol > o.tol) {
      refine_slot += est;
      mark(refine_slot);
    }
    need = std::max(need, refine_slot);
  }
  *round_len = std::min(need, 2 * chunk);
  *round_mask = mask;
}

// Captured rounds are kept per launch layout, at most GRAPH_CACHE of them; a
// new layout in a full cache replaces the least recently replayed one (after
// the stream has drained, so that no replay of it is in flight).
constexpr size_t GRAPH_CACHE = 256;

int graph_replay(gp_ctx* c, const std::string& key, const std::function<int(hipStream_t)>& enqueue) {
  hipStream_t s = c->stream;
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (c->graphs.size() >= GRAPH_CACHE) {
      auto lru = c->graphs.begin();
      for (auto jt = c->graphs.begin(); jt != c->graphs.end(); ++jt)
        if (jt->second.used < lru->second.used) lru = jt;
      HIPTRY(hipStreamSynchronize(s));
      (void)hipGraphExecDestroy(lru->second.exec);
      c->graphs.erase(lru);
    }
    HIPTRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const int est = enqueue(c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (est != GP_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return est;
    }
    HIPTRY(e);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPTRY(ei);
    it = c->graphs.emplace(key, gp_ctx::GraphEntry{exec, 0}).first;
  }
  it->second.used = ++c->graph_tick;
  HIPTRY(hipGraphLaunch(it->second.exec, s));
  return GP_OK;
}

int run_group(gp_ctx* c, const std::vector<Item>& items, const gp_opts& o, gp_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  std::string why;
  if (!valid_opts(o, &why)) return fail(GP_ERR_INVALID_ARG, why);
  const bool f32 = o.precision == GP_PREC_FP32_REFINE64;
  const size_t tsz = f32 ? sizeof(float) : sizeof(double);
  size_t totalR = 0;
  for (const Item& it : items) {
    if (!it.op || it.op->ctx != c) return fail(GP_ERR_INVALID_ARG, "item operator missing or from another context");
    if (it.R < 0) return fail(GP_ERR_INVALID_ARG, "R must be >= 0");
    if (it.R > 0 && (!it.b || !it.x)) return fail(GP_ERR_INVALID_ARG, "null b or x");
    if (!it.op->have_blocks || !it.op->have_alpha)
      return fail(GP_ERR_INVALID_ARG, "operator needs gp_op_set_blocks and gp_op_set_alpha first");
    totalR += (size_t)it.R;
  }
  // preconditioners (the red-black set-ups of many operators side by side)
  if (o.precond == GP_PRECOND_RB_IC0) {
    std::vector<gp_op*> todo;
    for (const Item& it : items)
      if (it.R > 0 && it.op->pc_built != o.precond && std::find(todo.begin(), todo.end(), it.op) == todo.end())
        todo.push_back(it.op);
    if (int st = rb_build_ops(c, todo)) return st;
    for (gp_op* op : todo) op->pc_want = o.precond;
  } else {
    for (const Item& it : items) {
      if (it.R > 0 && it.op->pc_built != o.precond) {
        int st = build_precond(it.op, o.precond);
        if (st) return st;
        it.op->pc_want = o.precond;
      }
    }
  }
  // the red-black incomplete Cholesky preconditioner has a solver of its own:
  // every operator's items stacked in one member, members grouped by K
  if (o.precond == GP_PRECOND_RB_IC0) {
    std::vector<gp_stats> all(totalR);
    std::vector<RbOpItems> ops;
    size_t base = 0;
    for (const Item& it : items) {
      if (it.R > 0) {
        size_t gi = 0;
        while (gi < ops.size() && ops[gi].op != it.op) ++gi;
        if (gi == ops.size()) ops.push_back(RbOpItems{it.op, {}});
        ops[gi].items.push_back(RbItem{it.R, it.b, it.x, all.data() + base});
      }
      base += (size_t)it.R;
    }
    const int st = rb_solve_group(c, ops, o);
    if (st != GP_OK && st != GP_ERR_NOT_CONVERGED && st != GP_ERR_BREAKDOWN) return st;
    if (stats) std::memcpy(stats, all.data(), totalR * sizeof(gp_stats));
    return st;
  }
  // problems, ordered by K so that each K forms one grouped launch
  std::vector<int> order;
  for (int i = 0; i < (int)items.size(); ++i)
    if (items[i].R > 0) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return items[a].op->K < items[b].op->K; });
  const int np = (int)order.size();
  if (np == 0) {
    if (stats) {
      const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
      for (size_t i = 0; i < totalR; ++i) stats[i] = gp_stats{GP_OK, 0, 0, 0, 0.0, us};
    }
    return GP_OK;
  }
  // workspace layout: the states of all problems are contiguous so that one
  // copy brings every right-hand side's phase to the host
  struct Layout {
    size_t vec[NVEC], st, part, prof;
  };
  std::vector<Layout> lay(np);
  std::vector<Plan> plans(np);
  std::vector<gp_opts> popts(np);
  for (int j = 0; j < np; ++j) {
    popts[j] = tuned_opts(c, items[order[j]].op, items[order[j]].R, o);
    plans[j] = plan_problem(items[order[j]].op, items[order[j]].R, popts[j], c->cus);
  }
  size_t off = 0;
  const size_t st_all = off;
  {
    size_t cnt = 0;
    for (int j = 0; j < np; ++j) {
      lay[j].st = st_all + cnt * sizeof(RhsState);
      cnt += (size_t)items[order[j]].R;
    }
    off = align_up(st_all + cnt * sizeof(RhsState), 256);
  }
  for (int j = 0; j < np; ++j) {
    const Item& it = items[order[j]];
    const size_t nv = (size_t)it.R * it.op->K * it.op->N;
    for (int v = 0; v < NVEC; ++v) {
      lay[j].vec[v] = off;
      off = align_up(off + nv * tsz, 256);
    }
    lay[j].part = off;
    off = align_up(off + (size_t)NPART * it.R * plans[j].pstride * sizeof(double), 256);
    lay[j].prof = off;
    off = align_up(off + NPROF * sizeof(long long), 256);
  }
  int st = ensure_ws(c, off);
  if (st) return st;
  st = ensure_probs(c, np);
  if (st) return st;
  char* ws = (char*)c->ws;
  // descriptors, one grouped launch per distinct K
  std::vector<LaunchGroup> groups;
  const SolveCfg cfg{o.tol, f32 ? o.inner_tol : 0.0, o.max_iter, o.max_outer, o.zero_guess ? 1 : 0, 0};
  const int fpb = finalize_rhs_per_block();
  for (int j = 0; j < np; ++j) {
    const Item& it = items[order[j]];
    Prob& p = c->h_probs[j];
    std::memset(&p, 0, sizeof(Prob));
    p.op = op_dev(it.op);
    p.b = it.b;
    p.x = it.x;
    p.d = ws + lay[j].vec[0];
    p.r = ws + lay[j].vec[1];
    p.p = ws + lay[j].vec[2];
    p.q = ws + lay[j].vec[3];
    p.st = (RhsState*)(ws + lay[j].st);
    p.part = (double*)(ws + lay[j].part);
    p.prof = c->prof_on ? (long long*)(ws + lay[j].prof) : nullptr;
    p.R = it.R;
    if (!groups.empty() && groups.back().K == it.op->K && groups.back().mv_mode != plans[j].mv_mode) {
      // one matvec kernel per grouped launch: follow the group's first problem
      gp_opts oj = popts[j];
      oj.matvec = groups.back().mv_mode ? GP_MATVEC_ZMARCH : GP_MATVEC_RASTER;
      plans[j] = plan_problem(it.op, it.R, oj, c->cus);
    }
    apply_plan(p, plans[j]);
    p.cfg = cfg;
    if (groups.empty() || groups.back().K != it.op->K)
      groups.push_back(LaunchGroup{it.op->K, j, 0, 0, 0, 0, 0, 0, plans[j].mv_mode, popts[j].wg_per_cu, 0, 0});
    LaunchGroup& g = groups.back();
    p.work_begin = g.W;
    g.W += p.work_count;
    p.work_begin_o = g.Wo;
    g.Wo += p.work_count_o;
    p.mv_begin = g.Wmv;
    g.Wmv += p.mv_count;
    p.fin_begin = g.F;
    g.F += (it.R + fpb - 1) / fpb;
    g.count += 1;
  }
  size_groups(groups, c->cus);
  hipStream_t s = c->stream;
  HIPTRY(hipMemcpyAsync(c->d_probs, c->h_probs, np * sizeof(Prob), hipMemcpyHostToDevice, s));
  HIPTRY(hipMemsetAsync(ws + st_all, 0, totalR * sizeof(RhsState), s));
  for (int j = 0; j < np; ++j) HIPTRY(hipMemsetAsync(ws + lay[j].prof, 0, NPROF * sizeof(long long), s));

  // One round = [x += d, refine, finalise] then a chunk of inner iterations
  // [matvec, finalise, update] x chunk.  Without profiling both are captured
  // once per launch layout and replayed as graphs.
  const int chunk = o.chunk > 0 ? o.chunk : 6;
  const bool graphs = c->use_graphs && !c->prof_on;
  std::string layout_key;
  if (graphs) {
    layout_key = std::to_string((uintptr_t)c->d_probs) + (f32 ? "f" : "d") + std::to_string(o.precond);
    for (int j = 0; j < np; ++j) layout_key += ":" + std::to_string(plans[j].Rc);
    for (const LaunchGroup& g : groups)
      layout_key += "|" + std::to_string(g.K) + "," + std::to_string(g.count) + "," + std::to_string(g.W) + "," +
                    std::to_string(g.F) + "," + std::to_string(g.nblk) + "," + std::to_string(g.mv_mode) + "," +
                    std::to_string(g.Wmv) + "," + std::to_string(g.nblk_mv) + "," + std::to_string(g.Wo) + "," +
                    std::to_string(g.nblk_o);
  }
  auto replay = [&](const std::string& key, const std::function<int(hipStream_t)>& enqueue) -> int {
    return graph_replay(c, key, enqueue);
  };
  const int pc = o.precond;
  // rounds of round_len iterations; with FP64 inner solves a round in which no
  // right-hand side iterates is the outer step alone
  int round_len = chunk;
  uint64_t round_mask = f32 && o.chunk > 0 ? ~0ull : 1ull;
  auto launch_round = [&](bool outer_only) -> int {
    if (outer_only) {
      if (!graphs) return enqueue_outer(c, s, f32, pc, groups, c->d_probs, true);
      return replay(layout_key + "|outer",
                    [&](hipStream_t q) { return enqueue_round_branched(c, q, f32, pc, groups, c->d_probs, 0, 1); });
    }
    const int n = round_len;
    const uint64_t m = round_mask;
    if (!graphs) return enqueue_round(c, s, f32, pc, groups, c->d_probs, n, m, true);
    return replay(layout_key + "|round" + std::to_string(n) + "/" + std::to_string(m),
                  [&](hipStream_t q) { return enqueue_round_branched(c, q, f32, pc, groups, c->d_probs, n, m); });
  };
  // host copy of every right-hand side's state
  std::vector<RhsState> hs(totalR);
  int n_outer = (int)totalR, n_inner = 0;
  auto read_states = [&]() -> int {
    HIPTRY(hipMemcpyAsync(hs.data(), ws + st_all, totalR * sizeof(RhsState), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    n_outer = n_inner = 0;
    for (const RhsState& h : hs) {
      n_outer += h.phase == PH_OUTER;
      n_inner += h.phase == PH_INNER;
    }
    return GP_OK;
  };
  // Hard cap on host rounds: every round either advances an inner iteration or
  // performs a refinement step, both bounded by max_iter and max_outer.
  const long max_rounds = (long)o.max_iter + 4L * o.max_outer + 8;
  long rounds = 0;
  auto plan = [&]() { plan_round(hs, o, f32, chunk, &round_len, &round_mask); };
  while (n_outer > 0 || n_inner > 0) {
    if (++rounds > max_rounds) return fail(GP_ERR_DEVICE, "solver driver made no progress");
    st = launch_round(!f32 && n_inner == 0);
    if (st) return st;
    st = read_states();
    if (st) return st;
    plan();
  }
  // results (hs holds the final states, in problem order)
  int ret = GP_OK;
  std::vector<gp_stats> all(totalR);
  std::vector<size_t> base(items.size());
  {
    size_t b = 0;
    for (size_t i = 0; i < items.size(); ++i) {
      base[i] = b;
      b += (size_t)items[i].R;
    }
  }
  const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  size_t hpos = 0;
  for (int j = 0; j < np; ++j) {
    const Item& it = items[order[j]];
    const size_t nv = (size_t)it.op->K * it.op->N;
    for (int r = 0; r < it.R; ++r) {
      const RhsState& h = hs[hpos++];
      // b = 0, or a zero start value never updated (ended at the first refinement)
      if (h.zero_b || (o.zero_guess && h.outer <= 1))
        HIPTRY(hipMemsetAsync(it.x + (size_t)r * nv, 0, nv * sizeof(double), s));
      gp_stats& g = all[base[order[j]] + r];
      g.status = h.phase == PH_DONE ? h.status : GP_ERR_NOT_CONVERGED;
      g.inner_iters = h.total_it;
      g.outer_steps = h.outer;
      g.reserved = 0;
      g.relres = h.relres;
      g.time_us = us;
      if (g.status != GP_OK && ret == GP_OK) ret = g.status;
    }
  }
  HIPTRY(hipStreamSynchronize(s));
  if (c->prof_on) {
    std::vector<long long> pf(NPROF);
    for (int j = 0; j < np; ++j) {
      const Item& it = items[order[j]];
      HIPTRY(hipMemcpy(pf.data(), ws + lay[j].prof, NPROF * sizeof(long long), hipMemcpyDeviceToHost));
      const double N = it.op->N, K = it.op->K, ts = (double)tsz;
      const double NB = K * (K + 1) / 2, NP = o.precond == GP_PRECOND_JACOBI ? K : NB;
      // algorithmic bytes: every vector entry, block and preconditioner entry
      // a launch needs, read or written once
      // x (unless the start value is zero) and b read, r and p written
      prof_add(c, GP_KERNEL_REFINE, pf[PF_REFINE_RHS] * N,
               pf[PF_REFINE_RHS] * N * K * (16 + 2 * ts) - pf[PF_REFINE_X0] * N * K * 8 +
                   pf[PF_REFINE_ACT] * N * (NB * 8 + NP * ts));
      // x read (not on the first step from a zero start value) and written; d
      // and/or the pending step's p read
      const double addsol_rhs = std::max<double>(std::max(pf[PF_ADDSOL_D], pf[PF_ADDSOL_P]), pf[PF_ADDSOL_FRESH]);
      prof_add(c, GP_KERNEL_ADDSOL, addsol_rhs * N,
               addsol_rhs * N * K * 16 - pf[PF_ADDSOL_FRESH] * N * K * 8 +
                   (pf[PF_ADDSOL_D] + pf[PF_ADDSOL_P]) * N * K * ts);
      // p and r read, q written; blocks and preconditioner once per launch
      prof_add(c, GP_KERNEL_MATVEC, pf[PF_MATVEC_RHS] * N,
               pf[PF_MATVEC_RHS] * N * 3 * K * ts + pf[PF_MATVEC_ACT] * N * (NB + NP) * ts);
      // p, q, r, d read (d not on the first step), d, r, p written
      prof_add(c, GP_KERNEL_UPDATE, pf[PF_UPDATE_RHS] * N,
               (pf[PF_UPDATE_RHS] - pf[PF_UPDATE_FRESH]) * N * 7 * K * ts + pf[PF_UPDATE_FRESH] * N * 6 * K * ts +
                   pf[PF_UPDATE_ACT] * N * NP * ts);
    }
    if (int e = prof_resolve(c)) return e;
  }
  if (stats) std::memcpy(stats, all.data(), totalR * sizeof(gp_stats));
  if (ret == GP_ERR_NOT_CONVERGED) return fail(ret, "some right-hand sides did not reach the tolerance");
  if (ret == GP_ERR_BREAKDOWN) return fail(ret, "PCG breakdown (non-finite value or loss of definiteness)");
  return ret;
}

}  // namespace rt
}  // namespace gp

// =================================================================== C ABI
extern "C" {

void gp_opts_default(gp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->inner_tol = 1e-4;
  o->max_iter = 2000;
  o->max_outer = 30;
  o->precond = GP_PRECOND_BLOCK_JACOBI;
  o->precision = GP_PREC_FP32_REFINE64;
  o->rhs_tile = 0;
  o->chunk = 0;
  o->wg_per_cu = 0;
  o->matvec = GP_MATVEC_AUTO;
  o->seed = 0;
}

const char* gp_last_error(void) { return g_err.c_str(); }

int gp_version(void) { return 10000; }

int gp_ctx_create(int device, void* hip_stream, size_t hbm_budget, gp_ctx** out) {
  if (!out) return fail(GP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(GP_ERR_DEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(GP_ERR_INVALID_ARG, "device index out of range");
  gp_ctx* c = new gp_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->budget = hbm_budget;
  if (int st = set_device(c)) {
    delete c;
    return st;
  }
  if (int st = scratch_address(device, &c->scratch)) {
    delete c;
    return st;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->cus = cus;
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(GP_ERR_DEVICE, "could not create the capture stream");
  }
  *out = c;
  return GP_OK;
}

int gp_ctx_set_stream(gp_ctx* c, void* hip_stream) {
  if (!c) return fail(GP_ERR_INVALID_ARG, "ctx is NULL");
  BusyGuard g(c);
  if (!g.ok) return fail(GP_ERR_BUSY, "context busy");
  c->stream = (hipStream_t)hip_stream;
  return GP_OK;
}

int gp_ctx_memory(const gp_ctx* c, size_t* used, size_t* budget) {
  if (!c) return fail(GP_ERR_INVALID_ARG, "ctx is NULL");
  if (used) *used = c->used;
  if (budget) *budget = c->budget;
  return GP_OK;
}

int gp_ctx_profile(gp_ctx* c, int enable) {
  if (!c) return fail(GP_ERR_INVALID_ARG, "ctx is NULL");
  BusyGuard g(c);
  if (!g.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  if (int st = prof_resolve(c)) return st;
  c->prof_on = enable != 0;
  if (enable)
    for (auto& a : c->acc) a = gp_prof{0, 0, 0.0, 0.0};
  return GP_OK;
}

int gp_ctx_profile_read(gp_ctx* c, int kind, gp_prof* out) {
  if (!c || !out) return fail(GP_ERR_INVALID_ARG, "ctx or out is NULL");
  if (kind < 0 || kind >= GP_KERNEL_KINDS) return fail(GP_ERR_INVALID_ARG, "unknown kernel kind");
  BusyGuard g(c);
  if (!g.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  if (int st = prof_resolve(c)) return st;
  *out = c->acc[kind];
  return GP_OK;
}

int gp_ctx_destroy(gp_ctx* c) {
  if (!c) return GP_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->ws) dev_free(c, c->ws, c->ws_cap);
  if (c->rhs) dev_free(c, c->rhs, c->rhs_cap * sizeof(double));
  if (c->zbuf) dev_free(c, c->zbuf, c->zcap * sizeof(double));
  if (c->pbuf) dev_free(c, c->pbuf, c->pcap * sizeof(int8_t));
  if (c->d_probs) dev_free(c, c->d_probs, c->probs_cap * sizeof(Prob));
  if (c->h_probs) (void)hipHostFree(c->h_probs);
  if (c->d_rbp) dev_free(c, c->d_rbp, c->rbp_cap * sizeof(RbProb));
  if (c->h_rbp) (void)hipHostFree(c->h_rbp);
  if (c->h_rbst) (void)hipHostFree(c->h_rbst);
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipStream_t b : c->branch) (void)hipStreamDestroy(b);
  for (hipEvent_t e : c->branch_ev) (void)hipEventDestroy(e);
  delete c;
  return GP_OK;
}

int gp_op_destroy(gp_op* op);

static void prof_perturb(gp_op* op, int R) {
  const double K = op->K, NB = K * (K + 1) / 2, N = op->N;
  prof_add(op->ctx, GP_KERNEL_PERTURB, R * N, R * N * K * (op->dirs + 2) * 8 + N * (NB + K) * 8);
}

int gp_op_create(gp_ctx* c, const uint8_t* mask_host, int nx, int ny, int nz, int conn, int K, gp_op** out) {
  if (!out) return fail(GP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!c || !mask_host) return fail(GP_ERR_INVALID_ARG, "ctx or mask is NULL");
  if (nx < 1 || ny < 1 || nz < 1) return fail(GP_ERR_INVALID_ARG, "grid dimensions must be >= 1");
  if (conn != 4 && conn != 6) return fail(GP_ERR_INVALID_ARG, "conn must be 4 or 6");
  if (K < 1 || K > KMAX) return fail(GP_ERR_INVALID_ARG, "K must lie in [1, 24]");
  const long ncell = (long)nx * ny * nz;
  if (ncell >= (long)INT_MAX) return fail(GP_ERR_INVALID_ARG, "grid too large");
  long N = 0;
  for (long i = 0; i < ncell; ++i) N += mask_host[i] != 0;
  if (N == 0) return fail(GP_ERR_INVALID_ARG, "empty mask");
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  gp_op* op = new gp_op();
  op->ctx = c;
  op->K = K;
  op->nx = nx;
  op->ny = ny;
  op->nz = nz;
  op->conn = conn;
  op->dirs = conn == 6 ? 3 : 2;
  hipStream_t s = c->stream;
  const int cpb = grid_cells_per_block();
  const int nblocks = (int)((ncell + cpb - 1) / cpb);
  uint8_t* d_mask = nullptr;
  int *d_counts = nullptr, *d_offsets = nullptr, *d_gridmap = nullptr;
  unsigned long long* d_edges = nullptr;
  int st = GP_OK;
  auto cleanup = [&]() {
    dev_free(c, d_mask, ncell);
    dev_free(c, d_counts, nblocks * sizeof(int));
    dev_free(c, d_offsets, (nblocks + 1) * sizeof(int));
    dev_free(c, d_edges, sizeof(unsigned long long));
  };
  do {
    if ((st = dev_alloc(c, ncell, (void**)&d_mask))) break;
    if ((st = dev_alloc(c, nblocks * sizeof(int), (void**)&d_counts))) break;
    if ((st = dev_alloc(c, (nblocks + 1) * sizeof(int), (void**)&d_offsets))) break;
    if ((st = op_alloc(op, (size_t)ncell, &d_gridmap))) break;
    op->gmap = d_gridmap;
    op->ncell = (size_t)ncell;
    if ((st = dev_alloc(c, sizeof(unsigned long long), (void**)&d_edges))) break;
    hipError_t e;
    if ((e = hipMemcpyAsync(d_mask, mask_host, ncell, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_grid_build(s, d_mask, ncell, d_counts, d_offsets, nblocks)) != hipSuccess) {
      st = fail(GP_ERR_DEVICE, std::string("grid build: ") + hipGetErrorString(e));
      break;
    }
    int Nd = 0;
    if ((e = hipMemcpyAsync(&Nd, d_offsets + nblocks, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      st = fail(GP_ERR_DEVICE, std::string("grid count: ") + hipGetErrorString(e));
      break;
    }
    if (Nd != N) {
      st = fail(GP_ERR_DEVICE, "device voxel count disagrees with the mask");
      break;
    }
    op->N = (int)N;
    op->ntiles = (int)((N + TILE - 1) / TILE);
    const size_t NB = (size_t)K * (K + 1) / 2;
    if (NB * (size_t)N * sizeof(double) > 0xFFFFFFFFull) {
      st = fail(GP_ERR_INVALID_ARG, "K(K+1)/2 * N * 8 bytes must stay below 4 GiB (32-bit buffer offsets)");
      break;
    }
    if ((st = op_alloc(op, 6 * (size_t)N, &op->nbr))) break;
    if ((st = op_alloc(op, (size_t)N, &op->lin))) break;
    if ((st = op_alloc(op, NB * N, &op->B64))) break;
    if ((st = op_alloc(op, NB * N, &op->B32))) break;
    if ((st = op_alloc(op, NB * N, &op->L64))) break;
    if ((st = op_alloc(op, NB * N, &op->P64))) break;
    if ((st = op_alloc(op, NB * N, &op->P32))) break;
    if ((st = op_alloc(op, 1, &op->d_bad))) break;
    if ((e = hipHostMalloc((void**)&op->h_out, (1 + 2 * KMAX) * sizeof(double), hipHostMallocDefault)) !=
        hipSuccess) {
      op->h_out = nullptr;
      st = fail(GP_ERR_OOM, std::string("pinned trace buffer: ") + hipGetErrorString(e));
      break;
    }
    unsigned long long E = 0;
    if ((e = hipMemsetAsync(d_edges, 0, sizeof(unsigned long long), s)) != hipSuccess ||
        (e = launch_grid_index(s, d_mask, ncell, d_offsets, nblocks, d_gridmap, op->lin, op->N, nx, ny, nz, conn,
                               op->nbr, d_edges)) != hipSuccess ||
        (e = hipMemcpyAsync(&E, d_edges, sizeof(E), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      st = fail(GP_ERR_DEVICE, std::string("grid index: ") + hipGetErrorString(e));
      break;
    }
    op->E = (int64_t)E;
  } while (false);
  cleanup();
  if (st) {
    gp_op_destroy(op);
    return st;
  }
  *out = op;
  return GP_OK;
}

int gp_op_destroy(gp_op* op) {
  if (!op) return GP_OK;
  gp_ctx* c = op->ctx;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  const size_t NB = (size_t)op->K * (op->K + 1) / 2, N = (size_t)op->N;
  op_free(op, op->nbr, 6 * N);
  op_free(op, op->lin, N);
  op_free(op, op->B64, NB * N);
  op_free(op, op->B32, NB * N);
  op_free(op, op->L64, NB * N);
  op_free(op, op->P64, NB * N);
  op_free(op, op->P32, NB * N);
  op_free(op, op->d_bad, 1);
  op_free(op, op->gmap, op->ncell);
  op_free(op, op->tr_part, op->tr_cap);
  if (op->h_bad) (void)hipHostFree(op->h_bad);
  if (op->h_out) (void)hipHostFree(op->h_out);
  rb_release(op);
  delete op;
  return GP_OK;
}

int gp_op_set_blocks(gp_op* op, const double* B, int64_t* bad_voxel) {
  if (bad_voxel) *bad_voxel = -1;
  if (!op || !B) return fail(GP_ERR_INVALID_ARG, "op or B is NULL");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  return install_blocks(op, B, bad_voxel);
}

}  // extern "C"

namespace gp {
namespace rt {

int install_blocks(gp_op* op, const double* B, int64_t* bad_voxel) {
  gp_ctx* c = op->ctx;
  if (int st = reset_bad(op)) return st;
  PROFILED(c, GP_KERNEL_PACK, launch_pack_blocks(c->stream, op->K, op->N, B, op->B64, op->B32, op->L64, op->d_bad));
  {
    const double K = op->K, NB = K * (K + 1) / 2;
    prof_add(c, GP_KERNEL_PACK, op->N, (double)op->N * (K * K * 8 + NB * 20));
  }
  int bad = INT_MAX;
  if (int st = read_bad(op, &bad)) return st;
  op->pc_built = -1;
  if (bad != INT_MAX) {
    op->have_blocks = false;
    if (bad_voxel) *bad_voxel = bad;
    return fail(GP_ERR_NOT_SPD, "data block of voxel " + std::to_string(bad) + " is not positive definite");
  }
  op->have_blocks = true;
  return GP_OK;
}

}  // namespace rt
}  // namespace gp

extern "C" {

int gp_op_set_alpha(gp_op* op, const double* alpha) {
  if (!op || !alpha) return fail(GP_ERR_INVALID_ARG, "op or alpha is NULL");
  for (int k = 0; k < op->K; ++k)
    if (!(alpha[k] >= 0.0) || !std::isfinite(alpha[k])) return fail(GP_ERR_INVALID_ARG, "alpha_k must be finite and >= 0");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  for (int k = 0; k < op->K; ++k) op->alpha[k] = alpha[k];
  op->have_alpha = true;
  op->pc_built = -1;
  return GP_OK;
}

int gp_op_query(const gp_op* op, int64_t* N, int64_t* E, int* K, size_t* bytes) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (N) *N = op->N;
  if (E) *E = op->E;
  if (K) *K = op->K;
  if (bytes) *bytes = op->bytes;
  return GP_OK;
}

int gp_op_voxel_index(const gp_op* op, int32_t* lin) {
  if (!op || !lin) return fail(GP_ERR_INVALID_ARG, "op or lin is NULL");
  HIPTRY(hipMemcpyAsync(lin, op->lin, (size_t)op->N * sizeof(int), hipMemcpyDeviceToDevice, op->ctx->stream));
  return GP_OK;
}

int gp_apply(gp_op* op, int R, const double* x, double* y) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (R < 0) return fail(GP_ERR_INVALID_ARG, "R must be >= 0");
  if (R == 0) return GP_OK;
  if (!x || !y) return fail(GP_ERR_INVALID_ARG, "x or y is NULL");
  if (x == y) return fail(GP_ERR_INVALID_ARG, "x and y must not alias");
  if (R > 65535) return fail(GP_ERR_INVALID_ARG, "R too large");
  if (!op->have_blocks || !op->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  PROFILED(c, GP_KERNEL_APPLY, launch_apply(c->stream, op_dev(op), R, x, y));
  {
    const double K = op->K, NB = K * (K + 1) / 2, N = op->N;
    prof_add(c, GP_KERNEL_APPLY, R * N, R * N * 2 * K * 8 + N * NB * 8);
  }
  return GP_OK;
}

int gp_solve(gp_op* op, int R, const double* b, double* x, const gp_opts* opts, gp_stats* stats) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  gp_opts o;
  if (opts) o = *opts; else gp_opts_default(&o);
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  std::vector<Item> items{Item{op, R, b, x}};
  return run_group(c, items, o, stats);
}

int gp_solve_batch(gp_ctx* c, int n, const gp_item* items, const gp_opts* opts, gp_stats* stats) {
  if (!c) return fail(GP_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 0 || (n > 0 && !items)) return fail(GP_ERR_INVALID_ARG, "bad item list");
  gp_opts o;
  if (opts) o = *opts; else gp_opts_default(&o);
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  std::vector<Item> v;
  for (int i = 0; i < n; ++i) v.push_back(Item{items[i].op, items[i].R, items[i].b, items[i].x});
  return run_group(c, v, o, stats);
}

int gp_perturb_rhs(gp_op* op, int R, const double* bw, const double* z1, const double* z2, double* b) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (R < 0 || R > 65535) return fail(GP_ERR_INVALID_ARG, "R out of range");
  if (R == 0) return GP_OK;
  if (!bw || !z1 || !z2 || !b) return fail(GP_ERR_INVALID_ARG, "null buffer (on-device random vectors are not available)");
  if (!op->have_blocks || !op->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  PROFILED(c, GP_KERNEL_PERTURB, launch_perturb(c->stream, op_dev(op), R, bw, z1, z2, b));
  prof_perturb(op, R);
  return GP_OK;
}

int gp_sample(gp_op* op, int R, const double* bw, const double* z1, const double* z2, double* w,
              const gp_opts* opts, gp_stats* stats) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (R < 0 || R > 65535) return fail(GP_ERR_INVALID_ARG, "R out of range");
  if (R == 0) return GP_OK;
  if (!bw || !w) return fail(GP_ERR_INVALID_ARG, "null buffer");
  if ((z1 == nullptr) != (z2 == nullptr)) return fail(GP_ERR_INVALID_ARG, "z1 and z2 must both be given or both NULL");
  if (!op->have_blocks || !op->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
  gp_opts o;
  if (opts) o = *opts; else gp_opts_default(&o);
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  if (int st = ensure_rhs(c, (size_t)R * op->K * op->N)) return st;
  if (!z1) {
    const size_t n1 = (size_t)R * op->K * op->dirs * op->N, n2 = (size_t)R * op->K * op->N;
    if (int st = ensure_buf(c, c->zbuf, c->zcap, n1 + n2)) return st;
    HIPTRY(launch_rng_normal(c->stream, o.seed, 1, n1, c->zbuf));
    HIPTRY(launch_rng_normal(c->stream, o.seed, 2, n2, c->zbuf + n1));
    z1 = c->zbuf;
    z2 = c->zbuf + n1;
  }
  PROFILED(c, GP_KERNEL_PERTURB, launch_perturb(c->stream, op_dev(op), R, bw, z1, z2, c->rhs));
  prof_perturb(op, R);
  std::vector<Item> items{Item{op, R, c->rhs, w}};
  return run_group(c, items, o, stats);
}

int gp_probe_rhs(gp_op* op, int m, const int8_t* probes, double* b) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (m < 0) return fail(GP_ERR_INVALID_ARG, "m must be >= 0");
  if (m == 0) return GP_OK;
  if (!probes || !b) return fail(GP_ERR_INVALID_ARG, "null buffer");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  PROFILED(c, GP_KERNEL_PROBE, launch_probe_rhs(c->stream, (long)m * op->K * op->N, probes, b));
  prof_add(c, GP_KERNEL_PROBE, (double)m * op->N, (double)m * op->N * op->K * 9.0);
  return GP_OK;
}

static int trace_reduce_impl(gp_op* op, int m, const int8_t* probes, const double* u, double* tr_total,
                             double* tr_kk, double* tr_Gkk) {
  gp_ctx* c = op->ctx;
  const size_t need = (size_t)2 * m * op->K * op->ntiles + (size_t)2 * m * op->K + 1 + 2 * KMAX;
  if (need > op->tr_cap) {
    HIPTRY(hipStreamSynchronize(c->stream));
    op_free(op, op->tr_part, op->tr_cap);
    op->tr_cap = 0;
    if (int st = op_alloc(op, need, &op->tr_part)) return st;
    op->tr_cap = need;
  }
  double* part = op->tr_part;
  double* pairbuf = part + (size_t)2 * m * op->K * op->ntiles;
  double* out = pairbuf + (size_t)2 * m * op->K;
  PROFILED(c, GP_KERNEL_TRACE, launch_trace(c->stream, op_dev(op), m, probes, u, part, pairbuf, out));
  prof_add(c, GP_KERNEL_TRACE, (double)m * op->N, (double)m * op->N * op->K * 9.0);
  const double* h = op->h_out;
  HIPTRY(hipMemcpyAsync(op->h_out, out, (1 + 2 * op->K) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  if (tr_total) *tr_total = h[0];
  for (int k = 0; k < op->K; ++k) {
    if (tr_kk) tr_kk[k] = h[1 + k];
    if (tr_Gkk) tr_Gkk[k] = h[1 + op->K + k];
  }
  return GP_OK;
}

int gp_rng_normal(gp_ctx* c, uint64_t seed, uint64_t stream, size_t n, double* out) {
  if (!c || (n > 0 && !out)) return fail(GP_ERR_INVALID_ARG, "ctx or out is NULL");
  if (int st = set_device(c)) return st;
  HIPTRY(launch_rng_normal(c->stream, seed, stream, n, out));
  return GP_OK;
}

int gp_rng_rademacher(gp_ctx* c, uint64_t seed, uint64_t stream, size_t n, int8_t* out) {
  if (!c || (n > 0 && !out)) return fail(GP_ERR_INVALID_ARG, "ctx or out is NULL");
  if (int st = set_device(c)) return st;
  HIPTRY(launch_rng_rademacher(c->stream, seed, stream, n, out));
  return GP_OK;
}

int gp_rng_gamma(gp_ctx* c, uint64_t seed, uint64_t stream, size_t n, double shape, const double* scale,
                 double* out) {
  if (!c || (n > 0 && !out)) return fail(GP_ERR_INVALID_ARG, "ctx or out is NULL");
  if (!(shape > 0.0) || !std::isfinite(shape)) return fail(GP_ERR_INVALID_ARG, "shape must be positive");
  if (int st = set_device(c)) return st;
  HIPTRY(launch_rng_gamma(c->stream, seed, stream, n, shape, scale, out));
  return GP_OK;
}

int gp_rng_raw(gp_ctx* c, uint64_t seed, uint64_t stream, size_t nblocks, uint32_t* out) {
  if (!c || (nblocks > 0 && !out)) return fail(GP_ERR_INVALID_ARG, "ctx or out is NULL");
  if (int st = set_device(c)) return st;
  HIPTRY(launch_rng_raw(c->stream, seed, stream, nblocks, out));
  return GP_OK;
}

int gp_trace_reduce(gp_op* op, int m, const int8_t* probes, const double* u, double* tr_total, double* tr_kk,
                    double* tr_Gkk) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (m < 1 || m > 65535) return fail(GP_ERR_INVALID_ARG, "m out of range");
  if (!probes || !u) return fail(GP_ERR_INVALID_ARG, "null buffer");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  return trace_reduce_impl(op, m, probes, u, tr_total, tr_kk, tr_Gkk);
}

int gp_trace_reduce_static(gp_op* op, int m, const int8_t* probes, const double* u, double* tr_total,
                           double* tr_kk, double* tr_Gkk) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (m < 1 || m > 65535) return fail(GP_ERR_INVALID_ARG, "m out of range");
  if (!probes || !u) return fail(GP_ERR_INVALID_ARG, "null buffer");
  const size_t need = (size_t)2 * m * op->K * op->ntiles + (size_t)2 * m * op->K + 1 + 2 * KMAX;
  if (need > TRACE_SCRATCH_DOUBLES)
    return fail(GP_ERR_INVALID_ARG, "2 m K ceil(N/256) + 2 m K + 49 doubles exceed the 16 MiB static scratch (" +
                                        std::to_string(need) + " > " + std::to_string(TRACE_SCRATCH_DOUBLES) + ")");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  if (!c->scratch) return fail(GP_ERR_DEVICE, "static scratch address unknown");
  double* part = c->scratch;
  double* pairbuf = part + (size_t)2 * m * op->K * op->ntiles;
  double* out = pairbuf + (size_t)2 * m * op->K;
  // every scratch value is written before it is read within this call
  // (per-tile partials for all tiles, probes and regressors; per-probe sums;
  // the 1 + 2K totals), so nothing is cleared
  HIPTRY(launch_trace(c->stream, op_dev(op), m, probes, u, part, pairbuf, out));
  HIPTRY(hipMemcpyAsync(op->h_out, out, (1 + 2 * op->K) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  const double* h = op->h_out;
  if (tr_total) *tr_total = h[0];
  for (int k = 0; k < op->K; ++k) {
    if (tr_kk) tr_kk[k] = h[1 + k];
    if (tr_Gkk) tr_Gkk[k] = h[1 + op->K + k];
  }
  return GP_OK;
}

int gp_trace(gp_op* op, int m, const int8_t* probes, double* u, double* tr_total, double* tr_kk, double* tr_Gkk,
             const gp_opts* opts, gp_stats* stats) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (m < 1 || m > 65535) return fail(GP_ERR_INVALID_ARG, "m out of range");
  if (!u) return fail(GP_ERR_INVALID_ARG, "null buffer");
  if (!op->have_blocks || !op->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
  gp_opts o;
  if (opts) o = *opts; else gp_opts_default(&o);
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  const size_t nv = (size_t)m * op->K * op->N;
  if (!probes) {
    if (int st = ensure_buf(c, c->pbuf, c->pcap, nv)) return st;
    HIPTRY(launch_rng_rademacher(c->stream, o.seed, 3, nv, c->pbuf));
    probes = c->pbuf;
  }
  if (int st = ensure_rhs(c, nv)) return st;
  PROFILED(c, GP_KERNEL_PROBE, launch_probe_rhs(c->stream, (long)nv, probes, c->rhs));
  prof_add(c, GP_KERNEL_PROBE, (double)m * op->N, (double)m * op->N * op->K * 9.0);
  o.zero_guess = 1;   // u starts at zero and is only written
  std::vector<Item> items{Item{op, m, c->rhs, u}};
  const int st = run_group(c, items, o, stats);
  if (st != GP_OK) return st;
  return trace_reduce_impl(op, m, probes, u, tr_total, tr_kk, tr_Gkk);
}

}  // extern "C"
