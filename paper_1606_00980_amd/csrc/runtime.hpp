// Internal host runtime shared by the C ABI (api.cpp) and the serving loop
// (server.cpp): context and operator records, allocation under the context's
// HBM budget, error reporting.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <functional>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "gmrf.h"

namespace gp {
namespace rt {

// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string& msg);

}  // namespace rt
}  // namespace gp

#define HIPTRY(call)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return gp::rt::fail(GP_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One autotuned launch configuration (see tune.cpp).
struct TuneEntry {
  int rhs_tile = 0, wg_per_cu = 0, matvec = 0;
  double us = 0.0;
};

struct gp_ctx {
  int device = 0;
  double* scratch = nullptr;   // device address of the library's static scratch array on this device
  int cus = 256;     // compute units of the device
  hipStream_t stream = nullptr;
  size_t budget = 0, used = 0;
  std::atomic<int> busy{0};
  // solver workspace arena (grown on demand, reused across calls)
  void* ws = nullptr;
  size_t ws_cap = 0;
  // right-hand-side staging for sample/trace, and on-device random vectors
  double* rhs = nullptr;
  size_t rhs_cap = 0;
  double* zbuf = nullptr;
  size_t zcap = 0;
  int8_t* pbuf = nullptr;
  size_t pcap = 0;
  // grouped-launch descriptors
  gp::Prob* d_probs = nullptr;
  gp::Prob* h_probs = nullptr;
  size_t probs_cap = 0;
  // profiling: event pairs around launches, resolved after the stream drains
  bool prof_on = false;
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> pending;   // (kind, first event of the pair)
  gp_prof acc[GP_KERNEL_KINDS] = {};
  // captured launch sequences, keyed by the grouped-launch layout
  hipStream_t cap_stream = nullptr;
  // branch streams and fork/join events for capturing the launch groups of a
  // round as parallel graph branches (default priority, non-blocking)
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> branch_ev;   // [0] fork, [1 + g] join of branch g
  struct GraphEntry {
    hipGraphExec_t exec;
    uint64_t used;   // graph_tick at its last replay
  };
  std::map<std::string, GraphEntry> graphs;
  uint64_t graph_tick = 0;
  bool use_graphs = true;
  // autotuned configurations keyed by tune_key()
  std::map<std::string, TuneEntry> tuned;
  // red-black solver: grouped-launch descriptors and a pinned copy of the states
  gp::RbProb* d_rbp = nullptr;
  gp::RbProb* h_rbp = nullptr;
  size_t rbp_cap = 0;
  gp::RhsState* h_rbst = nullptr;
  size_t rbst_cap = 0;
};

namespace gp {
namespace rt {
struct RbData;
}  // namespace rt
}  // namespace gp

struct gp_op {
  gp_ctx* ctx = nullptr;
  int N = 0, K = 0, nx = 0, ny = 0, nz = 0, conn = 0, dirs = 0, ntiles = 0;
  int64_t E = 0;
  int* nbr = nullptr;
  int* lin = nullptr;
  double* B64 = nullptr;
  float* B32 = nullptr;
  double* L64 = nullptr;
  double* P64 = nullptr;
  float* P32 = nullptr;
  int* d_bad = nullptr;
  int* h_bad = nullptr;      // pinned host copy of d_bad
  double* h_out = nullptr;   // pinned host buffer of the trace results (1 + 2 KMAX)
  int* gmap = nullptr;      // [nz][ny][nx] voxel number or -1
  size_t ncell = 0;
  double* tr_part = nullptr;
  size_t tr_cap = 0;
  double alpha[gp::KMAX] = {0};
  bool have_blocks = false, have_alpha = false;
  int pc_built = -1;
  int pc_want = GP_PRECOND_BLOCK_JACOBI;
  gp::rt::RbData* rb = nullptr;   // red-black split and its preconditioner, built on first use
  size_t bytes = 0;
};

namespace gp {
namespace rt {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct BusyGuard {
  gp_ctx* c;
  bool ok;
  explicit BusyGuard(gp_ctx* ctx) : c(ctx) {
    int expect = 0;
    ok = c->busy.compare_exchange_strong(expect, 1);
  }
  ~BusyGuard() {
    if (ok) c->busy.store(0);
  }
};

// Work decomposition of one problem (operator + R right-hand sides) for the
// grouped launches: raster tiles x chunks of Rc right-hand sides for the
// matvec and update (the matvec may instead use z-marching footprints), and
// tiles x chunks of Rco <= 4 for refine and addsol, which prefer short chunks.
struct Plan {
  int Rc, nchunks, work_count, pstride;
  int Rco, nchunks_o, work_count_o;
  int mv_mode, zs, nseg, nyt, mv_tiles, mv_nchunks, mv_count;
};
Plan plan_problem(const gp_op* op, int R, const gp_opts& o, int cus);
// Cache key of a tuned configuration: K, log2 N, R rounded up to a power of
// two, precision and preconditioner.
std::string tune_key(const gp_op* op, int R, const gp_opts& o);
// o with its automatic (zero) launch fields filled from the context's tuned
// entry for (op, R), when there is one.
gp_opts tuned_opts(const gp_ctx* c, const gp_op* op, int R, const gp_opts& o);
void apply_plan(Prob& p, const Plan& pl);

// One grouped launch per distinct K: problems [first, first + count) of the
// descriptor array, W raster work items (Wmv for a z-marching matvec), F
// finalising workgroups, nblk (nblk_mv) persistent workgroups.
struct LaunchGroup {
  int K, first, count, W, F, nblk, Wmv, nblk_mv, mv_mode, wpc;
  int Wo, nblk_o;   // refine / addsol work items and workgroups
};
// Number of inner vectors (d, r, p, q) per right-hand side in the inner precision.
constexpr int NVEC = 4;
// Persistent workgroup counts of every group: wg_per_cu (default 8) per
// compute unit, a multiple of the XCD count, no more than the work items.
void size_groups(std::vector<LaunchGroup>& gs, int cus);
// Enqueue on stream q, for every group: [x += d, refine, finalise] (the
// outer step of a solver round), or iters x [matvec, finalise, update].
// With `profiled` and profiling on, each launch is timed with events.
int enqueue_outer(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                  const Prob* d_probs, bool profiled);
int enqueue_inner(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                  const Prob* d_probs, int iters, bool profiled);
// One solver round of `chunk` iterations (chunk = 0: the outer step alone,
// when bit 0 of outer_mask is set).  Iteration i (0-based) is preceded
// by the outer step ([x += d, refine, finalise] for right-hand sides waiting
// on it) when bit i of outer_mask is set: with FP32 inner solves, which end
// every few iterations, the host places it where inner solves are expected to
// end, so a right-hand side rarely idles until the next round.
int enqueue_round(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                  const Prob* d_probs, int chunk, uint64_t outer_mask, bool profiled);
// The same round with each launch group on a branch stream forked from q and
// joined back into it (used while capturing, so that the groups of an uneven
// batch become parallel graph branches).
int enqueue_round_branched(gp_ctx* c, hipStream_t q, bool f32, int pc, const std::vector<LaunchGroup>& gs,
                           const Prob* d_probs, int chunk, uint64_t outer_mask);

// Branch streams (and fork/join events) for capturing n launch groups as
// parallel graph branches.
int ensure_branches(gp_ctx* c, size_t n);

// Per-launch event timing while profiling is on (gp_ctx_profile).
int prof_begin(gp_ctx* c, size_t* slot);
int prof_end(gp_ctx* c, int kind, size_t slot);
int prof_resolve(gp_ctx* c);
void prof_add(gp_ctx* c, int kind, double units, double bytes);
#define PROFILED(ctx, kind, launch)                                  \
  do {                                                               \
    size_t slot_ = 0;                                                \
    if ((ctx)->prof_on) {                                            \
      if (int st_ = prof_begin((ctx), &slot_)) return st_;           \
    }                                                                \
    const hipError_t le_ = (launch);                                 \
    if ((ctx)->prof_on) {                                            \
      if (int st_ = prof_end((ctx), (kind), slot_)) return st_;      \
    }                                                                \
    HIPTRY(le_);                                                     \
  } while (0)

#define PROFILED_IF(on, ctx, kind, launch) \
  do {                                      \
    if (on) {                               \
      PROFILED(ctx, kind, launch);          \
    } else {                                \
      HIPTRY(launch);                       \
    }                                       \
  } while (0)

int set_device(gp_ctx* c);
int dev_alloc(gp_ctx* c, size_t bytes, void** p);
void dev_free(gp_ctx* c, void* p, size_t bytes);
OpDev op_dev(const gp_op* op);
int build_precond(gp_op* op, int pc);
// Grow the context's solver workspace to at least `bytes`.
int ensure_ws(gp_ctx* c, size_t bytes);
// The operator's failure flag: reset to INT_MAX, and read (waits for the stream).
int reset_bad(gp_op* op);
int read_bad(gp_op* op, int* bad);
// Pack, factor and SPD-check device blocks B ([N][K][K] FP64) into op, as
// gp_op_set_blocks does (the caller holds the context).
int install_blocks(gp_op* op, const double* B, int64_t* bad_voxel);
bool valid_opts(const gp_opts& o, std::string* why);
// Length and outer-step mask (bit i: the outer step precedes iteration i) of
// the next solver round, planned from the right-hand sides' states.
void plan_round(const std::vector<RhsState>& hs, const gp_opts& o, bool f32, int chunk, int* round_len,
                uint64_t* round_mask);
// Launch the graph cached under key on the context's stream, capturing it
// first from enqueue(capture stream) when absent (the least recently used is
// dropped beyond GRAPH_CACHE).
int graph_replay(gp_ctx* c, const std::string& key, const std::function<int(hipStream_t)>& enqueue);
// Red-black incomplete Cholesky preconditioner (rbic.cpp): set-up for op, the
// grouped solves, and release of its data.
int rb_build(gp_op* op);
// The set-up of several operators (distinct), their launches side by side on
// branch streams when there are many.
int rb_build_ops(gp_ctx* c, const std::vector<gp_op*>& ops);
// Reads the set-up's positive-definiteness flag if it has not been read yet
// (waits for the stream); GP_ERR_NOT_SPD when a block failed.
int rb_check_built(gp_op* op);
void rb_release(gp_op* op);
RbDev rb_dev(const gp_op* op);
// One caller batch item of an operator: R right-hand sides b, solutions x,
// and where their statistics go.
struct RbItem {
  int R;
  const double* b;
  double* x;
  gp_stats* stats;
};
struct RbOpItems {
  gp_op* op;
  std::vector<RbItem> items;
};
// Solves every item of every operator together: the right-hand sides of an
// operator stacked in one member (at most 65535), the members grouped by K,
// one launch per group and kernel.
int rb_solve_group(gp_ctx* c, const std::vector<RbOpItems>& ops, const gp_opts& o);
// A member of a grouped red-black solve: its descriptor and the buffers
// outside it.
struct RbMember {
  gp_op* op = nullptr;
  int R = 0;
  bool f32 = true;
  RbProb desc{};
  double* t64 = nullptr;       // [R][K][NR] t = Q_nn^{-1} b_n of the split (for the recovery)
  long long* prof = nullptr;   // work counters while profiling
};
// One launch group: members [first, first + count) of the descriptor array,
// all with K regressors; work items of the black, red and outer launches and
// finalising workgroups.
struct RbGroup {
  int K, first, count, WB, WR, WO, F;
  int uw;   // 2 when some member stores the red-stage vector in pairs, else 1
};
// Device bytes of a member's vectors and partials (states excluded).
size_t rb_member_bytes(const gp_op* op, int R, bool f32);
// Lays out a member's buffers in mem (rb_member_bytes long) and fills its
// descriptor, except the work ranges that rb_groups sets.
void rb_member(gp_op* op, int R, bool f32, char* mem, RhsState* st, const SolveCfg& cfg, bool prof, RbMember* out);
// Groups the n descriptors h (sorted by K) and sets their work ranges and
// finalisation blocks; with outer_chunks the outer-step work items take the
// inner chunks of right-hand sides instead of one each.
std::vector<RbGroup> rb_groups(RbProb* h, int n, int rhs_tile, bool outer_chunks);
// Enqueues one solver round (see rbic.cpp) for every group on q; with
// `branched` each group on a branch stream forked from q and joined back.
int rb_enqueue_round(gp_ctx* c, hipStream_t q, bool f32, const std::vector<RbGroup>& gs, const RbProb* d_probs,
                     int len, uint64_t mask, bool tail, bool first, bool profiled, bool branched);
// Split of right-hand sides [r0, r0 + R) of a member (b, x in the caller's
// layout), and the recovery of their solutions into x, on stream s (timed
// when `profiled`, s is the context's stream and profiling is on).
int rb_split_member(gp_ctx* c, hipStream_t s, const RbMember& m, int r0, int R, const double* b, const double* x,
                    bool zero_guess, bool profiled);
int rb_recover_member(gp_ctx* c, hipStream_t s, const RbMember& m, int r0, int R, double* x, bool profiled);
// Grow the context's red-black descriptor array and pinned state copy.
int ensure_rb_probs(gp_ctx* c, size_t n);
int ensure_rb_states(gp_ctx* c, size_t n);

}  // namespace rt
}  // namespace gp
