// Autotuner for the grouped PCG launches: right-hand sides per workgroup,
// persistent workgroups per compute unit and the inner matvec kernel (for the
// red-black incomplete Cholesky solver, right-hand sides per work item).
//
// gp_autotune times every candidate on the caller's operator with R random
// right-hand sides (full solves to the requested tolerance, one warm-up and
// two timed runs each) and keeps the fastest in the context, keyed by K,
// log2 N, R rounded up to a power of two, precision and preconditioner.
// Solves whose launch options are left automatic use the tuned entry.  The
// table can be saved to and loaded from a small JSON file.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gmrf.h"
#include "launch.hpp"
#include "runtime.hpp"

using namespace gp;
using namespace gp::rt;

namespace gp {
namespace rt {

std::string tune_key(const gp_op* op, int R, const gp_opts& o) {
  int lg = 0;
  while ((1L << (lg + 1)) <= (long)op->N) ++lg;
  int rb = 1;
  while (rb < R) rb <<= 1;
  char buf[96];
  std::snprintf(buf, sizeof(buf), "K%d_N%d_R%d_p%d_c%d", op->K, lg, rb, o.precision, o.precond);
  return buf;
}

gp_opts tuned_opts(const gp_ctx* c, const gp_op* op, int R, const gp_opts& o) {
  gp_opts r = o;
  if (o.rhs_tile > 0 && o.wg_per_cu > 0 && o.matvec != GP_MATVEC_AUTO) return r;
  auto it = c->tuned.find(tune_key(op, R, o));
  if (it == c->tuned.end()) return r;
  if (r.rhs_tile == 0) r.rhs_tile = it->second.rhs_tile;
  if (r.wg_per_cu == 0) r.wg_per_cu = it->second.wg_per_cu;
  if (r.matvec == GP_MATVEC_AUTO) r.matvec = it->second.matvec;
  return r;
}

}  // namespace rt
}  // namespace gp

extern "C" {

int gp_autotune(gp_op* op, int R, const gp_opts* base, gp_opts* best) {
  if (!op) return fail(GP_ERR_INVALID_ARG, "op is NULL");
  if (R < 1 || R > 65535) return fail(GP_ERR_INVALID_ARG, "R out of range");
  if (!op->have_blocks || !op->have_alpha) return fail(GP_ERR_INVALID_ARG, "operator needs blocks and alpha");
  gp_opts o;
  if (base) o = *base; else gp_opts_default(&o);
  std::string why;
  if (!valid_opts(o, &why)) return fail(GP_ERR_INVALID_ARG, why);
  gp_ctx* c = op->ctx;
  const size_t nv = (size_t)R * op->K * op->N;
  double* buf = nullptr;
  {
    BusyGuard guard(c);
    if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
    if (int st = set_device(c)) return st;
    if (int st = dev_alloc(c, 2 * nv * sizeof(double), (void**)&buf)) return st;
    HIPTRY(launch_rng_normal(c->stream, 0x74756e65ULL, 9, nv, buf));
  }
  double* b = buf;
  double* x = buf + nv;
  struct Cand {
    int rc, wpc, mv;
  };
  std::vector<Cand> cands;
  for (int rc : {1, 2, 4, 8, 16}) {
    if (rc > R && rc != 1) continue;
    if (o.precond == GP_PRECOND_RB_IC0) {
      // the red-black solver launches one workgroup per work item: only the
      // right-hand sides per work item are tuned
      cands.push_back({rc, 0, GP_MATVEC_RASTER});
      continue;
    }
    for (int wpc : {4, 8})
      for (int mv : {GP_MATVEC_RASTER, GP_MATVEC_ZMARCH}) cands.push_back({rc, wpc, mv});
  }
  TuneEntry bestE;
  bestE.us = INFINITY;
  int ret = GP_OK;
  for (const Cand& cd : cands) {
    gp_opts t = o;
    t.rhs_tile = cd.rc;
    t.wg_per_cu = cd.wpc;
    t.matvec = cd.mv;
    double tsum = 0.0;
    bool ok = true;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      if (hipMemsetAsync(x, 0, nv * sizeof(double), c->stream) != hipSuccess) {
        ret = fail(GP_ERR_DEVICE, "hipMemsetAsync failed");
        ok = false;
        break;
      }
      const auto t0 = std::chrono::steady_clock::now();
      const int st = gp_solve(op, R, b, x, &t, nullptr);
      const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
      if (st != GP_OK) ok = false;
      if (rep > 0) tsum += us;
    }
    if (ret != GP_OK) break;
    if (ok && tsum / 2 < bestE.us) {
      bestE.us = tsum / 2;
      bestE.rhs_tile = cd.rc;
      bestE.wg_per_cu = cd.wpc;
      bestE.matvec = cd.mv;
    }
  }
  {
    BusyGuard guard(c);
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, buf, 2 * nv * sizeof(double));
    if (ret == GP_OK && std::isfinite(bestE.us)) c->tuned[tune_key(op, R, o)] = bestE;
  }
  if (ret != GP_OK) return ret;
  if (!std::isfinite(bestE.us)) return fail(GP_ERR_NOT_CONVERGED, "no candidate configuration converged");
  if (best) {
    *best = o;
    best->rhs_tile = bestE.rhs_tile;
    best->wg_per_cu = bestE.wg_per_cu;
    best->matvec = bestE.matvec;
  }
  return GP_OK;
}

int gp_tune_save(gp_ctx* c, const char* path) {
  if (!c || !path) return fail(GP_ERR_INVALID_ARG, "ctx or path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(GP_ERR_INVALID_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "{\"gmrf_tune\": 1, \"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : c->tuned) {
    std::fprintf(f, " {\"key\": \"%s\", \"rhs_tile\": %d, \"wg_per_cu\": %d, \"matvec\": %d, \"us\": %.3f}%s\n",
                 kv.first.c_str(), kv.second.rhs_tile, kv.second.wg_per_cu, kv.second.matvec, kv.second.us,
                 ++i < c->tuned.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return GP_OK;
}

int gp_tune_load(gp_ctx* c, const char* path) {
  if (!c || !path) return fail(GP_ERR_INVALID_ARG, "ctx or path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(GP_ERR_INVALID_ARG, std::string("cannot read ") + path);
  char line[512];
  int n = 0;
  while (std::fgets(line, sizeof(line), f)) {
    char key[96];
    TuneEntry e;
    if (std::sscanf(line, " {\"key\": \"%95[^\"]\", \"rhs_tile\": %d, \"wg_per_cu\": %d, \"matvec\": %d, \"us\": %lf",
                    key, &e.rhs_tile, &e.wg_per_cu, &e.matvec, &e.us) == 5) {
      if (e.rhs_tile < 1 || e.rhs_tile > RCMAX || e.wg_per_cu < 0 || e.matvec < GP_MATVEC_RASTER ||
          e.matvec > GP_MATVEC_ZMARCH)
        continue;
      c->tuned[key] = e;
      ++n;
    }
  }
  std::fclose(f);
  if (n == 0) return fail(GP_ERR_INVALID_ARG, std::string("no tuned entries in ") + path);
  return GP_OK;
}

}  // extern "C"
