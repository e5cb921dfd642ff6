// Data term of the AR(P) likelihood assembled on the device (Appendix A.2,
// Appendix B): the time-summed tensors are precomputed once per dataset, and
// each Gibbs or SVB iteration turns them, with the current noise precisions
// and AR coefficients, into the operator's blocks B_n and the vector b_w.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "gmrf.h"
#include "launch.hpp"
#include "runtime.hpp"

using namespace gp;
using namespace gp::rt;

struct gp_data {
  gp_op* op = nullptr;
  int T = 0, P = 0, K = 0, N = 0;
  double* X = nullptr;    // T x K
  double* G = nullptr;    // [X'X | R | S]
  double* YX = nullptr;   // [K][N]
  double* Bt = nullptr;   // [P][K][N]
  double* Dt = nullptr;   // [P][K][P][N]
  double* Bw = nullptr;   // [N][K][K] assembled blocks, before packing
  double* YY = nullptr;   // [N]
  double* dY = nullptr;   // [P][N]
  double* dd = nullptr;   // [P][P][N]
  double* Ja = nullptr;   // [N][P][P] assembled AR-coefficient blocks (allocated on first use)
  size_t nX = 0, nG = 0, nYX = 0, nBt = 0, nDt = 0, nBw = 0, nYY = 0, ndY = 0, ndd = 0, nJa = 0;
};

namespace {

void release(gp_data* d) {
  gp_ctx* c = d->op->ctx;
  dev_free(c, d->X, d->nX * sizeof(double));
  dev_free(c, d->G, d->nG * sizeof(double));
  dev_free(c, d->YX, d->nYX * sizeof(double));
  dev_free(c, d->Bt, d->nBt * sizeof(double));
  dev_free(c, d->Dt, d->nDt * sizeof(double));
  dev_free(c, d->Bw, d->nBw * sizeof(double));
  dev_free(c, d->YY, d->nYY * sizeof(double));
  dev_free(c, d->dY, d->ndY * sizeof(double));
  dev_free(c, d->dd, d->ndd * sizeof(double));
  dev_free(c, d->Ja, d->nJa * sizeof(double));
  delete d;
}

}  // namespace

extern "C" {

int gp_data_create(gp_op* op, int T, int P, const double* X_host, const double* Y, gp_data** out) {
  if (!out) return fail(GP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!op || !X_host || !Y) return fail(GP_ERR_INVALID_ARG, "op, X or Y is NULL");
  if (P < 0 || P > 4) return fail(GP_ERR_INVALID_ARG, "P must lie in [0, 4]");
  if (T <= P) return fail(GP_ERR_INVALID_ARG, "T must exceed P");
  const int K = op->K, N = op->N;
  if ((long)T * K > 8192) return fail(GP_ERR_INVALID_ARG, "T * K must not exceed 8192");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  gp_data* d = new gp_data();
  d->op = op;
  d->T = T;
  d->P = P;
  d->K = K;
  d->N = N;
  d->nX = (size_t)T * K;
  d->nG = (size_t)K * K + (size_t)K * K * P + (size_t)P * K * K * P;
  d->nYX = (size_t)K * N;
  d->nBt = std::max<size_t>(1, (size_t)P * K * N);
  d->nDt = std::max<size_t>(1, (size_t)P * K * P * N);
  d->nBw = (size_t)N * K * K;
  d->nYY = (size_t)N;
  d->ndY = std::max<size_t>(1, (size_t)P * N);
  d->ndd = std::max<size_t>(1, (size_t)P * P * N);
  int st = GP_OK;
  if ((st = dev_alloc(c, d->nX * sizeof(double), (void**)&d->X)) || (st = dev_alloc(c, d->nG * sizeof(double), (void**)&d->G)) ||
      (st = dev_alloc(c, d->nYX * sizeof(double), (void**)&d->YX)) ||
      (st = dev_alloc(c, d->nBt * sizeof(double), (void**)&d->Bt)) ||
      (st = dev_alloc(c, d->nDt * sizeof(double), (void**)&d->Dt)) ||
      (st = dev_alloc(c, d->nBw * sizeof(double), (void**)&d->Bw)) ||
      (st = dev_alloc(c, d->nYY * sizeof(double), (void**)&d->YY)) ||
      (st = dev_alloc(c, d->ndY * sizeof(double), (void**)&d->dY)) ||
      (st = dev_alloc(c, d->ndd * sizeof(double), (void**)&d->dd))) {
    release(d);
    return st;
  }
  hipError_t e = hipMemcpyAsync(d->X, X_host, d->nX * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_data_tensors(c->stream, T, K, P, N, d->X, Y, d->G, d->YX, d->Bt, d->Dt, d->YY, d->dY, d->dd);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    release(d);
    return fail(GP_ERR_DEVICE, std::string("data tensors: ") + hipGetErrorString(e));
  }
  *out = d;
  return GP_OK;
}

int gp_data_assemble(gp_data* d, const double* lambda, int Ns, const double* A, double* bw, int64_t* bad_voxel) {
  if (bad_voxel) *bad_voxel = -1;
  if (!d || !lambda) return fail(GP_ERR_INVALID_ARG, "data or lambda is NULL");
  if (Ns < 1) return fail(GP_ERR_INVALID_ARG, "Ns must be >= 1");
  if (d->P > 0 && !A) return fail(GP_ERR_INVALID_ARG, "A is NULL while P > 0");
  gp_op* op = d->op;
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  const int K = d->K, P = d->P, N = d->N;
  PROFILED(c, GP_KERNEL_DATA,
           launch_data_assemble(c->stream, K, P, N, Ns, d->G, d->YX, d->Bt, d->Dt, lambda, A, d->Bw, bw));
  {
    // tensors and draws read, blocks (both triangles) and b_w written
    const double per = (double)K + P * K + (double)P * K * P + 1 + (double)Ns * P + (double)K * K + (bw ? K : 0);
    prof_add(c, GP_KERNEL_DATA, N, (double)N * per * 8.0);
  }
  return install_blocks(op, d->Bw, bad_voxel);
}

int gp_data_lambda(gp_data* d, int Ns, const double* W, const double* A, double u1, double u2, double* rss,
                   double* scale, double* mean) {
  if (!d || !W) return fail(GP_ERR_INVALID_ARG, "data or W is NULL");
  if (Ns < 1) return fail(GP_ERR_INVALID_ARG, "Ns must be >= 1");
  if (d->P > 0 && !A) return fail(GP_ERR_INVALID_ARG, "A is NULL while P > 0");
  if (!(u1 > 0.0) || !(u2 >= 0.0)) return fail(GP_ERR_INVALID_ARG, "u1 > 0 and u2 >= 0 required");
  gp_ctx* c = d->op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  const double u2t = 0.5 * (d->T - d->P) + u2;
  PROFILED(c, GP_KERNEL_DATA,
           launch_data_rss(c->stream, d->K, d->P, d->N, Ns, d->G, d->YX, d->Bt, d->Dt, d->YY, d->dY, d->dd, W, A, u1,
                           u2t, rss, scale, mean));
  {
    const double K = d->K, P = d->P;
    prof_add(c, GP_KERNEL_DATA, d->N,
             (double)d->N * 8.0 * (K + P * K + P * K * P + 1 + P + P * P + Ns * (K + P) + 3));
  }
  HIPTRY(hipStreamSynchronize(c->stream));
  return GP_OK;
}

int gp_alpha_posterior(gp_op* op, int R, const double* W, double q1, double q2, double* qf_host, double* scale_host,
                       double* mean_host) {
  if (!op || !W || !scale_host || !mean_host) return fail(GP_ERR_INVALID_ARG, "null argument");
  if (R < 1) return fail(GP_ERR_INVALID_ARG, "R must be >= 1");
  if (!(q1 > 0.0) || !(q2 >= 0.0)) return fail(GP_ERR_INVALID_ARG, "q1 > 0 and q2 >= 0 required");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  const int K = op->K, nrk = R * K, nt = quadform_tiles(op->N);
  const size_t bytes = ((size_t)nrk * nt + nrk) * sizeof(double);
  double* buf = nullptr;
  if (int st = dev_alloc(c, bytes, (void**)&buf)) return st;
  std::vector<double> qf(nrk);
  hipError_t e = launch_quadform(c->stream, op_dev(op), R, W, buf, buf + (size_t)nrk * nt);
  if (e == hipSuccess)
    e = hipMemcpyAsync(qf.data(), buf + (size_t)nrk * nt, nrk * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, buf, bytes);
  if (e != hipSuccess) return fail(GP_ERR_DEVICE, std::string("quadratic forms: ") + hipGetErrorString(e));
  const double shape = 0.5 * op->N + q2;
  for (int k = 0; k < K; ++k) {
    double m = 0.0;
    for (int r = 0; r < R; ++r) m += qf[(size_t)r * K + k];
    m /= R;
    scale_host[k] = 1.0 / (0.5 * m + 1.0 / q1);
    mean_host[k] = scale_host[k] * shape;
  }
  if (qf_host) std::copy(qf.begin(), qf.end(), qf_host);
  return GP_OK;
}

void gp_hyper_default(gp_hyper* h) {
  if (!h) return;
  h->q1 = 10.0;
  h->q2 = 0.1;
  h->u1 = 10.0;
  h->u2 = 0.1;
  h->r1 = 10000.0;
  h->r2 = 0.1;
}

int gp_data_assemble_ar(gp_data* d, gp_op* op_a, const double* lambda, int Ns, const double* W, double* ba,
                        int64_t* bad_voxel) {
  if (bad_voxel) *bad_voxel = -1;
  if (!d || !op_a || !lambda || !W) return fail(GP_ERR_INVALID_ARG, "data, op_a, lambda or W is NULL");
  if (Ns < 1) return fail(GP_ERR_INVALID_ARG, "Ns must be >= 1");
  if (d->P < 1) return fail(GP_ERR_INVALID_ARG, "the data have no AR coefficients (P = 0)");
  const gp_op* op = d->op;
  if (op_a->ctx != op->ctx) return fail(GP_ERR_INVALID_ARG, "op_a belongs to another context");
  if (op_a->K != d->P) return fail(GP_ERR_INVALID_ARG, "op_a must have K = P");
  if (op_a->N != op->N || op_a->nx != op->nx || op_a->ny != op->ny || op_a->nz != op->nz)
    return fail(GP_ERR_INVALID_ARG, "op_a must be built on the data operator's mask");
  gp_ctx* c = op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  if (int st = set_device(c)) return st;
  const int K = d->K, P = d->P, N = d->N;
  if (!d->Ja) {
    d->nJa = (size_t)N * P * P;
    if (int st = dev_alloc(c, d->nJa * sizeof(double), (void**)&d->Ja)) {
      d->nJa = 0;
      return st;
    }
  }
  PROFILED(c, GP_KERNEL_DATA,
           launch_data_assemble_ar(c->stream, K, P, N, Ns, d->G, d->Bt, d->Dt, d->dY, d->dd, lambda, W, d->Ja, ba));
  {
    // tensors (B~, D, dY, dd), lambda and the draws read, blocks (both
    // triangles) and b_a written
    const double per = (double)P * K + (double)P * K * P + P + (double)P * P + 1 + (double)Ns * K + (double)P * P +
                       (ba ? P : 0);
    prof_add(c, GP_KERNEL_DATA, N, (double)N * per * 8.0);
  }
  return install_blocks(op_a, d->Ja, bad_voxel);
}

int gp_svb_step(gp_data* d, int Ns, const double* A, const double* z1, const double* z2, double* W, double* lambda,
                double* alpha_host, const gp_hyper* prior, double* bw_work, const gp_opts* opts, gp_stats* stats) {
  if (!d || !W || !lambda || !alpha_host || !bw_work) return fail(GP_ERR_INVALID_ARG, "null argument");
  if (Ns < 1) return fail(GP_ERR_INVALID_ARG, "Ns must be >= 1");
  gp_hyper h;
  if (prior) h = *prior; else gp_hyper_default(&h);
  gp_op* op = d->op;
  // q(W): data term with the current lambda and AR draws, prior alpha
  if (int st = gp_data_assemble(d, lambda, Ns, A, bw_work, nullptr)) return st;
  if (int st = gp_op_set_alpha(op, alpha_host)) return st;
  // Ns samples by Algorithm 2, warm-started from W, with the caller's (fixed) random vectors
  if (int st = gp_sample(op, Ns, bw_work, z1, z2, W, opts, stats)) return st;
  // alpha and lambda from the samples' Monte Carlo statistics
  std::vector<double> scale(op->K), mean(op->K);
  if (int st = gp_alpha_posterior(op, Ns, W, h.q1, h.q2, nullptr, scale.data(), mean.data())) return st;
  if (int st = gp_data_lambda(d, Ns, W, A, h.u1, h.u2, nullptr, nullptr, lambda)) return st;
  std::copy(mean.begin(), mean.end(), alpha_host);
  return GP_OK;
}

int gp_svb_step_ar(gp_data* d, gp_op* op_a, int Ns, const double* z1w, const double* z2w, double* W,
                   const double* z1a, const double* z2a, double* A, double* lambda, double* alpha_host,
                   double* beta_host, const gp_hyper* prior, double* bw_work, double* ba_work,
                   const gp_opts* opts, gp_stats* stats_w, gp_stats* stats_a) {
  if (!d || !op_a || !W || !A || !lambda || !alpha_host || !beta_host || !bw_work || !ba_work)
    return fail(GP_ERR_INVALID_ARG, "null argument");
  if (Ns < 1) return fail(GP_ERR_INVALID_ARG, "Ns must be >= 1");
  if (d->P < 1) return fail(GP_ERR_INVALID_ARG, "the data have no AR coefficients (P = 0)");
  const bool given = z1w && z2w && z1a && z2a;
  if (!given && (z1w || z2w || z1a || z2a))
    return fail(GP_ERR_INVALID_ARG, "z1w, z2w, z1a, z2a must all be given or all NULL");
  gp_hyper h;
  if (prior) h = *prior; else gp_hyper_default(&h);
  gp_op* op = d->op;
  // q(W): data term with the current lambda and AR draws, prior alpha, samples
  if (int st = gp_data_assemble(d, lambda, Ns, A, bw_work, nullptr)) return st;
  if (int st = gp_op_set_alpha(op, alpha_host)) return st;
  if (int st = gp_sample(op, Ns, bw_work, z1w, z2w, W, opts, stats_w)) return st;
  // q(A): the AR-coefficient system with the new W draws, prior beta, samples
  if (int st = gp_data_assemble_ar(d, op_a, lambda, Ns, W, ba_work, nullptr)) return st;
  if (int st = gp_op_set_alpha(op_a, beta_host)) return st;
  gp_opts oa;
  if (opts) oa = *opts; else gp_opts_default(&oa);
  if (!given) oa.seed = oa.seed ^ 0x9E3779B97F4A7C15ull;   // a stream of draws different from W's
  if (int st = gp_sample(op_a, Ns, ba_work, z1a, z2a, A, &oa, stats_a)) return st;
  // alpha, beta and lambda from the samples' Monte Carlo statistics
  std::vector<double> scale(std::max(op->K, op_a->K)), am(op->K), bm(op_a->K);
  if (int st = gp_alpha_posterior(op, Ns, W, h.q1, h.q2, nullptr, scale.data(), am.data())) return st;
  if (int st = gp_alpha_posterior(op_a, Ns, A, h.r1, h.r2, nullptr, scale.data(), bm.data())) return st;
  if (int st = gp_data_lambda(d, Ns, W, A, h.u1, h.u2, nullptr, nullptr, lambda)) return st;
  std::copy(am.begin(), am.end(), alpha_host);
  std::copy(bm.begin(), bm.end(), beta_host);
  return GP_OK;
}

int gp_gibbs_step(gp_data* d, const double* A, const double* z1, const double* z2, double* W, double* lambda,
                  double* alpha_host, const gp_hyper* prior, double* bw_work, uint64_t seed, uint64_t iteration,
                  const gp_opts* opts, gp_stats* stats) {
  if (!d || !W || !lambda || !alpha_host || !bw_work) return fail(GP_ERR_INVALID_ARG, "null argument");
  if ((z1 == nullptr) != (z2 == nullptr)) return fail(GP_ERR_INVALID_ARG, "z1 and z2 must both be given or both NULL");
  gp_hyper h;
  if (prior) h = *prior; else gp_hyper_default(&h);
  gp_op* op = d->op;
  gp_ctx* c = op->ctx;
  // W | lambda, A, alpha: one Algorithm-2 draw, started from the previous one
  if (int st = gp_data_assemble(d, lambda, 1, A, bw_work, nullptr)) return st;
  if (int st = gp_op_set_alpha(op, alpha_host)) return st;
  gp_opts o;
  if (opts) o = *opts; else gp_opts_default(&o);
  if (!z1) o.seed = seed ^ (iteration * 0x9E3779B97F4A7C15ull);
  if (int st = gp_sample(op, 1, bw_work, z1, z2, W, &o, stats)) return st;
  // alpha | W and lambda | W, A: scales on the device, Gamma draws
  const int K = op->K, N = op->N;
  std::vector<double> scale(K), mean(K);
  if (int st = gp_alpha_posterior(op, 1, W, h.q1, h.q2, nullptr, scale.data(), mean.data())) return st;
  double* buf = nullptr;
  const size_t bytes = ((size_t)2 * K + N) * sizeof(double);
  {
    BusyGuard guard(c);
    if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
    if (int st = set_device(c)) return st;
    if (int st = dev_alloc(c, bytes, (void**)&buf)) return st;
  }
  double* a_scale = buf;
  double* a_draw = buf + K;
  double* l_scale = buf + 2 * K;
  int st = GP_OK;
  hipError_t e = hipMemcpyAsync(a_scale, scale.data(), K * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_rng_gamma(c->stream, seed, 16 + 2 * iteration, K, 0.5 * N + h.q2, a_scale, a_draw);
  if (e == hipSuccess)
    e = hipMemcpyAsync(alpha_host, a_draw, K * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) st = fail(GP_ERR_DEVICE, std::string("alpha draw: ") + hipGetErrorString(e));
  if (st == GP_OK) st = gp_data_lambda(d, 1, W, A, h.u1, h.u2, nullptr, l_scale, nullptr);
  if (st == GP_OK) {
    e = launch_rng_gamma(c->stream, seed, 17 + 2 * iteration, N, 0.5 * (d->T - d->P) + h.u2, l_scale, lambda);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = fail(GP_ERR_DEVICE, std::string("lambda draw: ") + hipGetErrorString(e));
  }
  {
    BusyGuard guard(c);
    dev_free(c, buf, bytes);
  }
  return st;
}

int gp_alpha_extrapolate(int K, const double* a_jm2, const double* a_jm1, double* a_j) {
  if (K < 1 || !a_jm2 || !a_jm1 || !a_j) return fail(GP_ERR_INVALID_ARG, "K >= 1 and three arrays required");
  for (int k = 0; k < K; ++k) {
    const double d1 = a_jm1[k] - a_jm2[k], d2 = a_j[k] - a_jm1[k];
    const double curv = d2 - d1;   // second difference: the parabola is a_j + s t + (curv/2) t^2, t from j
    const double s = d2 + 0.5 * curv;
    double pred = a_jm1[k] + 20.0 * d2;
    if (curv != 0.0) {
      const double tv = -s / curv;   // the vertex, in iterations after j
      if (tv > 0.0) pred = a_j[k] + s * tv + 0.5 * curv * tv * tv;
    }
    a_j[k] = std::min(std::max(pred, a_j[k] / 5.0), 5.0 * a_j[k]);
  }
  return GP_OK;
}

int gp_data_destroy(gp_data* d) {
  if (!d) return GP_OK;
  gp_ctx* c = d->op->ctx;
  BusyGuard guard(c);
  if (!guard.ok) return fail(GP_ERR_BUSY, "context busy");
  (void)set_device(c);
  (void)hipStreamSynchronize(c->stream);
  release(d);
  return GP_OK;
}

}  // extern "C"
