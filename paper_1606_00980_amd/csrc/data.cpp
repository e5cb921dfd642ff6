// Data term of the AR(P) likelihood assembled on the device (Appendix A.2,
// Appendix B): the time-summed tensors are precomputed once per dataset, and
// each Gibbs or SVB iteration turns them, with the current noise precisions
// and AR coefficients, into the operator's blocks B_n and the vector b_w.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>

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
  size_t nX = 0, nG = 0, nYX = 0, nBt = 0, nDt = 0, nBw = 0;
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
  int st = GP_OK;
  if ((st = dev_alloc(c, d->nX * sizeof(double), (void**)&d->X)) || (st = dev_alloc(c, d->nG * sizeof(double), (void**)&d->G)) ||
      (st = dev_alloc(c, d->nYX * sizeof(double), (void**)&d->YX)) ||
      (st = dev_alloc(c, d->nBt * sizeof(double), (void**)&d->Bt)) ||
      (st = dev_alloc(c, d->nDt * sizeof(double), (void**)&d->Dt)) ||
      (st = dev_alloc(c, d->nBw * sizeof(double), (void**)&d->Bw))) {
    release(d);
    return st;
  }
  hipError_t e = hipMemcpyAsync(d->X, X_host, d->nX * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_data_tensors(c->stream, T, K, P, N, d->X, Y, d->G, d->YX, d->Bt, d->Dt);
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
