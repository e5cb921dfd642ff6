// Data term of the AR(P) likelihood on the device (Appendix A.2).
//
// Time-summed tensors, conditional on the first P scans (scans t = P..T-1,
// lagged design X~[t] with row p = X[t-1-p], lagged data d_t with entry
// p = y[t-1-p]):
//   global    XX = X'X (K x K), R = X'X~ (K x K x P), S = X~X~ (P x K x K x P)
//   per voxel YX_n = Y_n'X (K), Bt_n = Y_n'X~ + d_n X (P x K), Dt_n = d_n X~ (P x K x P)
// and, for noise precisions lambda and Ns draws A^j of the AR coefficients
// (the full conditional of W for Ns = 1, its SVB expectation for Ns > 1,
// Appendix B),
//   B_n = lambda_n (XX - mean_j [R a + (R a)' - a' S a]),  a = A^j_n
//   b_n = lambda_n (YX_n - mean_j [a' Bt_n - a' Dt_n a]).
// Layouts (device, voxel fastest): Y [T][N]; YX [K][N]; Bt [P][K][N];
// Dt [P][K][P][N]; globals [XX | R | S] with R[k][l][p], S[p][k][l][q];
// A [Ns][P][N]; output blocks [N][K][K] (both triangles) and b_w [K][N].
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace gp {

namespace {

constexpr int DT = 256;   // threads per workgroup

// One thread per global tensor entry.
__global__ __launch_bounds__(DT) void k_data_globals(int T, int K, int P, const double* __restrict__ X,
                                                     double* __restrict__ G) {
  const int e = blockIdx.x * DT + threadIdx.x;
  const int nXX = K * K, nR = K * K * P, nS = P * K * K * P;
  if (e >= nXX + nR + nS) return;
  double s = 0.0;
  if (e < nXX) {
    const int k = e / K, l = e % K;
    for (int t = P; t < T; ++t) s += X[t * K + k] * X[t * K + l];
  } else if (e < nXX + nR) {
    const int i = e - nXX, k = i / (K * P), l = (i / P) % K, p = i % P;
    for (int t = P; t < T; ++t) s += X[t * K + k] * X[(t - 1 - p) * K + l];
  } else {
    const int i = e - nXX - nR;
    const int p = i / (K * K * P), k = (i / (K * P)) % K, l = (i / P) % K, q = i % P;
    for (int t = P; t < T; ++t) s += X[(t - 1 - p) * K + k] * X[(t - 1 - q) * K + l];
  }
  G[e] = s;
}

// blockIdx.y = tensor entry (YX, then Bt, then Dt); threads over voxels.
// The design is staged in LDS (T*K doubles, dynamic).
__global__ __launch_bounds__(DT) void k_data_tensors(int T, int K, int P, int N, const double* __restrict__ X,
                                                     const double* __restrict__ Y, double* __restrict__ YX,
                                                     double* __restrict__ Bt, double* __restrict__ Dt) {
  extern __shared__ double sX[];
  for (int i = threadIdx.x; i < T * K; i += DT) sX[i] = X[i];
  __syncthreads();
  const int n = blockIdx.x * DT + threadIdx.x;
  if (n >= N) return;
  const int e = blockIdx.y;
  const __attribute__((address_space(1))) double* y = (const __attribute__((address_space(1))) double*)Y;
  double s = 0.0;
  if (e < K) {
    const int k = e;
    for (int t = P; t < T; ++t) s += y[(size_t)t * N + n] * sX[t * K + k];
    YX[(size_t)k * N + n] = s;
  } else if (e < K + P * K) {
    const int i = e - K, p = i / K, k = i % K;
    for (int t = P; t < T; ++t)
      s += y[(size_t)t * N + n] * sX[(t - 1 - p) * K + k] + y[(size_t)(t - 1 - p) * N + n] * sX[t * K + k];
    Bt[(size_t)i * N + n] = s;
  } else {
    const int i = e - K - P * K, p = i / (K * P), k = (i / P) % K, q = i % P;
    for (int t = P; t < T; ++t) s += y[(size_t)(t - 1 - p) * N + n] * sX[(t - 1 - q) * K + k];
    Dt[(size_t)i * N + n] = s;
  }
}

// blockIdx.y = output entry: packed (k, l), l <= k, of B_n, then k of b_n.
// Globals in LDS.
__global__ __launch_bounds__(DT) void k_data_assemble(int K, int P, int N, int Ns, const double* __restrict__ G,
                                                      const double* __restrict__ YX, const double* __restrict__ Bt,
                                                      const double* __restrict__ Dt,
                                                      const double* __restrict__ lambda,
                                                      const double* __restrict__ A, double* __restrict__ Bout,
                                                      double* __restrict__ bw) {
  extern __shared__ double sG[];
  const int nG = K * K + K * K * P + P * K * K * P;
  for (int i = threadIdx.x; i < nG; i += DT) sG[i] = G[i];
  __syncthreads();
  const int n = blockIdx.x * DT + threadIdx.x;
  if (n >= N) return;
  const double* XX = sG;
  const double* R = sG + K * K;
  const double* S = R + K * K * P;
  const int e = blockIdx.y, NB = K * (K + 1) / 2;
  const double lam = lambda[n];
  double acc = 0.0;   // sum over draws of the subtracted AR part
  if (e < NB) {
    int k = 0;
    while ((k + 1) * (k + 2) / 2 <= e) ++k;
    const int l = e - k * (k + 1) / 2;
    for (int j = 0; j < Ns; ++j) {
      double ra = 0.0, asa = 0.0;
      for (int p = 0; p < P; ++p) {
        const double ap = A[((size_t)j * P + p) * N + n];
        ra += (R[(k * K + l) * P + p] + R[(l * K + k) * P + p]) * ap;
        for (int q = 0; q < P; ++q) asa += ap * S[((p * K + k) * K + l) * P + q] * A[((size_t)j * P + q) * N + n];
      }
      acc += ra - asa;
    }
    const double v = lam * (XX[k * K + l] - acc / Ns);
    Bout[((size_t)n * K + k) * K + l] = v;
    Bout[((size_t)n * K + l) * K + k] = v;
  } else {
    const int k = e - NB;
    for (int j = 0; j < Ns; ++j) {
      double ab = 0.0, ada = 0.0;
      for (int p = 0; p < P; ++p) {
        const double ap = A[((size_t)j * P + p) * N + n];
        ab += ap * Bt[((size_t)p * K + k) * N + n];
        for (int q = 0; q < P; ++q)
          ada += ap * Dt[(((size_t)p * K + k) * P + q) * N + n] * A[((size_t)j * P + q) * N + n];
      }
      acc += ab - ada;
    }
    if (bw) bw[(size_t)k * N + n] = lam * (YX[(size_t)k * N + n] - acc / Ns);
  }
}

}  // namespace

hipError_t launch_data_tensors(hipStream_t s, int T, int K, int P, int N, const double* X, const double* Y,
                               double* G, double* YX, double* Bt, double* Dt) {
  const int nG = K * K + K * K * P + P * K * K * P;
  hipLaunchKernelGGL(k_data_globals, dim3((nG + DT - 1) / DT), dim3(DT), 0, s, T, K, P, X, G);
  if (hipError_t e = hipGetLastError()) return e;
  const int entries = K + P * K + P * K * P;
  hipLaunchKernelGGL(k_data_tensors, dim3((N + DT - 1) / DT, entries), dim3(DT), (size_t)T * K * sizeof(double), s,
                     T, K, P, N, X, Y, YX, Bt, Dt);
  return hipGetLastError();
}

hipError_t launch_data_assemble(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* YX,
                                const double* Bt, const double* Dt, const double* lambda, const double* A,
                                double* Bout, double* bw) {
  const int nG = K * K + K * K * P + P * K * K * P;
  const int entries = K * (K + 1) / 2 + K;
  hipLaunchKernelGGL(k_data_assemble, dim3((N + DT - 1) / DT, entries), dim3(DT), (size_t)nG * sizeof(double), s, K,
                     P, N, Ns, G, YX, Bt, Dt, lambda, A, Bout, bw);
  return hipGetLastError();
}

}  // namespace gp
