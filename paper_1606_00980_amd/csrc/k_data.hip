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
// The lambda full conditional also needs YY_n = y'y, dY_n[p] = sum_t y[t-1-p] y[t]
// and dd_n[p][q] = sum_t y[t-1-p] y[t-1-q]; its bracket is the whitened
// residual sum of squares
//   rss_n = YY - 2 YX'w + w'XXw - 2 dY'a + a'dd a + 2 a'Bt w - 2 w'(R a)w
//           - 2 a'(Dt w)a + w'(a'S a)w.
// Layouts (device, voxel fastest): Y [T][N]; YX [K][N]; Bt [P][K][N];
// Dt [P][K][P][N]; YY [N]; dY [P][N]; dd [P][P][N]; globals [XX | R | S] with
// R[k][l][p], S[p][k][l][q]; A [Ns][P][N]; W [Ns][K][N]; output blocks
// [N][K][K] (both triangles) and b_w [K][N].
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

// blockIdx.y = tensor entry (YX, Bt, Dt, YY, dY, dd in that order); threads over voxels.
// The design is staged in LDS (T*K doubles, dynamic).
__global__ __launch_bounds__(DT) void k_data_tensors(int T, int K, int P, int N, const double* __restrict__ X,
                                                     const double* __restrict__ Y, double* __restrict__ YX,
                                                     double* __restrict__ Bt, double* __restrict__ Dt,
                                                     double* __restrict__ YY, double* __restrict__ dY,
                                                     double* __restrict__ dd) {
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
  } else if (e < K + P * K + P * K * P) {
    const int i = e - K - P * K, p = i / (K * P), k = (i / P) % K, q = i % P;
    for (int t = P; t < T; ++t) s += y[(size_t)(t - 1 - p) * N + n] * sX[(t - 1 - q) * K + k];
    Dt[(size_t)i * N + n] = s;
  } else if (e == K + P * K + P * K * P) {
    for (int t = P; t < T; ++t) s += y[(size_t)t * N + n] * y[(size_t)t * N + n];
    YY[n] = s;
  } else if (e < K + P * K + P * K * P + 1 + P) {
    const int p = e - (K + P * K + P * K * P + 1);
    for (int t = P; t < T; ++t) s += y[(size_t)(t - 1 - p) * N + n] * y[(size_t)t * N + n];
    dY[(size_t)p * N + n] = s;
  } else {
    const int i = e - (K + P * K + P * K * P + 1 + P), p = i / P, q = i % P;
    for (int t = P; t < T; ++t) s += y[(size_t)(t - 1 - p) * N + n] * y[(size_t)(t - 1 - q) * N + n];
    dd[(size_t)i * N + n] = s;
  }
}

// One thread per (voxel, row k): row k of B_n and entry k of b_n.  The draws
// enter through their first two moments at the voxel, m1 = mean_j a and
// m2 = mean_j a a' (both brackets are linear in them):
//   B_kl = lambda (XX_kl - sum_p (R_klp + R_lkp) m1_p + sum_pq S_pklq m2_pq)
//   b_k  = lambda (YX_k - sum_p Bt_pk m1_p + sum_pq Dt_pkq m2_pq).
constexpr int PMAX = 4;   // largest AR order

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
  const int k = blockIdx.y;
  const double lam = lambda[n];
  double m1[PMAX] = {0.0, 0.0, 0.0, 0.0}, m2[PMAX][PMAX] = {};
  for (int j = 0; j < Ns; ++j) {
    double a[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) a[p] = p < P ? A[((size_t)j * P + p) * N + n] : 0.0;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      m1[p] += a[p];
#pragma unroll
      for (int q = 0; q < PMAX; ++q) m2[p][q] += a[p] * a[q];
    }
  }
  const double inv = Ns > 0 ? 1.0 / Ns : 0.0;
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    m1[p] *= inv;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) m2[p][q] *= inv;
  }
  // b_k first: its loads are independent of each other
  if (bw) {
    double bt[PMAX], dt[PMAX][PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      bt[p] = p < P ? Bt[((size_t)p * K + k) * N + n] : 0.0;
#pragma unroll
      for (int q = 0; q < PMAX; ++q) dt[p][q] = p < P && q < P ? Dt[(((size_t)p * K + k) * P + q) * N + n] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      acc += bt[p] * m1[p];
#pragma unroll
      for (int q = 0; q < PMAX; ++q) acc -= dt[p][q] * m2[p][q];
    }
    bw[(size_t)k * N + n] = lam * (YX[(size_t)k * N + n] - acc);
  }
  double* row = Bout + ((size_t)n * K + k) * K;
  for (int l = 0; l < K; ++l) {
    double acc = 0.0;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      if (p < P) {
        acc += (R[(k * K + l) * P + p] + R[(l * K + k) * P + p]) * m1[p];
#pragma unroll
        for (int q = 0; q < PMAX; ++q)
          if (q < P) acc -= S[((p * K + k) * K + l) * P + q] * m2[p][q];
      }
    }
    row[l] = lam * (XX[k * K + l] - acc);
  }
}

// One thread per voxel: the Monte Carlo mean over the Ns pairs (W^j, A^j) of
// the residual quadratic form, then the Gamma posterior of lambda_n:
// 1/u1t = rss/2 + 1/u1, mean = u1t * u2t (u2t = (T-P)/2 + u2).
__global__ __launch_bounds__(DT) void k_data_rss(int K, int P, int N, int Ns, const double* __restrict__ G,
                                                 const double* __restrict__ YX, const double* __restrict__ Bt,
                                                 const double* __restrict__ Dt, const double* __restrict__ YY,
                                                 const double* __restrict__ dY, const double* __restrict__ dd,
                                                 const double* __restrict__ Wall, const double* __restrict__ A,
                                                 double u1, double u2t, double* __restrict__ rss_out,
                                                 double* __restrict__ scale, double* __restrict__ mean) {
  extern __shared__ double sG[];
  const int nG = K * K + K * K * P + P * K * K * P;
  for (int i = threadIdx.x; i < nG; i += DT) sG[i] = G[i];
  __syncthreads();
  const int n = blockIdx.x * DT + threadIdx.x;
  if (n >= N) return;
  const double* XX = sG;
  const double* R = sG + K * K;
  const double* S = R + K * K * P;
  double w[KMAX], a[4];
  double tot = 0.0;
  for (int j = 0; j < Ns; ++j) {
    for (int k = 0; k < K; ++k) w[k] = Wall[((size_t)j * K + k) * N + n];
    for (int p = 0; p < P; ++p) a[p] = A[((size_t)j * P + p) * N + n];
    double v = YY[n];
    for (int k = 0; k < K; ++k) {
      double xw = 0.0;
      for (int l = 0; l < K; ++l) xw += XX[k * K + l] * w[l];
      v += w[k] * xw - 2.0 * YX[(size_t)k * N + n] * w[k];
    }
    for (int p = 0; p < P; ++p) {
      v -= 2.0 * dY[(size_t)p * N + n] * a[p];
      for (int q = 0; q < P; ++q) v += a[p] * dd[((size_t)p * P + q) * N + n] * a[q];
      for (int k = 0; k < K; ++k) {
        v += 2.0 * a[p] * Bt[((size_t)p * K + k) * N + n] * w[k];
        for (int q = 0; q < P; ++q) v -= 2.0 * a[p] * Dt[(((size_t)p * K + k) * P + q) * N + n] * w[k] * a[q];
      }
    }
    for (int k = 0; k < K; ++k) {
      for (int l = 0; l < K; ++l) {
        double ra = 0.0, asa = 0.0;
        for (int p = 0; p < P; ++p) {
          ra += R[(k * K + l) * P + p] * a[p];
          for (int q = 0; q < P; ++q) asa += a[p] * S[((p * K + k) * K + l) * P + q] * a[q];
        }
        v += w[k] * (asa - 2.0 * ra) * w[l];
      }
    }
    tot += v;
  }
  const double rss = tot / Ns;
  const double u1t = 1.0 / (0.5 * rss + 1.0 / u1);
  if (rss_out) rss_out[n] = rss;
  if (scale) scale[n] = u1t;
  if (mean) mean[n] = u1t * u2t;
}

// The AR-coefficient system (full conditional of A, Appendix A.2; its SVB
// expectation over Ns draws W^j for Ns > 1): blockIdx.y = output entry,
// packed (p, q), q <= p, of
//   J_n = lambda_n (dd_n - mean_j [D_n w + (D_n w)' - w' S w]),
// then p of
//   b_n = lambda_n (dY_n - mean_j [Bt_n w - w' R w]),          w = W^j_n,
// with (D_n w)[p][q] = sum_k Dt[p][k][q] w_k, (w'Sw)[p][q] = sum_kl w_k S[p][k][l][q] w_l,
// (Bt w)[p] = sum_k Bt[p][k] w_k, (w'Rw)[p] = sum_kl w_k R[k][l][p] w_l.  Globals in LDS.
__global__ __launch_bounds__(DT) void k_data_assemble_ar(int K, int P, int N, int Ns, const double* __restrict__ G,
                                                         const double* __restrict__ Bt, const double* __restrict__ Dt,
                                                         const double* __restrict__ dY,
                                                         const double* __restrict__ dd,
                                                         const double* __restrict__ lambda,
                                                         const double* __restrict__ W, double* __restrict__ Jout,
                                                         double* __restrict__ ba) {
  extern __shared__ double sG[];
  const int nG = K * K + K * K * P + P * K * K * P;
  for (int i = threadIdx.x; i < nG; i += DT) sG[i] = G[i];
  __syncthreads();
  const int n = blockIdx.x * DT + threadIdx.x;
  if (n >= N) return;
  const double* R = sG + K * K;
  const double* S = R + K * K * P;
  const int e = blockIdx.y, NBp = P * (P + 1) / 2;
  const double lam = lambda[n];
  double acc = 0.0;   // sum over draws of the W-dependent part
  if (e < NBp) {
    int p = 0;
    while ((p + 1) * (p + 2) / 2 <= e) ++p;
    const int q = e - p * (p + 1) / 2;
    for (int j = 0; j < Ns; ++j) {
      double dw = 0.0, wsw = 0.0;
      for (int k = 0; k < K; ++k) {
        const double wk = W[((size_t)j * K + k) * N + n];
        dw += (Dt[(((size_t)p * K + k) * P + q) * N + n] + Dt[(((size_t)q * K + k) * P + p) * N + n]) * wk;
        double sw = 0.0;
        for (int l = 0; l < K; ++l) sw += S[((p * K + k) * K + l) * P + q] * W[((size_t)j * K + l) * N + n];
        wsw += wk * sw;
      }
      acc += dw - wsw;
    }
    const double v = lam * (dd[((size_t)p * P + q) * N + n] - acc / Ns);
    Jout[((size_t)n * P + p) * P + q] = v;
    Jout[((size_t)n * P + q) * P + p] = v;
  } else {
    const int p = e - NBp;
    for (int j = 0; j < Ns; ++j) {
      double bw = 0.0, wrw = 0.0;
      for (int k = 0; k < K; ++k) {
        const double wk = W[((size_t)j * K + k) * N + n];
        bw += Bt[((size_t)p * K + k) * N + n] * wk;
        double rw = 0.0;
        for (int l = 0; l < K; ++l) rw += R[(k * K + l) * P + p] * W[((size_t)j * K + l) * N + n];
        wrw += wk * rw;
      }
      acc += bw - wrw;
    }
    if (ba) ba[(size_t)p * N + n] = lam * (dY[(size_t)p * N + n] - acc / Ns);
  }
}

// Per (sample r, regressor k, tile): sum over the tile's voxels of the squared
// differences to the in-mask +x, +y, +z neighbours (one term per adjacent
// pair, so the total is W_k D_w W_k').  Fixed-order workgroup reduction.
__global__ __launch_bounds__(DT) void k_quadform_partials(OpDev op, const double* __restrict__ W,
                                                          double* __restrict__ part) {
  __shared__ double s_red[DT / 64];
  const int N = op.N;
  const int tile = blockIdx.x, rk = blockIdx.y;
  const int n = tile * DT + threadIdx.x;
  double v = 0.0;
  if (n < N) {
    const double* w = W + (size_t)rk * N;
    const double c = w[n];
    for (int d = 0; d < op.dirs; ++d) {
      const int m = op.nbr[(size_t)(2 * d + 1) * N + n];
      if (m != n) {
        const double e = c - w[m];
        v += e * e;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < DT / 64; ++i) t += s_red[i];
    part[(size_t)rk * gridDim.x + tile] = t;
  }
}

// One wavefront per (r, k): the tile partials in a fixed order.
__global__ __launch_bounds__(64) void k_quadform_final(int nrk, int ntiles, const double* __restrict__ part,
                                                       double* __restrict__ out) {
  const int rk = blockIdx.x;
  if (rk >= nrk) return;
  double v = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += 64) v += part[(size_t)rk * ntiles + t];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (threadIdx.x == 0) out[rk] = v;
}

}  // namespace

hipError_t launch_data_tensors(hipStream_t s, int T, int K, int P, int N, const double* X, const double* Y,
                               double* G, double* YX, double* Bt, double* Dt, double* YY, double* dY, double* dd) {
  const int nG = K * K + K * K * P + P * K * K * P;
  GP_LAUNCH(k_data_globals, dim3((nG + DT - 1) / DT), dim3(DT), 0, s, T, K, P, X, G);
  if (hipError_t e = hipGetLastError()) return e;
  const int entries = K + P * K + P * K * P + 1 + P + P * P;
  GP_LAUNCH(k_data_tensors, dim3((N + DT - 1) / DT, entries), dim3(DT), (size_t)T * K * sizeof(double), s,
                     T, K, P, N, X, Y, YX, Bt, Dt, YY, dY, dd);
  return hipGetLastError();
}

hipError_t launch_data_rss(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* YX,
                           const double* Bt, const double* Dt, const double* YY, const double* dY, const double* dd,
                           const double* W, const double* A, double u1, double u2t, double* rss, double* scale,
                           double* mean) {
  const int nG = K * K + K * K * P + P * K * K * P;
  GP_LAUNCH(k_data_rss, dim3((N + DT - 1) / DT), dim3(DT), (size_t)nG * sizeof(double), s, K, P, N, Ns, G, YX,
                     Bt, Dt, YY, dY, dd, W, A, u1, u2t, rss, scale, mean);
  return hipGetLastError();
}

int quadform_tiles(int N) { return (N + DT - 1) / DT; }

hipError_t launch_quadform(hipStream_t s, const OpDev& op, int R, const double* W, double* part, double* out) {
  const int nt = quadform_tiles(op.N), nrk = R * op.K;
  GP_LAUNCH(k_quadform_partials, dim3(nt, nrk), dim3(DT), 0, s, op, W, part);
  if (hipError_t e = hipGetLastError()) return e;
  GP_LAUNCH(k_quadform_final, dim3(nrk), dim3(64), 0, s, nrk, nt, part, out);
  return hipGetLastError();
}

hipError_t launch_data_assemble(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* YX,
                                const double* Bt, const double* Dt, const double* lambda, const double* A,
                                double* Bout, double* bw) {
  const int nG = K * K + K * K * P + P * K * K * P;
  if (P > PMAX) return hipErrorInvalidValue;
  GP_LAUNCH(k_data_assemble, dim3((N + DT - 1) / DT, K), dim3(DT), (size_t)nG * sizeof(double), s, K,
                     P, N, Ns, G, YX, Bt, Dt, lambda, A, Bout, bw);
  return hipGetLastError();
}

hipError_t launch_data_assemble_ar(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* Bt,
                                   const double* Dt, const double* dY, const double* dd, const double* lambda,
                                   const double* W, double* Jout, double* ba) {
  const int nG = K * K + K * K * P + P * K * K * P;
  const int entries = P * (P + 1) / 2 + P;
  GP_LAUNCH(k_data_assemble_ar, dim3((N + DT - 1) / DT, entries), dim3(DT), (size_t)nG * sizeof(double), s,
                     K, P, N, Ns, G, Bt, Dt, dY, dd, lambda, W, Jout, ba);
  return hipGetLastError();
}

}  // namespace gp
