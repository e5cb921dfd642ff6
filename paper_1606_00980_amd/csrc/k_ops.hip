// Operator construction and the non-iterative operations:
//   * mask -> compact voxel numbering and 6-neighbour table (Section 2, the
//     unweighted graph Laplacian over in-mask neighbours; Section 3.1, one
//     incidence row per adjacent pair)
//   * packing and Cholesky factorisation of the data blocks B_n (the L_data of
//     Algorithm 2, step 1)
//   * Jacobi / block-Jacobi preconditioner set-up from the voxel blocks of Q
//   * FP64 operator application y = Q x (Section 3)
//   * perturbed right-hand sides of Algorithm 2, step 4
//   * Hutchinson reductions for tr(Q^{-1}), tr([Q^{-1}]_kk), tr(D_w [Q^{-1}]_kk)
//     (the trace inside E[W_k D_w W_k'], Section 3.3)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "launch.hpp"
#include "pcg.hpp"
#include "spd.hpp"

namespace gp {

// ------------------------------------------------------------------ grid
constexpr int SCAN_BLOCK = 256;
constexpr int CELLS_PER_THREAD = 4;
constexpr int CELLS_PER_BLOCK = SCAN_BLOCK * CELLS_PER_THREAD;

__device__ inline int block_exclusive_scan(int v, int* s_tmp /*[SCAN_BLOCK]*/, int* total) {
  const int t = threadIdx.x;
  s_tmp[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
    const int add = t >= off ? s_tmp[t - off] : 0;
    __syncthreads();
    s_tmp[t] += add;
    __syncthreads();
  }
  const int incl = s_tmp[t];
  if (total) *total = s_tmp[SCAN_BLOCK - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_mask_count(const uint8_t* __restrict__ mask,
                                                           long ncell, int* __restrict__ counts) {
  __shared__ int s_tmp[SCAN_BLOCK];
  const long base = (long)blockIdx.x * CELLS_PER_BLOCK + (long)threadIdx.x * CELLS_PER_THREAD;
  int c = 0;
  for (int i = 0; i < CELLS_PER_THREAD; ++i) c += (base + i < ncell && mask[base + i] != 0) ? 1 : 0;
  int total;
  block_exclusive_scan(c, s_tmp, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Exclusive scan of nb block counts in one workgroup; offsets[nb] = total.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_counts(const int* __restrict__ counts, int nb,
                                                            int* __restrict__ offsets) {
  __shared__ int s_tmp[SCAN_BLOCK];
  const int per = (nb + SCAN_BLOCK - 1) / SCAN_BLOCK;
  const int lo = threadIdx.x * per;
  int sum = 0;
  for (int i = lo; i < lo + per && i < nb; ++i) sum += counts[i];
  int total;
  int run = block_exclusive_scan(sum, s_tmp, &total);
  for (int i = lo; i < lo + per && i < nb; ++i) {
    offsets[i] = run;
    run += counts[i];
  }
  if (threadIdx.x == 0) offsets[nb] = total;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_mask_index(const uint8_t* __restrict__ mask, long ncell,
                                                           const int* __restrict__ offsets,
                                                           int* __restrict__ gridmap,
                                                           int* __restrict__ lin) {
  __shared__ int s_tmp[SCAN_BLOCK];
  const long base = (long)blockIdx.x * CELLS_PER_BLOCK + (long)threadIdx.x * CELLS_PER_THREAD;
  int c = 0;
  for (int i = 0; i < CELLS_PER_THREAD; ++i) c += (base + i < ncell && mask[base + i] != 0) ? 1 : 0;
  int n = offsets[blockIdx.x] + block_exclusive_scan(c, s_tmp, nullptr);
  for (int i = 0; i < CELLS_PER_THREAD; ++i) {
    const long l = base + i;
    if (l >= ncell) break;
    if (mask[l] != 0) {
      gridmap[l] = n;
      lin[n] = (int)l;
      ++n;
    } else {
      gridmap[l] = -1;
    }
  }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_neighbours(int N, const int* __restrict__ lin,
                                                           const int* __restrict__ gridmap, int nx,
                                                           int ny, int nz, int conn,
                                                           int* __restrict__ nbr,
                                                           unsigned long long* __restrict__ edges) {
  __shared__ int s_tmp[SCAN_BLOCK];
  const int n = blockIdx.x * SCAN_BLOCK + threadIdx.x;
  int e = 0;
  if (n < N) {
    const long l = lin[n];
    const int x = (int)(l % nx);
    const int y = (int)((l / nx) % ny);
    const int z = (int)(l / ((long)nx * ny));
    const long sx = 1, sy = nx, sz = (long)nx * ny;
    int m[6];
    m[0] = x > 0 ? gridmap[l - sx] : -1;
    m[1] = x < nx - 1 ? gridmap[l + sx] : -1;
    m[2] = y > 0 ? gridmap[l - sy] : -1;
    m[3] = y < ny - 1 ? gridmap[l + sy] : -1;
    m[4] = (conn == 6 && z > 0) ? gridmap[l - sz] : -1;
    m[5] = (conn == 6 && z < nz - 1) ? gridmap[l + sz] : -1;
    for (int d = 0; d < 6; ++d) nbr[(size_t)d * N + n] = m[d] >= 0 ? m[d] : n;
    e = (m[1] >= 0) + (m[3] >= 0) + (m[5] >= 0);
  }
  int total;
  block_exclusive_scan(e, s_tmp, &total);
  if (threadIdx.x == 0 && total > 0) atomicAdd(edges, (unsigned long long)total);
}

hipError_t launch_grid_build(hipStream_t s, const uint8_t* mask, long ncell, int* counts, int* offsets,
                             int nblocks) {
  GP_LAUNCH(k_mask_count, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, mask, ncell, counts);
  GP_LAUNCH(k_scan_counts, dim3(1), dim3(SCAN_BLOCK), 0, s, counts, nblocks, offsets);
  return hipGetLastError();
}

hipError_t launch_grid_index(hipStream_t s, const uint8_t* mask, long ncell, const int* offsets,
                             int nblocks, int* gridmap, int* lin, int N, int nx, int ny, int nz, int conn,
                             int* nbr, unsigned long long* edges) {
  GP_LAUNCH(k_mask_index, dim3(nblocks), dim3(SCAN_BLOCK), 0, s, mask, ncell, offsets, gridmap,
                     lin);
  GP_LAUNCH(k_neighbours, dim3((N + SCAN_BLOCK - 1) / SCAN_BLOCK), dim3(SCAN_BLOCK), 0, s, N, lin,
                     gridmap, nx, ny, nz, conn, nbr, edges);
  return hipGetLastError();
}

int grid_cells_per_block() { return CELLS_PER_BLOCK; }

// ---------------------------------------------------------------- blocks
// Symmetrise B_n, store it packed in FP64 and FP32, and factor B_n = L L'.
template <int K>
__global__ __launch_bounds__(TILE) void k_pack_blocks(int N, const double* __restrict__ B,
                                                      double* __restrict__ B64, float* __restrict__ B32,
                                                      double* __restrict__ L64, int* __restrict__ bad) {
  constexpr int NB = Tri<K>::NB;
  const int n = blockIdx.x * TILE + threadIdx.x;
  if (n >= N) return;
  const double* Bn = B + (size_t)n * K * K;
  double a[NB];
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int j = 0; j <= k; ++j) a[pk(k, j)] = 0.5 * (Bn[k * K + j] + Bn[j * K + k]);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    B64[(size_t)i * N + n] = a[i];
    B32[(size_t)i * N + n] = (float)a[i];
  }
  double L[NB];
  bool ok = true;
  if constexpr (K <= KREG) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double dj = a[pk(j, j)];
#pragma unroll
      for (int l = 0; l < j; ++l) dj -= L[pk(j, l)] * L[pk(j, l)];
      ok = ok && (dj > 0.0) && (dj == dj);
      const double ljj = sqrt(dj > 0.0 ? dj : 1.0);
      L[pk(j, j)] = ljj;
#pragma unroll
      for (int i = j + 1; i < K; ++i) {
        double v = a[pk(i, j)];
#pragma unroll
        for (int l = 0; l < j; ++l) v -= L[pk(i, l)] * L[pk(j, l)];
        L[pk(i, j)] = v / ljj;
      }
    }
  } else {
#pragma unroll 1
    for (int i = 0; i < NB; ++i) L[i] = a[i];
    ok = cholesky_dyn(K, L);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) L64[(size_t)i * N + n] = L[i];
  if (!ok) atomicMin(bad, n);
}

// Preconditioner from the voxel block of Q, M_n = B_n + diag_k(alpha_k deg_n):
// the inverse diagonal (Jacobi) or the inverse of the whole block (block Jacobi).
template <int K>
__global__ __launch_bounds__(TILE) void k_precond(OpDev op, int pc, double* __restrict__ P64,
                                                  float* __restrict__ P32, int* __restrict__ bad) {
  constexpr int NB = Tri<K>::NB;
  const int n = blockIdx.x * TILE + threadIdx.x;
  const int N = op.N;
  if (n >= N) return;
  int deg = 0;
  for (int d = 0; d < 6; ++d) deg += op.nbr[(size_t)d * N + n] != n;
  double a[NB];
  load_soa(op.B64, N, n, a);
#pragma unroll
  for (int k = 0; k < K; ++k) a[pk(k, k)] += op.alpha64[k] * (double)deg;
  if (pc == PC_JACOBI) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double dk = a[pk(k, k)];
      ok = ok && dk > 0.0;
      const double inv = 1.0 / dk;
      P64[(size_t)k * N + n] = inv;
      P32[(size_t)k * N + n] = (float)inv;
    }
    if (!ok) atomicMin(bad, n);
    return;
  }
  // Cholesky M = L L', then M^{-1} = L^{-T} L^{-1}.
  double inv[NB];
  const bool ok = spd_inverse_any<K>(a, inv);
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    P64[(size_t)i * N + n] = inv[i];
    P32[(size_t)i * N + n] = (float)inv[i];
  }
  if (!ok) atomicMin(bad, n);
}

// ----------------------------------------------------------------- apply
template <int K>
__global__ __launch_bounds__(TILE) void k_apply(OpDev op, const double* __restrict__ x,
                                                double* __restrict__ y) {
  constexpr int NB = Tri<K>::NB;
  const int N = op.N;
  const int n = blockIdx.x * TILE + threadIdx.x;
  const int r = blockIdx.y;
  if (n >= N) return;
  int nb[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) nb[d] = op.nbr[(size_t)d * N + n];
  double B[NB];
  load_soa(op.B64, N, n, B);
  const double* xr = x + (size_t)r * K * N;
  double xo[K];
#pragma unroll
  for (int k = 0; k < K; ++k) xo[k] = xr[(size_t)k * N + n];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s6 = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) s6 += xo[k] - xr[(size_t)k * N + nb[d]];
    double v = op.alpha64[k] * s6;
#pragma unroll
    for (int j = 0; j < K; ++j) v += B[pk(k, j)] * xo[j];
    y[(size_t)r * K * N + (size_t)k * N + n] = v;
  }
}

// -------------------------------------------------------------- perturb
// b_r = b_w + (blkdiag_k sqrt(alpha_k) G_w)' z1_r + H' L_data H z2_r
// Row (n, n+e_d) of G_w has +1 at n and -1 at n+e_d; its z1 entry sits in slot
// (k, d, n).  So (G_w' z1)_n = sum_d [z1(d, n) if n+e_d in mask]
//                              - [z1(d, n-e_d) if n-e_d in mask].
template <int K>
__global__ __launch_bounds__(TILE) void k_perturb(OpDev op, const double* __restrict__ bw,
                                                  const double* __restrict__ z1,
                                                  const double* __restrict__ z2,
                                                  double* __restrict__ b, int R, int tb) {
  constexpr int NB = Tri<K>::NB;
  const int N = op.N, dirs = op.dirs;
  // items (right-hand side, tile) by blocks of tb tiles: every right-hand
  // side sweeps a block's tiles before the next one starts, and the items go
  // to the XCDs in contiguous ranges, so that the block's Cholesky factors and
  // neighbour table stay in the XCD's L2 across the right-hand sides and the
  // lower neighbours' z1 values (a plane back) were just read for the same
  // right-hand side
  const int W = gridDim.x;
  const int item = xcd_remap(blockIdx.x, W);
  const int per = tb * R;
  const int blk = item / per, rem = item - blk * per;
  const int len = min(tb, op.ntiles - blk * tb);
  const int r = rem / len, tile = blk * tb + rem % len;
  const int n = tile * TILE + threadIdx.x;
  if (n >= N) return;
  int nb[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) nb[d] = op.nbr[(size_t)d * N + n];
  double L[NB];
  load_soa(op.L64, N, n, L);
  double zz[K];
#pragma unroll
  for (int j = 0; j < K; ++j) zz[j] = z2[((size_t)r * K + j) * N + n];
  // every z1 load issued unconditionally before any use (a missing neighbour
  // is the voxel itself, so each address is valid; its term is dropped by a
  // select), so the loads of all regressors and directions are in flight together
  double hv[K][3], lv[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double* zk = z1 + ((size_t)r * K + k) * dirs * N;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int dd = d < dirs ? d : 0;
      hv[k][d] = zk[(size_t)dd * N + n];
      lv[k][d] = zk[(size_t)dd * N + nb[2 * dd]];
    }
  }
  double pr[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    pr[k] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pr[k] += d < dirs && nb[2 * d + 1] != n ? hv[k][d] : 0.0;
      pr[k] -= d < dirs && nb[2 * d] != n ? lv[k][d] : 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double dt = 0.0;
#pragma unroll
    for (int j = 0; j <= k; ++j) dt += L[pk(k, j)] * zz[j];
    b[((size_t)r * K + k) * N + n] = bw[(size_t)k * N + n] + sqrt(op.alpha64[k]) * pr[k] + dt;
  }
}

// b[r][i] += bw[i] for R right-hand sides of length kn.
__global__ void k_add_broadcast(long total, long kn, const double* __restrict__ bw, double* __restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) b[i] += bw[i % kn];
}

__global__ void k_probe_rhs(long total, const int8_t* __restrict__ v, double* __restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) b[i] = (double)v[i];
}

// ----------------------------------------------------------------- trace
// Per (probe i, regressor k, tile): sum_n v u and sum_n (D_w v)_n u, where
// (D_w v)_n = sum_d (v_n - v_nb_d(n)).  Partials laid out [2][m][K][ntiles].
template <int K>
__global__ __launch_bounds__(TILE) void k_trace_partials(OpDev op, const int8_t* __restrict__ v,
                                                         const double* __restrict__ u,
                                                         double* __restrict__ part, int m) {
  // per-thread terms, then block reductions of them through LDS, G terms at a
  // time (24 KB of LDS)
  constexpr int NV = 2 * K, G = NV < 12 ? NV : 12;
  __shared__ double s_val[G][TILE];
  __shared__ double s_mid[G][TILE / 16];
  const int N = op.N, nt = op.ntiles;
  const int tile = blockIdx.x, i = blockIdx.y;
  const int n = tile * TILE + threadIdx.x;
  const bool valid = n < N;
  const int nn = valid ? n : N - 1;
  int nb[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) nb[d] = op.nbr[(size_t)d * N + nn];
  // every load of the voxel issued before any use
  int vv[K][7];
  double un[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const size_t off = ((size_t)i * K + k) * N;
    vv[k][6] = v[off + nn];
#pragma unroll
    for (int d = 0; d < 6; ++d) vv[k][d] = v[off + nb[d]];
    un[k] = u[off + nn];
  }
  double val[NV];   // [0, K): v_k u_k, [K, 2K): (G v)_k u_k
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double gv = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) gv += (double)(vv[k][6] - vv[k][d]);
    val[k] = valid ? (double)vv[k][6] * un[k] : 0.0;
    val[K + k] = valid ? gv * un[k] : 0.0;
  }
#pragma unroll
  for (int g0 = 0; g0 < NV; g0 += G) {
    const int ng = NV - g0 < G ? NV - g0 : G;
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < ng) s_val[j][threadIdx.x] = val[g0 + j];
    __syncthreads();
    // ng x 16 partial sums of 16 terms, then ng sums of 16 partials, each in
    // a fixed order
    for (int t = threadIdx.x; t < ng * (TILE / 16); t += TILE) {
      const int q = t / (TILE / 16), c = t % (TILE / 16);
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) acc += s_val[q][c * 16 + j];
      s_mid[q][c] = acc;
    }
    __syncthreads();
    if (threadIdx.x < ng) {
      const int e = g0 + threadIdx.x, which = e / K, k = e % K;
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < TILE / 16; ++c) t += s_mid[threadIdx.x][c];
      part[(((size_t)which * m + i) * K + k) * nt + tile] = t;
    }
    __syncthreads();
  }
}

// Sums over tiles, one wavefront per (which, probe, regressor) pair:
// pairbuf[q] = sum_t part[q][t] in a fixed order.
__global__ __launch_bounds__(TILE) void k_trace_pairs(const double* __restrict__ part, int pairs, int nt,
                                                      double* __restrict__ pairbuf) {
  const int q = blockIdx.x * (TILE / WAVE) + (int)(threadIdx.x / WAVE);
  if (q >= pairs) return;
  const int lane = threadIdx.x % WAVE;
  double s = 0.0;
  for (int t = lane; t < nt; t += WAVE) s += part[(size_t)q * nt + t];
  s = wave_sum(s);
  if (lane == 0) pairbuf[q] = s;
}

// out[0] = (1/m) sum_{i,k} vu, out[1+k] = (1/m) sum_i vu_k,
// out[1+K+k] = (1/m) sum_i (Gv)u_k, each sum over probes in a fixed order.
__global__ __launch_bounds__(WAVE) void k_trace_final(const double* __restrict__ pairbuf, int m, int K,
                                                      double* __restrict__ out) {
  const int k = threadIdx.x;
  double a = 0.0, g = 0.0;
  if (k < K) {
    for (int i = 0; i < m; ++i) {
      a += pairbuf[(0 * (size_t)m + i) * K + k];
      g += pairbuf[(1 * (size_t)m + i) * K + k];
    }
    out[1 + k] = a / m;
    out[1 + K + k] = g / m;
  }
  // total over regressors in order k = 0..K-1
  double tot = 0.0;
  for (int j = 0; j < K; ++j) tot += __shfl(a, j, WAVE);
  if (k == 0) out[0] = tot / m;
}

// --------------------------------------------------------------- launchers
#define GP_K_CASES(X)                                                                                  \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
      X(20) X(21) X(22) X(23) X(24)

hipError_t launch_pack_blocks(hipStream_t s, int K, int N, const double* B, double* B64, float* B32,
                              double* L64, int* bad) {
  const dim3 g((N + TILE - 1) / TILE), b(TILE);
  switch (K) {
#define X(KK) case KK: GP_LAUNCH(k_pack_blocks<KK>, g, b, 0, s, N, B, B64, B32, L64, bad); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_precond(hipStream_t s, const OpDev& op, int pc, double* P64, float* P32, int* bad) {
  const dim3 g((op.N + TILE - 1) / TILE), b(TILE);
  switch (op.K) {
#define X(KK) case KK: GP_LAUNCH(k_precond<KK>, g, b, 0, s, op, pc, P64, P32, bad); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_apply(hipStream_t s, const OpDev& op, int R, const double* x, double* y) {
  const dim3 g((op.N + TILE - 1) / TILE, R), b(TILE);
  switch (op.K) {
#define X(KK) case KK: GP_LAUNCH(k_apply<KK>, g, b, 0, s, op, x, y); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_perturb(hipStream_t s, const OpDev& op, int R, const double* bw, const double* z1,
                          const double* z2, double* b) {
  if (op.ntiles == 0 || R == 0) return hipSuccess;
  const dim3 g((unsigned)((long)op.ntiles * R)), bl(TILE);
  // tiles per block: two planes of voxels and two tiles, the block's packed
  // factors at most 1.5 MB
  const long reach = ((long)op.N / (op.nz > 0 ? op.nz : 1) + TILE - 1) / TILE;
  const long cap = std::max(4L, (long)(1536 << 10) / ((long)(op.K * (op.K + 1) / 2) * TILE * 8));
  const int tb = (int)std::max(1L, std::min({2 * reach + 2, cap, (long)op.ntiles}));
  switch (op.K) {
#define X(KK) case KK: GP_LAUNCH(k_perturb<KK>, g, bl, 0, s, op, bw, z1, z2, b, R, tb); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_add_broadcast(hipStream_t s, int R, long kn, const double* bw, double* b) {
  const long total = (long)R * kn;
  const int bs = 256;
  GP_LAUNCH(k_add_broadcast, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, total, kn, bw, b);
  return hipGetLastError();
}

hipError_t launch_probe_rhs(hipStream_t s, long total, const int8_t* v, double* b) {
  const int bs = 256;
  GP_LAUNCH(k_probe_rhs, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, total, v, b);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, int kind, const Prob* probs, int nprob, int nblocks) {
  const dim3 g(nblocks), b(FIN_WAVES * WAVE);
  switch (kind) {
    case 0: GP_LAUNCH(k_finalize<0>, g, b, 0, s, probs, nprob); break;
    case 1: GP_LAUNCH(k_finalize<1>, g, b, 0, s, probs, nprob); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int finalize_rhs_per_block() { return FIN_WAVES; }

hipError_t launch_trace(hipStream_t s, const OpDev& op, int m, const int8_t* v, const double* u,
                        double* part, double* pairbuf, double* out) {
  const dim3 g(op.ntiles, m), b(TILE);
  switch (op.K) {
#define X(KK) case KK: GP_LAUNCH(k_trace_partials<KK>, g, b, 0, s, op, v, u, part, m); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  const int pairs = 2 * m * op.K;
  GP_LAUNCH(k_trace_pairs, dim3((pairs + TILE / WAVE - 1) / (TILE / WAVE)), dim3(TILE), 0, s, part, pairs,
                     op.ntiles, pairbuf);
  GP_LAUNCH(k_trace_final, dim3(1), dim3(WAVE), 0, s, pairbuf, m, op.K, out);
  return hipGetLastError();
}

}  // namespace gp
