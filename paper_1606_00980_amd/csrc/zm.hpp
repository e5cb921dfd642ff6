// Z-marching variant of the PCG matvec step (same arithmetic as k_matvec in
// pcg.hpp):  q = Q p and the seven per-tile inner products of the step.
//
// A workgroup owns a 64 x 4 (x, y) footprint of the grid, a segment of z
// slices and a few right-hand sides.  It walks the slices upwards: the own
// voxel's values at z-1, z and z+1 stay in registers, the in-plane
// neighbours come from a one-cell-halo copy of the slice in LDS, and the
// voxel's block B_n is loaded once per slice for all of the workgroup's
// right-hand sides.  Every vector entry is then fetched about once per
// launch (plus the segment's two boundary slices and the halo, which the
// neighbouring workgroups have just fetched), instead of once per neighbour
// as in the raster kernel, whose z-neighbour slice lies beyond the L2 reuse
// distance when many right-hand sides stream together.
#pragma once
#include "pcg.hpp"

namespace gp {

constexpr int ZFX = 64;   // footprint width: one wavefront per grid row
constexpr int ZFY = 4;    // footprint height: four rows per workgroup

// right-hand sides per z-marching workgroup
template <int K> struct ZRc { static constexpr int v = K <= 4 ? 4 : (K <= 8 ? 2 : 1); };

// Waits for this workgroup's LDS traffic and meets the other wavefronts,
// without waiting for outstanding global loads (the prefetch of the next
// slice stays in flight across the barrier).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

struct ZWhere {
  int p, chunk, tile, seg, yt, xt;
};

// Work items of a problem: tile major ((xt, yt, seg)), right-hand-side chunk
// minor, so consecutive items share the footprint's blocks in L2.
__device__ inline ZWhere zlocate(const Prob* __restrict__ probs, int nprob, int item) {
  ZWhere w;
  int p = 0;
  while (p + 1 < nprob && item >= probs[p + 1].mv_begin) ++p;
  w.p = p;
  const Prob& pr = probs[p];
  int local = item - pr.mv_begin;
  w.chunk = local % pr.mv_nchunks;
  local /= pr.mv_nchunks;
  w.tile = local;
  w.seg = local % pr.nseg;
  local /= pr.nseg;
  w.yt = local % pr.nyt;
  w.xt = local / pr.nyt;
  return w;
}

template <typename T, int PC, int K>
__global__ __launch_bounds__(ZFX * ZFY) void k_matvec_zm(const Prob* __restrict__ probs, int nprob, int W) {
  constexpr int NB = Tri<K>::NB;
  constexpr int RC = ZRc<K>::v;
  constexpr int ROWS = ZFY + 2, COLS = ZFX + 2;
  __shared__ T s_p[RC * K][ROWS][COLS];
  __shared__ int s_n[ROWS][COLS];
  __shared__ double s_red[RC * NPART][ZFY];
  const int lane = threadIdx.x % ZFX, ty = threadIdx.x / ZFX;
  for (Sweep sw = sweep_begin(W); sw.item < sw.end; sw.item += sw.step) {
    const ZWhere w = zlocate(probs, nprob, sw.item);
    const Prob& pr = probs[w.p];
    const OpDev& op = pr.op;
    const int r0 = w.chunk * RC;
    const int r1 = min(pr.R, r0 + RC);
    if (!any_in_phase(pr, r0, r1, PH_INNER)) continue;
    if (w.tile == 0 && w.chunk == 0) prof_launch(pr, PF_MATVEC_ACT, PH_INNER);
    const int N = op.N, nx = op.nx, ny = op.ny, nz = op.nz;
    const bool zc = op.dirs == 3;   // 4-neighbour operators do not couple slices
    const __attribute__((address_space(1))) int* gm = (const __attribute__((address_space(1))) int*)op.gmap;
    bool act[RC];
    Rsrc pb[RC], rb[RC], qb[RC];
    const unsigned row = (unsigned)N * sizeof(T);
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const int r = r0 + i;
      act[i] = r < r1 && pr.st[r].phase == PH_INNER;
      const size_t off = (size_t)(r < r1 ? r : r0) * K * N;
      pb[i] = Slab<T>((const T*)pr.p + off, K, N).rs;
      rb[i] = Slab<T>((const T*)pr.r + off, K, N).rs;
      qb[i] = Slab<T>((T*)pr.q + off, K, N).rs;
    }
    // direction p of right-hand side i, regressor k, voxel m
    auto pval = [&](int i, int k, int m) -> T { return bload<T>(pb[i], (unsigned)m * sizeof(T), (unsigned)k * row); };
    auto cell = [&](int xx, int yy, int zz) -> int {
      return (xx >= 0 && xx < nx && yy >= 0 && yy < ny && zz >= 0 && zz < nz) ? gm[((size_t)zz * ny + yy) * nx + xx]
                                                                              : -1;
    };
    const int x0 = w.xt * ZFX, y0 = w.yt * ZFY;
    const int zs = w.seg * pr.zs, ze = min(nz, zs + pr.zs);
    const int x = x0 + lane, y = y0 + ty;
    int n_prv = cell(x, y, zs - 1), n_cur = cell(x, y, zs);
    T v_prv[RC][K], v_cur[RC][K];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        v_prv[i][k] = (act[i] && n_prv >= 0) ? pval(i, k, n_prv) : (T)0;
        v_cur[i][k] = (act[i] && n_cur >= 0) ? pval(i, k, n_cur) : (T)0;
      }
    }
    double acc[RC][NPART];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
#pragma unroll
      for (int v = 0; v < NPART; ++v) acc[i][v] = 0.0;
    }
#pragma unroll 1
    for (int z = zs; z < ze; ++z) {
      // prefetch the own voxel one slice up (the +z neighbour of this step)
      const int n_nxt = cell(x, y, z + 1);
      T v_nxt[RC][K];
#pragma unroll
      for (int i = 0; i < RC; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k) v_nxt[i][k] = (act[i] && n_nxt >= 0) ? pval(i, k, n_nxt) : (T)0;
      }
      // the slice with a one-cell halo into LDS
      s_n[ty + 1][lane + 1] = n_cur;
#pragma unroll
      for (int i = 0; i < RC; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k) s_p[i * K + k][ty + 1][lane + 1] = v_cur[i][k];
      }
      auto halo = [&](int row, int col, int xx, int yy) {
        const int m = cell(xx, yy, z);
        s_n[row][col] = m;
        if (m >= 0) {
#pragma unroll
          for (int i = 0; i < RC; ++i) {
#pragma unroll
            for (int k = 0; k < K; ++k) s_p[i * K + k][row][col] = act[i] ? pval(i, k, m) : (T)0;
          }
        }
      };
      if (ty == 0) halo(0, lane + 1, x, y0 - 1);
      if (ty == ZFY - 1) halo(ROWS - 1, lane + 1, x, y0 + ZFY);
      if (lane == 0) halo(ty + 1, 0, x0 - 1, y);
      if (lane == ZFX - 1) halo(ty + 1, COLS - 1, x0 + ZFX, y);
      lds_barrier();
      if (n_cur >= 0) {
        T B[NB];
        load_soa(Slab<T>(OpT<T>::B(op), NB, N), (unsigned)n_cur * sizeof(T), B);
        const int nb_n[4] = {s_n[ty + 1][lane], s_n[ty + 1][lane + 2], s_n[ty][lane + 1], s_n[ty + 2][lane + 1]};
        const unsigned o = (unsigned)n_cur * sizeof(T);
#pragma unroll
        for (int i = 0; i < RC; ++i) {
          if (!act[i]) continue;
          T qv[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int pl = i * K + k;
            const T c = v_cur[i][k];
            T s6 = 0;
            if (nb_n[0] >= 0) s6 += c - s_p[pl][ty + 1][lane];
            if (nb_n[1] >= 0) s6 += c - s_p[pl][ty + 1][lane + 2];
            if (nb_n[2] >= 0) s6 += c - s_p[pl][ty][lane + 1];
            if (nb_n[3] >= 0) s6 += c - s_p[pl][ty + 2][lane + 1];
            if (zc && n_prv >= 0) s6 += c - v_prv[i][k];
            if (zc && n_nxt >= 0) s6 += c - v_nxt[i][k];
            qv[k] = OpT<T>::alpha(op, k) * s6;
          }
#pragma unroll
          for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < K; ++j) qv[k] += B[pk(k, j)] * v_cur[i][j];
          }
          T rv[K];
#pragma unroll
          for (int k = 0; k < K; ++k) rv[k] = bload<T>(rb[i], o, (unsigned)k * row);
          T rPr, qPr, qPq;
          precond_forms<T, PC, K>(Slab<T>(OpT<T>::P(op), PSize<PC, K>::n, N), o, rv, qv, rPr, qPr, qPq);
          T spq = 0, srr = 0, sqr = 0, sqq = 0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            bstore(qb[i], o, (unsigned)k * row, qv[k]);
            spq += v_cur[i][k] * qv[k];
            srr += rv[k] * rv[k];
            sqr += qv[k] * rv[k];
            sqq += qv[k] * qv[k];
          }
          acc[i][0] += spq;
          acc[i][1] += rPr;
          acc[i][2] += qPr;
          acc[i][3] += qPq;
          acc[i][4] += srr;
          acc[i][5] += sqr;
          acc[i][6] += sqq;
        }
      }
      lds_barrier();
      n_prv = n_cur;
      n_cur = n_nxt;
#pragma unroll
      for (int i = 0; i < RC; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          v_prv[i][k] = v_cur[i][k];
          v_cur[i][k] = v_nxt[i][k];
        }
      }
    }
    // per right-hand side: the values summed over each wavefront, then the rows in order
#pragma unroll
    for (int i = 0; i < RC; ++i) wave_deposit<NPART>(&s_red[0][0], i, acc[i]);
    __syncthreads();
    if (threadIdx.x < RC * NPART) {
      const int i = threadIdx.x / NPART, v = threadIdx.x % NPART, r = r0 + i;
      if (r < r1 && act[i]) {
        double t = 0.0;
        for (int j = 0; j < ZFY; ++j) t += s_red[i * NPART + v][j];
        pr.part[((size_t)v * pr.R + r) * pr.pstride + w.tile] = t;
      }
    }
    __syncthreads();
  }
}

}  // namespace gp
