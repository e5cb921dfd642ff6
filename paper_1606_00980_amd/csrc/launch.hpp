// Host-side launch entry points of the kernels (one definition per source file).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace gp {

// Per-launch timing while profiling: the launches made between prof_begin
// and prof_end carry the pair of events in their dispatch packets
// (hipExtLaunchKernelGGL), the first launch's start and the last one's stop,
// so that the elapsed time is the kernels' own, without the dispatch of the
// packets.  Outside such a span `stop` is null and launches are plain.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  bool first = true;   // no launch has taken the start event yet
};
LaunchTiming& launch_timing();

#define GP_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                        \
  do {                                                                                            \
    ::gp::LaunchTiming& lt_ = ::gp::launch_timing();                                              \
    if (lt_.stop) {                                                                               \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, lt_.first ? lt_.start : nullptr,  \
                            lt_.stop, 0, __VA_ARGS__);                                            \
      lt_.first = false;                                                                          \
    } else {                                                                                      \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                        \
    }                                                                                             \
  } while (0)

// k_ops.hip
hipError_t launch_grid_build(hipStream_t s, const uint8_t* mask, long ncell, int* counts, int* offsets,
                             int nblocks);
hipError_t launch_grid_index(hipStream_t s, const uint8_t* mask, long ncell, const int* offsets,
                             int nblocks, int* gridmap, int* lin, int N, int nx, int ny, int nz, int conn,
                             int* nbr, unsigned long long* edges);
int grid_cells_per_block();
hipError_t launch_pack_blocks(hipStream_t s, int K, int N, const double* B, double* B64, float* B32,
                              double* L64, int* bad);
hipError_t launch_precond(hipStream_t s, const OpDev& op, int pc, double* P64, float* P32, int* bad);
hipError_t launch_apply(hipStream_t s, const OpDev& op, int R, const double* x, double* y);
hipError_t launch_perturb(hipStream_t s, const OpDev& op, int R, const double* bw, const double* z1,
                          const double* z2, double* b);
hipError_t launch_probe_rhs(hipStream_t s, long total, const int8_t* v, double* b);
hipError_t launch_add_broadcast(hipStream_t s, int R, long kn, const double* bw, double* b);
hipError_t launch_trace(hipStream_t s, const OpDev& op, int m, const int8_t* v, const double* u,
                        double* part, double* pairbuf, double* out);

// Finalising launch after a refine (kind 0) or matvec (1) launch:
// nblocks = sum over problems of ceil(R / finalize_rhs_per_block()).
hipError_t launch_finalize(hipStream_t s, int kind, const Prob* probs, int nprob, int nblocks);
int finalize_rhs_per_block();

// k_data.hip: time-summed AR(P) data tensors and the data term assembled from them
hipError_t launch_data_tensors(hipStream_t s, int T, int K, int P, int N, const double* X, const double* Y,
                               double* G, double* YX, double* Bt, double* Dt, double* YY, double* dY, double* dd);
hipError_t launch_data_rss(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* YX,
                           const double* Bt, const double* Dt, const double* YY, const double* dY, const double* dd,
                           const double* W, const double* A, double u1, double u2t, double* rss, double* scale,
                           double* mean);
// W_k D_w W_k' for R samples: partials [R*K][quadform_tiles(N)], out [R*K] (device)
int quadform_tiles(int N);
hipError_t launch_quadform(hipStream_t s, const OpDev& op, int R, const double* W, double* part, double* out);
// J_n [N][P][P] (both triangles) and b_a [P][N] (may be null) of the AR-coefficient system
hipError_t launch_data_assemble_ar(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* Bt,
                                   const double* Dt, const double* dY, const double* dd, const double* lambda,
                                   const double* W, double* Jout, double* ba);
hipError_t launch_data_assemble(hipStream_t s, int K, int P, int N, int Ns, const double* G, const double* YX,
                                const double* Bt, const double* Dt, const double* lambda, const double* A,
                                double* Bout, double* bw);

// k_rng.hip: Philox4x32-10 normals, Rademacher signs and raw words
hipError_t launch_rng_normal(hipStream_t s, uint64_t seed, uint64_t stream, size_t n, double* out);
hipError_t launch_rng_rademacher(hipStream_t s, uint64_t seed, uint64_t stream, size_t n, int8_t* out);
// out[e] = scale[e] (or 1) * Gamma(shape, 1), Marsaglia-Tsang on the Philox streams
hipError_t launch_rng_gamma(hipStream_t s, uint64_t seed, uint64_t stream, size_t n, double shape,
                            const double* scale, double* out);
hipError_t launch_rng_raw(hipStream_t s, uint64_t seed, uint64_t stream, size_t nblocks, uint32_t* out);

// k_pcg_f64.hip / k_pcg_f32.hip: grouped launches over `nprob` problems that
// all have K regressors; W = total work items (tiles x right-hand-side chunks),
// swept by nblk persistent workgroups (a multiple of 8, one XCD range each);
// pc = PC_JACOBI or PC_BLOCK.
hipError_t launch_refine_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_matvec_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_matvec_zm_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_update_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_addsol_f64(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_refine_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_matvec_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_matvec_zm_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_update_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk);
hipError_t launch_addsol_f32(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk);
// right-hand sides per z-marching workgroup for K regressors
int zm_rhs_per_block(int K);

// k_rbic_f32.hip / k_rbic_f64.hip: red-black incomplete Cholesky.  Vectors of
// the black system are [R][K][NB], red ones [R][K][NR].  Set-up, split and
// recovery take one operator's descriptor by value; the solver-round launches
// are grouped over several operators and read their descriptors from device
// memory, so that rounds can be replayed as graphs while alpha or buffers
// change.
hipError_t launch_rb_setup(hipStream_t s, const RbDev& rb, const double* B64, double* P64, float* P32,
                           double* D64, float* D32, double* S64, float* S32, int* bad);
// With r set (a zero start value), the split also takes the first refinement:
// r = c, p = S_m^{-1} r in the inner precision (f32: float vectors, else
// double), and its partials at right-hand side r0 + i of the solve.
struct RbSplitFirst {
  void* r;
  void* p;
  double* part;
  size_t vstride;
  int pstride, r0;
  bool f32;
};
hipError_t launch_rb_split(hipStream_t s, const RbDev& rb, int R, const double* b, const double* x, int zero_guess,
                           double* t, double* c, double* xB, double* bbpart, const RbSplitFirst& first);
// Grouped solver-round launches over the nprob members of one K group (device
// descriptors probs, every member with K regressors); W = the launch's work
// items: black-tile items (tiles x chunks of Rc right-hand sides) for matvec
// and update, red-tile items for the red stages, black-tile items
// of one right-hand side for refine and addsol.  T is the inner precision.
template <typename T> hipError_t launch_rbg_red(hipStream_t s, int K, const RbProb* probs, int nprob, int W);
// pairs: some member stores the red-stage vector in right-hand-side pairs
template <typename T>
hipError_t launch_rbg_matvec(hipStream_t s, int K, const RbProb* probs, int nprob, int W, bool pairs);
template <typename T> hipError_t launch_rbg_update(hipStream_t s, int K, const RbProb* probs, int nprob, int W);
template <typename T> hipError_t launch_rbg_refine(hipStream_t s, int K, const RbProb* probs, int nprob, int W);
template <typename T> hipError_t launch_rbg_addsol(hipStream_t s, int K, const RbProb* probs, int nprob, int W);
#define GP_RBG_DECL(T)                                                                                       \
  template <> hipError_t launch_rbg_red<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W);        \
  template <> hipError_t launch_rbg_matvec<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W,      \
                                              bool pairs);                                                    \
  template <> hipError_t launch_rbg_update<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W);     \
  template <> hipError_t launch_rbg_refine<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W);     \
  template <> hipError_t launch_rbg_addsol<T>(hipStream_t s, int K, const RbProb* probs, int nprob, int W);
GP_RBG_DECL(float)
GP_RBG_DECL(double)
#undef GP_RBG_DECL
// the FP64 red stage of the refinement (u64 from x_B), red-tile items
hipError_t launch_rbg_red64(hipStream_t s, int K, const RbProb* probs, int nprob, int W);
// finalisation after refine (kind 0) or the black stage (1): nblocks =
// sum over members of ceil(R / 4)
hipError_t launch_rbg_finalize(hipStream_t s, int kind, const RbProb* probs, int nprob, int nblocks);
hipError_t launch_rb_recover(hipStream_t s, const RbDev& rb, int R, const RhsState* st, const double* t,
                             const double* u64, const double* xB, double* x);

}  // namespace gp
