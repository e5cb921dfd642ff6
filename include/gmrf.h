/*
 * gmrf.h -- C ABI of the MI355X GMRF posterior-precision library.
 *
 * The library solves, samples from and estimates traces of the Gaussian
 * Markov random field posterior of the spatial GLM for fMRI of Siden, Eklund,
 * Bolin and Villani (Fast Bayesian whole-brain fMRI analysis with spatial 3D
 * priors):
 *
 *   w_r = vec(W') ~ N(Q^{-1} b, Q^{-1}),
 *   Q   = diag(alpha) (x) D_w  +  H' blkdiag_n(B_n) H           (Section 3,
 *         full conditional of w_r; Appendix A.2 for the AR(P) data term)
 *
 * where D_w = G_w'G_w is the unweighted graph Laplacian of a 3D (6-neighbour)
 * or 2D (4-neighbour) voxel mask (Section 2 and Section 3.1), B_n is the SPD
 * K x K data block of voxel n and H is the permutation between voxel-major
 * and k-major ordering.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: every function returns GP_OK (0) or a negative GP_ERR_* code.
 *    gp_last_error() returns a message for the calling thread's last failure.
 *    No C++ exception crosses this boundary.
 *  - Memory: pointers documented as "device" are HIP device pointers on the
 *    context's device; "host" pointers are ordinary host memory.  The caller
 *    owns every buffer it passes; the library never frees caller memory.  The
 *    library owns operator data and solver workspace, charged to the
 *    context's HBM budget.
 *  - Ordering: work is issued on the context's HIP stream.  Functions that
 *    return statistics or host results block until that work has completed;
 *    the others are stream-ordered and return after enqueueing.
 *  - Voxels: in-mask voxels are numbered n = 0..N-1 in increasing linear index
 *    l = x + nx*(y + ny*z) (x fastest).
 *  - Vectors: a batch of R vectors is contiguous FP64 laid out [R][K][N]; each
 *    [K][N] slab is the paper's k-major w_r = vec(W') (Section 3).
 *  - Data blocks: FP64 [N][K][K], row-major, symmetric (the two triangles are
 *    averaged).
 *  - Threads: one context must not be used by two threads at once; calls that
 *    overlap on one context return GP_ERR_BUSY.
 */
#ifndef GMRF_H
#define GMRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GP_OK                 0
#define GP_ERR_INVALID_ARG   -1  /* bad size, pointer, enum, or state        */
#define GP_ERR_NOT_SPD       -2  /* a K x K block is not positive definite    */
#define GP_ERR_OOM           -3  /* HBM budget or device allocation exceeded  */
#define GP_ERR_BUSY          -4  /* the context is in use by another call     */
#define GP_ERR_NOT_CONVERGED -5  /* iteration cap reached before tolerance    */
#define GP_ERR_BREAKDOWN     -6  /* non-finite value or loss of definiteness  */
#define GP_ERR_DEVICE        -7  /* a HIP runtime call failed                 */
#define GP_ERR_TIMEOUT       -8  /* a served request passed its deadline      */
#define GP_ERR_CANCELLED     -9  /* a served request was cancelled            */

/* Largest number of regressors K of an operator (and of the per-regressor
 * arrays of gp_result).                                                      */
#define GP_KMAX 24

/* ---- preconditioners and precision modes ----------------------------- */
#define GP_PRECOND_JACOBI        0  /* inverse of diag(Q)                      */
#define GP_PRECOND_BLOCK_JACOBI  1  /* inverse of each voxel's K x K block of Q */
/* Incomplete Cholesky factor of Q with zero fill in K x K voxel blocks, on the
 * two-colour voxel order (even x + y + z first) -- the preconditioner M of
 * Algorithm 2 (steps 6-7) and Section 3.1, with the red-black order in place
 * of a fill-reducing one.  PCG with it is carried out as the equivalent
 * half-size PCG on the Schur complement of the odd voxels with its diagonal
 * blocks as preconditioner; the even voxels are solved exactly from their rows
 * (start values included), so the reported residual is that of the whole
 * system.  Needs R <= 65535 per operator and call.                        */
#define GP_PRECOND_RB_IC0        2

#define GP_MATVEC_AUTO    0  /* the tuned choice, else the raster kernel        */
#define GP_MATVEC_RASTER  1  /* one voxel per thread, neighbours via an index table */
#define GP_MATVEC_ZMARCH  2  /* (x, y) footprints walking z, slices in LDS      */

#define GP_PREC_FP64          0  /* every step in FP64                          */
#define GP_PREC_FP32_REFINE64 1  /* FP32 inner PCG, FP64 residual/update/test   */

typedef struct gp_ctx gp_ctx;
typedef struct gp_op gp_op;
typedef struct gp_data gp_data;

/* Solver options.  Initialise with gp_opts_default(). */
typedef struct gp_opts {
  double   tol;        /* stop when ||b - Q x||_2 / ||b||_2 <= tol, per right-hand
                          side, with the residual recomputed in FP64 (Section
                          3.1, PCG tolerance delta).  Default 1e-8.             */
  double   inner_tol;  /* FP32 mode: each inner solve reduces its residual by
                          this factor before the next FP64 refinement step.
                          Default 1e-4.  Ignored in FP64 mode.                  */
  int      max_iter;   /* cap on PCG iterations summed over refinement steps
                          (default 2000)                                        */
  int      max_outer;  /* cap on FP64 residual evaluations (default 30)         */
  int      precond;    /* GP_PRECOND_*; default GP_PRECOND_BLOCK_JACOBI          */
  int      precision;  /* GP_PREC_*; default GP_PREC_FP32_REFINE64              */
  int      rhs_tile;   /* right-hand sides per workgroup, 0 = automatic          */
  int      chunk;      /* PCG iterations enqueued between host checks, 0 = auto  */
  int      wg_per_cu;  /* persistent workgroups per compute unit, 0 = auto       */
  int      matvec;     /* GP_MATVEC_*: inner matvec kernel, 0 = automatic        */
  int      zero_guess; /* 1: the start value is zero -- x is not read on entry
                          (only written), which saves a pass over it; 0: x holds
                          the start value (default)                              */
  uint64_t seed;       /* Philox key used when gp_sample / gp_trace are given no
                          random vectors (see gp_rng_normal)                     */
} gp_opts;

/* Per right-hand-side result. */
typedef struct gp_stats {
  int    status;       /* GP_OK, GP_ERR_NOT_CONVERGED or GP_ERR_BREAKDOWN        */
  int    inner_iters;  /* PCG iterations (all refinement steps)                  */
  int    outer_steps;  /* FP64 residual evaluations                              */
  int    reserved;
  double relres;       /* final FP64 ||b - Q x|| / ||b|| (0 when b = 0)          */
  double time_us;      /* wall time of the whole call, microseconds              */
} gp_stats;

/* One solve in a batch: R right-hand sides of one operator. */
typedef struct gp_item {
  gp_op*        op;
  int           R;
  const double* b;     /* device, [R][K][N]                                     */
  double*       x;     /* device, [R][K][N]; in: start value, out: solution      */
} gp_item;

/* Kernel kinds reported by the profiler. */
#define GP_KERNEL_REFINE   0  /* FP64 residual + preconditioned restart        */
#define GP_KERNEL_MATVEC   1  /* direction update and q = Q p                  */
#define GP_KERNEL_UPDATE   2  /* solution/residual update, preconditioner      */
#define GP_KERNEL_ADDSOL   3  /* FP64 solution += inner correction             */
#define GP_KERNEL_PERTURB  4  /* Algorithm 2 right-hand sides                  */
#define GP_KERNEL_PRECOND  5  /* preconditioner set-up                         */
#define GP_KERNEL_PACK     6  /* data-block ingest and Cholesky                */
#define GP_KERNEL_PROBE    7  /* probe -> FP64 right-hand side                 */
#define GP_KERNEL_TRACE    8  /* Hutchinson reductions                         */
#define GP_KERNEL_APPLY    9  /* FP64 y = Q x                                  */
#define GP_KERNEL_DATA    10  /* data tensors and data-term assembly          */
/* red-black incomplete Cholesky solver (GP_PRECOND_RB_IC0)                   */
#define GP_KERNEL_RB_RED     11  /* even-voxel stage u = Q_nn^{-1}(alpha .* sum v) of an inner step */
#define GP_KERNEL_RB_MATVEC  12  /* odd-voxel stage q = S p, inner products    */
#define GP_KERNEL_RB_UPDATE  13  /* d, r, p update on the odd voxels           */
#define GP_KERNEL_RB_REFINE  14  /* FP64 residual of the Schur system          */
#define GP_KERNEL_RB_ADDSOL  15  /* FP64 odd-voxel solution += correction      */
#define GP_KERNEL_RB_EDGE    16  /* split of b and x, recovery of the solution */
#define GP_KERNEL_RB_RED64   17  /* even-voxel stage of the FP64 refinement     */
#define GP_KERNEL_KINDS   18

/* Accumulated per kernel kind while profiling is enabled.  `units` counts
 * (right-hand side, voxel) pairs processed; `bytes` is the algorithmic HBM
 * traffic of those launches (each vector, block and factor entry moved once;
 * neighbour re-reads and index tables excluded); `ms` is the sum of the
 * launches' durations measured with HIP events on the context's stream.    */
typedef struct gp_prof {
  int64_t launches;
  int64_t units;
  double  ms;
  double  bytes;
} gp_prof;

void        gp_opts_default(gp_opts* opts);
const char* gp_last_error(void);
int         gp_version(void);

/* ---- context ----------------------------------------------------------
 * gp_ctx_create: bind to HIP device `device`, issue work on `hip_stream`
 * (a hipStream_t; NULL selects the device's null stream) and cap the bytes
 * the library may allocate at `hbm_budget` (0 = no cap).                    */
int gp_ctx_create(int device, void* hip_stream, size_t hbm_budget, gp_ctx** out);
int gp_ctx_set_stream(gp_ctx* ctx, void* hip_stream);
/* bytes currently allocated by the library for this context (host out)     */
int gp_ctx_memory(const gp_ctx* ctx, size_t* used, size_t* budget);
int gp_ctx_destroy(gp_ctx* ctx);
/* gp_ctx_profile: enable (1) or disable (0) per-launch event timing on this
 * context; enabling clears the accumulated figures.  While it is on, rounds
 * run eagerly (no graph replay) and each launch's kernels carry a pair of
 * HIP events in their dispatch packets, so a launch's time is its kernels'
 * time.  gp_ctx_profile_read synchronises the stream and copies the figures
 * of one GP_KERNEL_* kind into *out (host).                                  */
int gp_ctx_profile(gp_ctx* ctx, int enable);
int gp_ctx_profile_read(gp_ctx* ctx, int kind, gp_prof* out);

/* ---- operator ----------------------------------------------------------
 * gp_op_create: build the masked-grid operator (Section 2: the unweighted
 * graph Laplacian over in-mask neighbours, free boundary; Section 3.1: one
 * incidence row per adjacent pair).  mask_host: host, nx*ny*nz bytes, nonzero
 * = in mask, linear index l = x + nx*(y + ny*z).  conn: 6 (3D) or 4 (2D, then
 * nz must be 1).  K: regressors, 1..24.  Rejects an empty mask.  The
 * operator is unusable until gp_op_set_blocks and gp_op_set_alpha succeed.  */
int gp_op_create(gp_ctx* ctx, const uint8_t* mask_host, int nx, int ny, int nz,
                 int conn, int K, gp_op** out);

/* gp_op_set_blocks: ingest the data blocks B_n (device, FP64 [N][K][K]; the
 * X'X (x) diag(lambda) term of Section 3, or the AR(P) blocks of Appendix
 * A.2) and factor each as B_n = L_n L_n' (the L_data of Algorithm 2).
 * Returns GP_ERR_NOT_SPD if some block is not positive definite; then
 * *bad_voxel_host (if non-NULL) receives the smallest failing voxel.
 * Marks the preconditioner stale; the next solve rebuilds it.              */
int gp_op_set_blocks(gp_op* op, const double* B, int64_t* bad_voxel_host);

/* ---- data term on the device (Appendix A.2, Appendix B) ------------------
 * gp_data_create: precompute, once per dataset, the time-summed data of the
 * AR(P) likelihood conditional on the first P scans (Appendix A.2, the tensors
 * it isolates from the Gibbs loop): globally X'X, R = X'X~ and S = X~X~, per
 * voxel Y_n'X, B~_n = Y_n'X~ + d_n X and D_n = d_n X~, where X~ is the lagged
 * design (lag p+1 in slot p) and d_n the lagged data.  X_host: host, T x K
 * row-major, the design of the operator's K regressors.  Y: device, FP64
 * [T][N], the data of the operator's voxels in its voxel order.  Requires
 * 0 <= P <= 4, T > P and T*K <= 8192.  The tensors live on the device under
 * the context's budget until gp_data_destroy.  Blocking.                  */
int gp_data_create(gp_op* op, int T, int P, const double* X_host, const double* Y, gp_data** out);

/* gp_data_assemble: the data term from the tensors, for noise precisions
 * lambda (device, N) and Ns >= 1 draws of the AR coefficients A (device,
 * [Ns][P][N]; NULL when P = 0):
 *   B_n = lambda_n (X'X - mean_j [R a + (R a)' - a' S a]),
 *   b_n = lambda_n (Y_n'X - mean_j [a' B~_n - a' D_n a]),   a = A[j][.][n]
 * -- the full conditional of W for Ns = 1 (Appendix A.2) and its SVB
 * expectation over Monte Carlo draws for Ns > 1 (Appendix B).  The blocks
 * are installed in the operator as gp_op_set_blocks does (factorised,
 * GP_ERR_NOT_SPD with *bad_voxel_host on failure); b_n is written to bw
 * (device, FP64 [K][N], the k-major b_w; may be NULL).  Blocking.          */
int gp_data_assemble(gp_data* d, const double* lambda, int Ns, const double* A, double* bw,
                     int64_t* bad_voxel_host);

/* gp_data_lambda: the noise-precision posterior (Appendix A.2, full
 * conditional of lambda; Appendix B for its SVB form): per voxel, the mean
 * over Ns pairs (W^j, A^j) of the whitened residual sum of squares
 *   rss_n = Y'Y - 2Y'XW + W'X'XW - 2Y'd'A + A'dd'A + 2A'B~W - 2W'(RA)W
 *           - 2A'(DW)A + W'(A'SA)W        (W = W^j_{.,n}, A = A^j_{.,n}),
 * then lambda_n ~ Ga(scale u1t_n, shape u2t) with 1/u1t_n = rss_n/2 + 1/u1 and
 * u2t = (T-P)/2 + u2; mean = u1t_n * u2t.  W: device [Ns][K][N] (the k-major
 * samples); A: device [Ns][P][N] (NULL when P = 0).  Outputs (device, N
 * doubles each, any may be NULL): rss, scale, mean.  Blocking.            */
int gp_data_lambda(gp_data* d, int Ns, const double* W, const double* A, double u1, double u2, double* rss,
                   double* scale, double* mean);

/* gp_data_assemble_ar: the system of the AR coefficients (Appendix A.2, full
 * conditional of A; Appendix B for its SVB expectation over Ns >= 1 draws of
 * W), for noise precisions lambda (device, N) and draws W (device,
 * [Ns][K][N]):
 *   J_n  = lambda_n mean_j [d_n d_n' - D_n w - (D_n w)' + w' S w],
 *   b_an = lambda_n mean_j [Y_n'd_n' - w' B~_n' + w' R w],        w = W[j][.][n],
 * with (D_n w)[p][q] = sum_k D_n[p][k][q] w_k, (w'Sw)[p][q] =
 * sum_kl w_k S[p][k][l][q] w_l, (w'B~')[p] = sum_k B~_n[p][k] w_k and
 * (w'Rw)[p] = sum_kl w_k R[k][l][p] w_l.  The P x P blocks J_n are installed
 * in op_a as gp_op_set_blocks does (factorised, GP_ERR_NOT_SPD with
 * *bad_voxel_host on failure): op_a is an operator with K = P built on the
 * same mask as the data's operator (same nx, ny, nz and N), whose alpha plays
 * the prior precisions beta of A, so that op_a is
 *   J~ = diag(beta) (x) D_a + H_a' blkdiag_n(J_n) H_a   with D_a = D_w,
 * and every solver, sampler and trace entry point applies to it.  b_a is
 * written to ba (device [P][N], the p-major vec(A'); may be NULL).  Requires
 * P >= 1.  Blocking.                                                        */
int gp_data_assemble_ar(gp_data* d, gp_op* op_a, const double* lambda, int Ns, const double* W, double* ba,
                        int64_t* bad_voxel_host);
int gp_data_destroy(gp_data* d);

/* Gamma prior parameters of alpha_k ~ Ga(q1, q2), lambda_n ~ Ga(u1, u2) and
 * of the AR-coefficient precisions beta_p ~ Ga(r1, r2) (scale, shape;
 * Section 2).  gp_hyper_default: the values the paper uses, q1 = u1 = 10,
 * r1 = 10000, q2 = u2 = r2 = 0.1.                                          */
typedef struct gp_hyper {
  double q1, q2, u1, u2, r1, r2;
} gp_hyper;
void gp_hyper_default(gp_hyper* h);

/* gp_svb_step: one iteration of the spatial VB scheme for W, alpha and lambda
 * with the AR coefficients held at Ns given draws (Section 3.3, Appendix B):
 *   1. the data term with the current mean noise precisions lambda (device N)
 *      and the draws A (device [Ns][P][N], NULL when P = 0), into the operator
 *      and bw_work (device [K][N]);
 *   2. alpha_host (K) as the spatial precisions;
 *   3. Ns samples of q(W) by Algorithm 2 into W (device [Ns][K][N]), which
 *      holds the previous samples as warm starts; z1, z2 as in gp_sample (the
 *      same vectors every iteration, or NULL for device draws from
 *      opts->seed, which repeat when the seed does);
 *   4. alpha_host <- the posterior means of gp_alpha_posterior over the Ns
 *      samples; lambda <- the posterior means of gp_data_lambda over the Ns
 *      pairs (W^j, A^j).
 * prior: NULL for gp_hyper_default.  stats: Ns entries of the sampling
 * solves.  Blocking.                                                          */
int gp_svb_step(gp_data* d, int Ns, const double* A, const double* z1, const double* z2, double* W,
                double* lambda, double* alpha_host, const gp_hyper* prior, double* bw_work,
                const gp_opts* opts, gp_stats* stats);

/* gp_svb_step_ar: one iteration of the spatial VB scheme over W, the AR
 * coefficients A and the precisions alpha, beta, lambda (Section 3.3,
 * Appendix B), in the order:
 *   1. q(W) as steps 1-3 of gp_svb_step, with the draws A (device [Ns][P][N])
 *      and alpha_host (K), samples into W (device [Ns][K][N], warm starts),
 *      random vectors z1w, z2w;
 *   2. q(A): gp_data_assemble_ar with lambda and the new W into op_a and
 *      ba_work (device [P][N]), beta_host (P) as op_a's spatial precisions,
 *      Ns samples by Algorithm 2 into A (warm starts), random vectors z1a
 *      ([Ns][P][dirs][N]), z2a ([Ns][P][N]);
 *   3. alpha_host <- gp_alpha_posterior means over W (q1, q2); beta_host <-
 *      gp_alpha_posterior means over A on op_a (r1, r2); lambda <- the
 *      gp_data_lambda means over the pairs (W^j, A^j) (u1, u2).
 * z1w, z2w, z1a, z2a: all given or all NULL (device draws: W's from
 * opts->seed as in gp_sample, A's from that seed XOR 0x9E3779B97F4A7C15).
 * prior: NULL for gp_hyper_default.  stats_w, stats_a: Ns entries each (may
 * be NULL).  Requires P >= 1.  Blocking.                                    */
int gp_svb_step_ar(gp_data* d, gp_op* op_a, int Ns, const double* z1w, const double* z2w, double* W,
                   const double* z1a, const double* z2a, double* A, double* lambda, double* alpha_host,
                   double* beta_host, const gp_hyper* prior, double* bw_work, double* ba_work,
                   const gp_opts* opts, gp_stats* stats_w, gp_stats* stats_a);

/* gp_gibbs_step: one iteration of the Gibbs sampler of Section 3.2 for W,
 * alpha and lambda, with the AR coefficients held at A (device [P][N], NULL
 * when P = 0):
 *   1. the data term with lambda (device N) and A into the operator and
 *      bw_work (device [K][N]); alpha_host (K) as the spatial precisions;
 *   2. one draw of W from its full conditional by Algorithm 2 into W (device
 *      [K][N], which holds the previous draw as the start value), with the
 *      random vectors z1, z2 (as in gp_sample) or, when both are NULL, drawn
 *      on the device from seed ^ (iteration * 0x9E3779B97F4A7C15);
 *   3. alpha_k ~ Ga(scale_k, N/2 + q2), 1/scale_k = W_k D_w W_k'/2 + 1/q1, by
 *      gp_rng_gamma(seed, stream 16 + 2 iteration) into alpha_host;
 *   4. lambda_n ~ Ga(scale_n, (T-P)/2 + u2), 1/scale_n = rss_n/2 + 1/u1 (the
 *      whitened residual sum of squares of the new W and A), by
 *      gp_rng_gamma(seed, stream 17 + 2 iteration) into lambda.
 * prior: NULL for gp_hyper_default.  stats: one entry.  Blocking.           */
int gp_gibbs_step(gp_data* d, const double* A, const double* z1, const double* z2, double* W, double* lambda,
                  double* alpha_host, const gp_hyper* prior, double* bw_work, uint64_t seed, uint64_t iteration,
                  const gp_opts* opts, gp_stats* stats);

/* gp_alpha_extrapolate: the first convergence device of the SVB implementation
 * (Appendix C): from the posterior means of the last three iterations, a_jm2,
 * a_jm1 and a_j (host, K each; a_j as the update equation proposed it), put
 * the quadratic in the iteration number through them; if its vertex lies
 * after iteration j, the prediction is its value there, otherwise
 * a_jm1 + 20 (a_j - a_jm1); a_j is replaced by the prediction limited to
 * [a_j / 5, 5 a_j].  Meant for every other SVB iteration; applies alike to
 * beta.  Host only (no device work).                                        */
int gp_alpha_extrapolate(int K, const double* a_jm2, const double* a_jm1, double* a_j);

/* gp_alpha_posterior: the spatial-precision posterior (Section 3.2 full
 * conditional; Section 3.3 and Appendix B for the SVB Monte Carlo form):
 * qf[r][k] = W_k D_w W_k' = ||G_w W_k'||^2 of each of R samples W (device,
 * [R][K][N]), then alpha_k ~ Ga(scale_k, shape) with
 * 1/scale_k = mean_r qf[r][k] / 2 + 1/q1 and shape = N/2 + q2; mean_k =
 * scale_k * shape.  Outputs on the host: qf (R*K, may be NULL), scale (K),
 * mean (K).  On an AR-coefficient operator (K = P, see gp_data_assemble_ar)
 * with samples of A and (r1, r2) it is the posterior of beta (Appendix A.2,
 * full conditional of beta), which has the same form.  Blocking.            */
int gp_alpha_posterior(gp_op* op, int R, const double* W, double q1, double q2, double* qf_host,
                       double* scale_host, double* mean_host);

/* gp_op_set_alpha: spatial precisions alpha_k >= 0 (host, K doubles; the
 * prior precision of regressor k, Section 2).  Marks the preconditioner (the
 * K x K voxel blocks B_n + diag(alpha_k deg_n) and their inverses) stale; the
 * next solve rebuilds it, and reports GP_ERR_NOT_SPD if a block fails.       */
int gp_op_set_alpha(gp_op* op, const double* alpha_host);

/* gp_op_query: any out pointer may be NULL.  N voxels, E adjacent pairs
 * (rows of G_w), K, and device bytes held by the operator.                  */
int gp_op_query(const gp_op* op, int64_t* N, int64_t* E, int* K, size_t* bytes);

/* gp_op_voxel_index: device int32 [N] receives the linear index of voxel n. */
int gp_op_voxel_index(const gp_op* op, int32_t* lin);
int gp_op_destroy(gp_op* op);

/* ---- operations -------------------------------------------------------- */

/* gp_apply: y = Q x in FP64 for R vectors (device [R][K][N] each); the
 * product of Section 3's precision with a vector.  Stream-ordered.          */
int gp_apply(gp_op* op, int R, const double* x, double* y);

/* gp_solve: x = Q^{-1} b for R right-hand sides by preconditioned conjugate
 * gradients (Section 3.1), stopping each right-hand side when its FP64
 * relative residual is <= opts->tol.  b: device [R][K][N]; x: device
 * [R][K][N], read as the start value (the warm start of Section 3.1) and
 * overwritten with the solution.  A zero b gives x = 0 after no iterations.
 * stats: host array of R entries (may be NULL).  Returns GP_OK when every
 * right-hand side converged, else the first failing status.  Blocking.     */
int gp_solve(gp_op* op, int R, const double* b, double* x, const gp_opts* opts,
             gp_stats* stats);

/* gp_solve_batch: the solves of n items (uneven operators and R) advanced
 * together, one grouped launch per kernel and step.  stats: host array of
 * sum(items[i].R) entries in item order (may be NULL).  Blocking.            */
int gp_solve_batch(gp_ctx* ctx, int n, const gp_item* items, const gp_opts* opts,
                   gp_stats* stats);

/* gp_perturb_rhs: Algorithm 2, step 4, for R draws:
 *   b_r = b_w + (blkdiag_k sqrt(alpha_k) G_w)' z1_r + H' L_data H z2_r.
 * bw: device [K][N] (shared by all draws); z1: device [R][K][dirs][N] with
 * dirs = 3 (3D: +x,+y,+z) or 2 (2D: +x,+y), slot (k,d,n) holding the entry of
 * the adjacent pair (n, n+e_d) -- slots whose n+e_d lies outside the mask are
 * ignored; z2: device [R][K][N]; b: device [R][K][N] output.  Stream-ordered. */
int gp_perturb_rhs(gp_op* op, int R, const double* bw, const double* z1,
                   const double* z2, double* b);

/* gp_sample: Algorithm 2 -- gp_perturb_rhs then gp_solve.  w: device
 * [R][K][N], in: start values, out: samples.  When z1 and z2 are both NULL
 * they are drawn on the device: z1 = gp_rng_normal(opts->seed, stream 1),
 * z2 = gp_rng_normal(opts->seed, stream 2), in the layouts above.  Blocking. */
int gp_sample(gp_op* op, int R, const double* bw, const double* z1, const double* z2,
              double* w, const gp_opts* opts, gp_stats* stats);

/* gp_probe_rhs: b_i = v_i as FP64 (device int8 [m][K][N] in {-1,+1} to device
 * FP64 [m][K][N]).  Stream-ordered.                                          */
int gp_probe_rhs(gp_op* op, int m, const int8_t* probes, double* b);

/* gp_trace_reduce: Hutchinson estimates from probes v_i and solutions
 * u_i = Q^{-1} v_i (device int8 [m][K][N], device FP64 [m][K][N]):
 *   tr_total = (1/m) sum_i v_i'u_i                ~ tr(Q^{-1})
 *   tr_kk[k] = (1/m) sum_i v_ik'u_ik              ~ tr([Q^{-1}]_kk)
 *   tr_Gkk[k]= (1/m) sum_i (D_w v_ik)'u_ik        ~ tr(D_w [Q^{-1}]_kk)
 * the last being the trace in E[W_k D_w W_k'] (Section 3.3).  Host outputs
 * (tr_kk, tr_Gkk: K doubles each; any may be NULL).  Blocking.               */
int gp_trace_reduce(gp_op* op, int m, const int8_t* probes, const double* u,
                    double* tr_total, double* tr_kk, double* tr_Gkk);

/* gp_trace_reduce_static: gp_trace_reduce for callers that cannot allocate
 * memory -- code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, same results (bitwise: the same
 * kernels in the same order), but the call makes no device or host
 * allocation: its device scratch (the per-tile partials, the per-probe sums
 * and the 1 + 2K totals) is a library-owned static device array of 16 MiB per
 * GPU, held until the process ends, and the results reach the host through a
 * pinned buffer the operator allocated at gp_op_create.  Requires
 * 2 m K ceil(N/256) + 2 m K + 49 <= 2097152 (doubles in 16 MiB), else
 * GP_ERR_INVALID_ARG with nothing launched.  Every call on one GPU uses that
 * GPU's one array (each call writes every value it reads, so nothing carries
 * over): calls that overlap on one GPU -- from two contexts, threads or
 * streams -- race and may return each other's values.  Blocking.          */
int gp_trace_reduce_static(gp_op* op, int m, const int8_t* probes, const double* u,
                           double* tr_total, double* tr_kk, double* tr_Gkk);

/* gp_trace: gp_probe_rhs, gp_solve from u = 0, gp_trace_reduce.  u: device
 * FP64 [m][K][N] workspace that receives the solutions.  When probes is NULL
 * they are drawn on the device: gp_rng_rademacher(opts->seed, stream 3).
 * Blocking.                                                                  */
int gp_trace(gp_op* op, int m, const int8_t* probes, double* u, double* tr_total,
             double* tr_kk, double* tr_Gkk, const gp_opts* opts, gp_stats* stats);

/* ---- autotuning -----------------------------------------------------------
 * gp_autotune: time every launch configuration (right-hand sides per
 * workgroup 1/2/4/8/16, persistent workgroups per compute unit 4/8, raster or
 * z-marching matvec; with GP_PRECOND_RB_IC0 the right-hand sides per work
 * item alone) with full solves of R random right-hand sides on this
 * operator under *base (host; NULL = defaults), keep the fastest in the
 * context for (K, log2 N, R rounded up to a power of two, precision,
 * preconditioner) and copy it into *best (host, may be NULL).  Later solves
 * whose rhs_tile / wg_per_cu / matvec are left automatic use it.  Blocking.
 * gp_tune_save / gp_tune_load: the context's table as a JSON file.          */
int gp_autotune(gp_op* op, int R, const gp_opts* base, gp_opts* best);
int gp_tune_save(gp_ctx* ctx, const char* path);
int gp_tune_load(gp_ctx* ctx, const char* path);

/* ---- random vectors ----------------------------------------------------
 * Counter-based Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw,
 * SC'11), keyed by `seed` (key words = low, high 32 bits) with counter
 * (q low, q high, stream low, stream high) for block q.  These supply the
 * N(0, I) vectors z1, z2 of Algorithm 2 (steps 2-3) and Rademacher probes.
 *  gp_rng_normal     : out[e], e < n, device FP64.  Pair q = e/2 takes the
 *                      block's words w0..w3, u1 = (((w1:w0) >> 11) + 0.5) 2^-53,
 *                      u2 likewise from (w3:w2); out[2q] = sqrt(-2 ln u1)
 *                      cos(2 pi u2), out[2q+1] = sqrt(-2 ln u1) sin(2 pi u2).
 *  gp_rng_rademacher : out[e], device int8; bit e % 128 of block q = e/128
 *                      (w0 least significant) gives +1 when set, else -1.
 *  gp_rng_raw        : the 4 words of blocks 0..nblocks-1, device uint32.
 *  gp_rng_gamma      : out[e] = scale[e] G_e with G_e ~ Gamma(shape, 1) (the
 *                      full conditionals of alpha and lambda, Section 3.2 and
 *                      Appendix A.2, for Gibbs sampling), by Marsaglia and
 *                      Tsang's rejection method (ACM TOMS 2000): a = shape
 *                      (shape + 1 below one), d = a - 1/3, c = 1/sqrt(9d);
 *                      attempt t < 64 of element e takes x, the cosine
 *                      Box-Muller normal of block 128e + 2t, and u from
 *                      (w1:w0) of block 128e + 2t + 1; with v = (1 + c x)^3 it
 *                      accepts d v when v > 0 and u < 1 - 0.0331 x^4 or
 *                      ln u < x^2/2 + d(1 - v + ln v); after 64 rejections
 *                      G = d.  For shape < 1, G is multiplied by U^(1/shape)
 *                      with U from (w3:w2) of block 128e + 1.  scale: device
 *                      FP64 [n], or NULL for 1; out: device FP64 [n].
 * Stream-ordered.                                                          */
int gp_rng_normal(gp_ctx* ctx, uint64_t seed, uint64_t stream, size_t n, double* out);
int gp_rng_rademacher(gp_ctx* ctx, uint64_t seed, uint64_t stream, size_t n, int8_t* out);
int gp_rng_raw(gp_ctx* ctx, uint64_t seed, uint64_t stream, size_t nblocks, uint32_t* out);
int gp_rng_gamma(gp_ctx* ctx, uint64_t seed, uint64_t stream, size_t n, double shape, const double* scale,
                 double* out);

/* ---- serving ---------------------------------------------------------------
 * A request loop over resident operators: requests (solve, sample, trace) are
 * submitted from any thread, admitted in arrival order while the server's HBM
 * budget and right-hand-side slots allow, join the running grouped solve at
 * the next round boundary (continuous batching) and retire at the round
 * boundary after their last right-hand side is done.  The
 * server runs on its own thread and HIP stream and holds its context busy
 * until destroyed; its operators must not be modified meanwhile.  Results do
 * not depend on which other requests share a round (batch-invariant
 * reductions): a request's result is bitwise the same alone and in the mix.
 * Every preconditioner is served (with GP_PRECOND_RB_IC0 each request is a
 * member of the grouped red-black solve).
 *
 * A server round: admit waiting requests (their workspaces carved from the
 * server's device memory, their right-hand sides prepared on the device), run
 * a round of iterations of every admitted right-hand side (about `chunk`,
 * planned from their states as the solvers plan theirs: the FP64 refinement
 * step first for requests just admitted and where inner solves are expected
 * to end), read the states, retire finished requests (one wait for all of the
 * round's retirements).  A request that fails (breakdown,
 * iteration cap, its deadline, cancellation, or an allocation error at
 * admission) retires with that status alone; the others go on unchanged.
 *
 * Request kinds, all on operator `op_index` with b_w = bw[op_index]:
 *  GP_REQ_SOLVE : x = Q^{-1}(b_w + n), n = gp_rng_normal(seed, stream 4)   (R = 1)
 *  GP_REQ_SAMPLE: Algorithm 2 with z1, z2 = gp_rng_normal(seed, 1), (seed, 2)  (R = 1)
 *  GP_REQ_TRACE : Hutchinson with cfg.probes Rademacher probes
 *                 gp_rng_rademacher(seed, 3); u = Q^{-1} v (Section 3.3)   (R = probes)
 * `out` (device FP64 [R][K][N], may be NULL) receives x, the sample or u; it
 * is written only when the request succeeds.                                */
#define GP_REQ_SOLVE  0
#define GP_REQ_SAMPLE 1
#define GP_REQ_TRACE  2

typedef struct gp_server gp_server;

typedef struct gp_server_cfg {
  size_t  hbm_budget;      /* bytes of request workspace (default 16 GiB): the device
                              memory the server takes for workspaces, in slabs of
                              1 GiB (or one request's size) kept until
                              gp_server_destroy, and the cap on the running
                              requests' bytes; a request waits while its workspace
                              does not fit                                           */
  int     max_active_rhs;  /* right-hand-side slots advanced together (default 1024)   */
  int     chunk;           /* inner iterations per round (default 4)                  */
  int     probes;          /* probes per trace request (default 16)                   */
  int     manual;          /* 0: rounds run as requests arrive (default); 1: a round
                              runs only when gp_server_step grants it (deterministic
                              schedules for replay and testing)                       */
  int     reserved;
  gp_opts opts;            /* solver options for every request                       */
} gp_server_cfg;

typedef struct gp_request {
  int      kind;           /* GP_REQ_*                                                */
  int      op_index;       /* index into the server's operators                      */
  uint64_t seed;           /* Philox key of the request's random vectors             */
  double*  out;            /* device result buffer or NULL                           */
  double   timeout_ms;     /* > 0: the request fails with GP_ERR_TIMEOUT if it has not
                              finished this long after submission (checked at round
                              boundaries); 0: no deadline                            */
} gp_request;

typedef struct gp_result {
  uint64_t ticket;
  int      kind, op_index, status, rhs;  /* status: GP_OK or the first failing one */
  int      iters_max, reserved;
  double   relres_max;
  double   latency_us;     /* submit -> result available                             */
  double   queue_us;       /* submit -> admitted (0 if never admitted)               */
  int64_t  admit_round;    /* index of the first server round the request took part in
                              (-1 if never admitted)                                 */
  int64_t  retire_round;   /* number of server rounds run when it retired            */
  double   trace_total;    /* GP_REQ_TRACE: estimates as in gp_trace_reduce          */
  double   trace_kk[GP_KMAX];   /* entries k < K of the operator are set           */
  double   trace_Gkk[GP_KMAX];
} gp_result;

typedef struct gp_server_stats {
  int64_t submitted, completed, rhs_solved, peak_active_rhs;
  int64_t failed;                           /* completed with a status other than GP_OK */
  int64_t rounds;                           /* solver rounds run                       */
  double  p50_us, p99_us, mean_us, max_us;  /* latency over successful requests       */
  double  elapsed_s;                        /* first submit -> last completion        */
  double  solves_per_s, requests_per_s;
} gp_server_stats;

void gp_server_cfg_default(gp_server_cfg* cfg);
/* ops: host array of nops operators of ctx (blocks and alpha set); bw: host
 * array of nops device pointers to FP64 [K][N] data right-hand sides.
 * Builds each operator's preconditioner for cfg->opts.precond (GP_ERR_NOT_SPD
 * if a block fails).                                                        */
int gp_server_create(gp_ctx* ctx, int nops, gp_op* const* ops, const double* const* bw,
                     const gp_server_cfg* cfg, gp_server** out);
/* thread-safe; returns at once with a ticket (host out).  GP_ERR_OOM if the
 * request alone exceeds the server's budget.                                */
int gp_server_submit(gp_server* srv, const gp_request* req, uint64_t* ticket);
/* thread-safe: a waiting request retires at once with GP_ERR_CANCELLED, a
 * running one at the next round boundary; GP_ERR_INVALID_ARG if the ticket
 * is unknown or has already finished.                                       */
int gp_server_cancel(gp_server* srv, uint64_t ticket);
/* manual mode only: run `rounds` more server rounds (admission, one solver
 * round of every admitted right-hand side, retirement) and wait until they
 * have run; a round with no admitted request does nothing and still counts. */
int gp_server_step(gp_server* srv, int rounds);
/* copies up to max finished results into out (host), *n receives the count  */
int gp_server_poll(gp_server* srv, gp_result* out, int max, int* n);
/* waits until every submitted request has finished (timeout_ms < 0: no limit);
 * GP_ERR_BUSY on timeout.  In manual mode it returns GP_ERR_BUSY at once
 * while requests remain (rounds are the caller's).                           */
int gp_server_drain(gp_server* srv, int timeout_ms);
int gp_server_get_stats(gp_server* srv, gp_server_stats* out);
int gp_server_destroy(gp_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* GMRF_H */
