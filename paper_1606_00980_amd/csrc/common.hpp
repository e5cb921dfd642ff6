// Plain structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gp {

constexpr int KMAX = 24;     // largest supported number of regressors
constexpr int TILE = 256;    // voxels per workgroup in the voxel-parallel kernels
constexpr int NPART = 7;     // reduction values per (right-hand side, tile), at most
constexpr int NPROF = 12;    // profiling counters per problem
// profiling counter slots (right-hand sides processed, launches with work)
enum ProfSlot : int {
  PF_REFINE_RHS = 0, PF_REFINE_ACT, PF_ADDSOL_D, PF_ADDSOL_P, PF_MATVEC_RHS,
  PF_MATVEC_ACT, PF_UPDATE_RHS, PF_UPDATE_FRESH, PF_UPDATE_ACT,
  PF_REFINE_X0,      // refinements with a zero start value (x not read)
  PF_ADDSOL_FRESH,   // first x += d from a zero start value (x written, not read)
};
constexpr int RCMAX = 16;    // right-hand sides per workgroup, upper bound
constexpr int UPAIR_KMAX = 10;   // FP32 red-stage vectors stored in right-hand-side pairs up to this K
constexpr int PC_JACOBI = 0; // preconditioner kinds as seen by the kernels
constexpr int PC_BLOCK = 1;

// Life cycle of one right-hand side inside a solve.
enum Phase : int {
  PH_OUTER = 0,   // waits for an FP64 residual evaluation (refinement step)
  PH_INNER = 1,   // inner PCG iterations in progress
  PH_DONE = 2,    // finished (converged, capped or broken down)
};

// Status codes mirrored from gmrf.h for device code.
enum DevStatus : int { ST_OK = 0, ST_NOT_CONVERGED = -5, ST_BREAKDOWN = -6 };

// Per right-hand-side solver state, written only by the finalising workgroup.
struct RhsState {
  double bnorm2;    // ||b||^2
  double rr64;      // last FP64 ||b - Qx||^2
  double rho;       // r'z of the next inner iteration (three-term expansion)
  double a;         // step length of the last inner iteration
  double beta;      // direction update coefficient of the next iteration
  double target2;   // inner stop threshold on ||r||^2
  double relres;    // last FP64 relative residual
  unsigned long long slots;   // bit i: an outer step came after i of this right-hand side's own iterations
  int phase, status, inner_it, total_it;
  int outer;
  int has_d;        // the inner correction d holds a valid sum
  int pend;         // a * p of the last iteration is still to be added to x
  int zero_b;
};

// Device view of one operator.
struct OpDev {
  const int* nbr;        // [6][N]: -x,+x,-y,+y,-z,+z neighbour, or the voxel itself
  const double* B64;     // packed lower triangle of B_n, [K(K+1)/2][N]
  const float* B32;
  const double* P64;     // preconditioner: packed inverse block or inverse diagonal
  const float* P32;
  const double* L64;     // packed lower Cholesky factor of B_n
  const int* gmap;       // [nz][ny][nx]: voxel number, or -1 outside the mask
  int N, K, ntiles, dirs;
  int nx, ny, nz, spare;
  double alpha64[KMAX];
  float alpha32[KMAX];
};

struct SolveCfg {
  double tol, inner_tol;
  int max_iter, max_outer;
  int zero_guess;   // start value zero: x neither read by the first refinement nor by the first x += d
  int spare;
};

// One member of a grouped launch: an operator with R right-hand sides.
struct Prob {
  OpDev op;
  const double* b;       // FP64 [R][K][N]
  double* x;             // FP64 [R][K][N]
  void* d;               // inner vectors in the inner precision, [R][K][N]
  void* r;
  void* p;
  void* q;
  RhsState* st;          // [R]
  double* part;          // [NPART][R][pstride]
  long long* prof;       // [NPROF] work counters, or null when not profiling
  int R, Rc, nchunks, work_begin, work_count;   // matvec / update: Rc right-hand sides per work item
  int Rco, nchunks_o, work_begin_o, work_count_o;   // refine / addsol: Rco per work item
  int fin_begin;         // first finalising workgroup of this problem
  int pstride;           // partials per (value, right-hand side): max(raster, z-march tiles)
  // z-marching matvec (mv_mode = 1): footprint tiles x segments of zs slices
  int mv_mode, zs, nseg, nyt, mv_tiles, mv_nchunks, mv_begin, mv_count;
  SolveCfg cfg;
};

// Device view of the red-black split of an operator for the incomplete
// Cholesky preconditioner: voxels with even x + y + z ("red") and odd
// ("black"), each numbered compactly in increasing voxel order.  Adjacent
// voxels always have different colours.
struct RbDev {
  const int* blk;        // [NB] voxel of black position i
  const int* red;        // [NR] voxel of red position j
  const int* nbB;        // [6][NB] red position of each neighbour of black i, or -1
  const int* nbR;        // [6][NR] black position of each neighbour of red j, or -1
  const int* vpos;       // [N] 2 * (position in its colour) + colour (1 = black)
  const double* D64;     // [NBt][NB] packed Q_mm = B_m + diag(alpha) deg_m (black)
  const float* D32;
  const double* S64;     // [NBt][NB] packed inverse of the Schur block S_m (black)
  const float* S32;
  const double* P64;     // [NBt][NR] packed inverse of Q_nn (red)
  const float* P32;
  long long* prof;       // [NPROF] work counters while profiling, else null
  int NB, NR, ntB, ntR, N, K;
  int ntN;               // tiles of 256 voxels over all N (split, recovery, ||b||^2 partials)
  int tbB, tbR;          // tiles per block of the work order (black, red)
  int zero_start;        // the start value is zero: x is not read
  double alpha64[KMAX];
  float alpha32[KMAX];
};

// One member of a grouped red-black launch: an operator's colour split and
// preconditioner with R right-hand sides, their states and vectors, and where
// its work items start in the launches of its group (all members of a group
// have the same K).
struct RbProb {
  RbDev rb;
  Prob pr;               // st, part, R, pstride, cfg, prof, fin_begin (the finalisers' view)
  const double* bb;      // [R][ntN] ||b||^2 partials of the split
  const double* c64;     // [R][K][NB] black right-hand side of the Schur system
  double* xB;            // [R][K][NB] black solution (FP64)
  double* u64;           // [R][K][NR] red stage of the FP64 refinement
  void* d;               // inner vectors [R][K][NB]
  void* r;
  void* p;
  void* q;
  void* u;               // [R][K][NR] red stage of an inner step
  int Rc, nch;           // right-hand sides per inner work item, chunks of them
  int Rco, ncho;         // right-hand sides per outer (refine, x_B += d) work item, chunks of them
  int wB, wR, wO;        // first black-tile, red-tile and outer work item
  int uw;                // right-hand sides per row set of u: 2 (pairs) or 1
};

// Packed index of the symmetric (k, j) entry, lower triangle row-major.
__host__ __device__ constexpr int pk(int k, int j) {
  return k >= j ? k * (k + 1) / 2 + j : j * (j + 1) / 2 + k;
}

}  // namespace gp
