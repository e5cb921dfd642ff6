// Red-black incomplete Cholesky: set-up, split, recovery and finalisation
// launches, the FP64 red stage of the refinement, and the grouped solver-round
// launches with FP64 inner vectors (the kernels are in rbic.hpp; the FP32
// round launches are in k_rbic_f32.hip).
#include "rbic.hpp"

namespace gp {

hipError_t launch_rb_setup(hipStream_t s, const RbDev& rb, const double* B64, double* P64, float* P32,
                           double* D64, float* D32, double* S64, float* S32, int* bad) {
  const int gr = (rb.NR + TILE - 1) / TILE, gb = (rb.NB + TILE - 1) / TILE;
#define X(KK)                                                                                         \
  case KK:                                                                                            \
    if (gr > 0) GP_LAUNCH(k_rb_setup_red<KK>, dim3(gr), dim3(TILE), 0, s, rb, B64, P64, P32, bad); \
    if (gb > 0)                                                                                       \
      GP_LAUNCH(k_rb_setup_black<KK>, dim3(gb), dim3(TILE), 0, s, rb, B64, D64, D32, S64, S32, bad); \
    break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_rb_split(hipStream_t s, const RbDev& rb, int R, const double* b, const double* x, int zero_guess,
                           double* t, double* c, double* xB, double* bbpart, const RbSplitFirst& first) {
  const RbFirst<float> f32{first.f32 ? (float*)first.r : nullptr, (float*)first.p, first.part, first.vstride,
                           first.pstride, first.r0};
  const RbFirst<double> f64{first.f32 ? nullptr : (double*)first.r, (double*)first.p, first.part, first.vstride,
                            first.pstride, first.r0};
  // right-hand sides per workgroup of the voxel pass (the red inverse held
  // across them): the largest of 4, 2, 1 that leaves 1024 workgroups; the
  // black pass (its time is in the gathers of t) takes one
  int rcv = 1;
  for (int cand : {4, 2})
    if ((long)rb.ntN * ((R + cand - 1) / cand) >= 1024) {
      rcv = cand;
      break;
    }
  const int rcb = 1;
  const int nchv = (R + rcv - 1) / rcv, nchb = (R + rcb - 1) / rcb;
#define X(KK)                                                                                              \
  case KK:                                                                                                 \
    GP_LAUNCH(k_rb_split_voxels<KK>, grid2(rb.ntN, nchv), dim3(TILE), 0, s, rb, R, rcv, b, x, zero_guess, t, c, \
                       xB, bbpart);                                                                        \
    if (rb.ntB > 0) {                                                                                      \
      if (first.f32)                                                                                       \
        GP_LAUNCH((k_rb_split_black<KK, float>), grid2(rb.ntB, nchb), dim3(TILE), 0, s, rb, R, rcb, t, c, f32); \
      else                                                                                                 \
        GP_LAUNCH((k_rb_split_black<KK, double>), grid2(rb.ntB, nchb), dim3(TILE), 0, s, rb, R, rcb, t, c, f64); \
    }                                                                                                      \
    break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

RB_INST(double)

hipError_t launch_rb_recover(hipStream_t s, const RbDev& rb, int R, const RhsState* st, const double* t,
                             const double* u64, const double* xB, double* x) {
  if (rb.ntN == 0) return hipSuccess;
#define X(KK) \
  case KK: GP_LAUNCH(k_rb_recover<KK>, grid2(rb.ntN, R), dim3(TILE), 0, s, rb, st, t, u64, xB, x); break;
  RB_K_SWITCH(rb.K, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_rbg_red64(hipStream_t s, int K, const RbProb* probs, int nprob, int W) {
  if (W == 0) return hipSuccess;
#define X(KK)                                                                                               \
  case KK:                                                                                                  \
    if constexpr (HoldRb<double, KK, 1>::v)                                                                 \
      GP_LAUNCH((k_rb_red<double, KK, true, true>), dim3(W), dim3(TILE), 0, s, probs, nprob);     \
    else                                                                                                    \
      GP_LAUNCH((k_rb_red<double, KK, false, true>), dim3(W), dim3(TILE), 0, s, probs, nprob);    \
    break;
  RB_K_SWITCH(K, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_rbg_finalize(hipStream_t s, int kind, const RbProb* probs, int nprob, int nblocks) {
  if (nblocks == 0) return hipSuccess;
  if (kind == 0)
    GP_LAUNCH(k_rb_finalize<0>, dim3(nblocks), dim3(FIN_WAVES * WAVE), 0, s, probs, nprob);
  else
    GP_LAUNCH(k_rb_finalize<1>, dim3(nblocks), dim3(FIN_WAVES * WAVE), 0, s, probs, nprob);
  return hipGetLastError();
}

}  // namespace gp
