// Launch switches of the PCG kernels over K (1..KMAX) and the preconditioner,
// for one inner precision T.  Included by k_pcg_f32.hip and k_pcg_f64.hip,
// which compile the two precisions in parallel.
#pragma once
#include "launch.hpp"
#include "pcg.hpp"
#include "zm.hpp"

namespace gp {

#define GP_K_CASES(X)                                                                                  \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
      X(20) X(21) X(22) X(23) X(24)

// Kernel templated on <T, PC, K> launched with (probs, nprob, W).
#define GP_PC_SWITCH(KERNEL, BLOCKDIM)                                                         \
  const dim3 g(nblk), b(BLOCKDIM);                                                             \
  switch (K) {                                                                                 \
    GP_K_CASES(GP_PC_CASE_##KERNEL)                                                            \
    default: return hipErrorInvalidValue;                                                      \
  }                                                                                            \
  return hipGetLastError();

#define GP_PC_CASE(KERNEL, KK)                                                                 \
  case KK:                                                                                     \
    if (pc == PC_BLOCK)                                                                        \
      GP_LAUNCH((KERNEL<T, PC_BLOCK, KK>), g, b, 0, s, probs, nprob, W);               \
    else                                                                                       \
      GP_LAUNCH((KERNEL<T, PC_JACOBI, KK>), g, b, 0, s, probs, nprob, W);              \
    break;
#define GP_PC_CASE_k_refine(KK) GP_PC_CASE(k_refine, KK)
#define GP_PC_CASE_k_matvec(KK) GP_PC_CASE(k_matvec, KK)
#define GP_PC_CASE_k_matvec_zm(KK) GP_PC_CASE(k_matvec_zm, KK)
#define GP_PC_CASE_k_update(KK) GP_PC_CASE(k_update, KK)

template <typename T>
hipError_t launch_refine_t(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  GP_PC_SWITCH(k_refine, TILE)
}

template <typename T>
hipError_t launch_matvec_t(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  GP_PC_SWITCH(k_matvec, TILE)
}

template <typename T>
hipError_t launch_matvec_zm_t(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  GP_PC_SWITCH(k_matvec_zm, ZFX * ZFY)
}

template <typename T>
hipError_t launch_update_t(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  GP_PC_SWITCH(k_update, TILE)
}

template <typename T>
hipError_t launch_addsol_t(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk) {
  const dim3 g(nblk), b(TILE);
  switch (K) {
#define X(KK) case KK: GP_LAUNCH((k_addsol<T, KK>), g, b, 0, s, probs, nprob, W); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gp
