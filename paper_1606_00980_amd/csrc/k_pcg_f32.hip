// Launchers of the PCG kernels with inner precision float.
#include "launch.hpp"
#include "pcg.hpp"
#include "zm.hpp"

namespace gp {

#define GP_K_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_refine_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  const dim3 g(nblk), b(TILE);
  switch (K) {
#define X(KK)                                                                                   \
  case KK:                                                                                      \
    if (pc == PC_BLOCK)                                                                         \
      hipLaunchKernelGGL((k_refine<float, PC_BLOCK, KK>), g, b, 0, s, probs, nprob, W);          \
    else                                                                                        \
      hipLaunchKernelGGL((k_refine<float, PC_JACOBI, KK>), g, b, 0, s, probs, nprob, W);         \
    break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_matvec_f32(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk, int parity) {
  const dim3 g(nblk), b(TILE);
  switch (K) {
#define X(KK) case KK: hipLaunchKernelGGL((k_matvec<float, KK>), g, b, 0, s, probs, nprob, W, parity); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_matvec_zm_f32(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk, int parity) {
  const dim3 g(nblk), b(ZFX * ZFY);
  switch (K) {
#define X(KK) case KK: hipLaunchKernelGGL((k_matvec_zm<float, KK>), g, b, 0, s, probs, nprob, W, parity); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int zm_rhs_per_block(int K) {
  switch (K) {
#define X(KK) case KK: return ZRc<KK>::v;
    GP_K_CASES(X)
#undef X
    default: return 1;
  }
}

hipError_t launch_update_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk, int parity) {
  const dim3 g(nblk), b(TILE);
  switch (K) {
#define X(KK)                                                                                   \
  case KK:                                                                                      \
    if (pc == PC_BLOCK)                                                                         \
      hipLaunchKernelGGL((k_update<float, PC_BLOCK, KK>), g, b, 0, s, probs, nprob, W, parity);  \
    else                                                                                        \
      hipLaunchKernelGGL((k_update<float, PC_JACOBI, KK>), g, b, 0, s, probs, nprob, W, parity); \
    break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_addsol_f32(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk) {
  const dim3 g(nblk), b(TILE);
  switch (K) {
#define X(KK) case KK: hipLaunchKernelGGL((k_addsol<float, KK>), g, b, 0, s, probs, nprob, W); break;
    GP_K_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gp
