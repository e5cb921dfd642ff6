// PCG kernels with inner precision float (FP64 refinement and solution).
#include "pcg_launch.hpp"

namespace gp {

hipError_t launch_refine_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_refine_t<float>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_matvec_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_matvec_t<float>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_matvec_zm_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_matvec_zm_t<float>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_update_f32(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_update_t<float>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_addsol_f32(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_addsol_t<float>(s, K, probs, nprob, W, nblk);
}

int zm_rhs_per_block(int K) {
  switch (K) {
#define X(KK) case KK: return ZRc<KK>::v;
    GP_K_CASES(X)
#undef X
    default: return 1;
  }
}

}  // namespace gp
