// PCG kernels with inner precision double.
#include "pcg_launch.hpp"

namespace gp {

hipError_t launch_refine_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_refine_t<double>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_matvec_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_matvec_t<double>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_matvec_zm_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_matvec_zm_t<double>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_update_f64(hipStream_t s, int pc, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_update_t<double>(s, pc, K, probs, nprob, W, nblk);
}
hipError_t launch_addsol_f64(hipStream_t s, int K, const Prob* probs, int nprob, int W, int nblk) {
  return launch_addsol_t<double>(s, K, probs, nprob, W, nblk);
}

}  // namespace gp
