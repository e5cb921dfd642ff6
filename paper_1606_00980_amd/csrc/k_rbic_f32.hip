// Red-black incomplete Cholesky: the solver-round launches with FP32 inner
// vectors (the kernels are in rbic.hpp).
#include "rbic.hpp"

namespace gp {

RB_INST(float)

}  // namespace gp
