// Per-call Fletcher-Powell kernels for n > 16, float64: every compiled chunk
// size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

FpDppLaunch fp_dpp_entry(int C, bool hess) {
    return hess ? fp_dpp_entry_c<F64, true, false>(C) : fp_dpp_entry_c<F64, false, false>(C);
}

}  // namespace chessfad
