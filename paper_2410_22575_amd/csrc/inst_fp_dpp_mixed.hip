// Per-call Fletcher-Powell kernels for n > 16, mixed precision: every
// compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

FpDppLaunch fp_dpp_entry_mixed(int C, bool hess) {
    return hess ? fp_dpp_entry_c<F32C, true, false>(C) : fp_dpp_entry_c<F32C, false, false>(C);
}

}  // namespace chessfad
