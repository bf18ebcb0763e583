// Symmetric forms of the per-call Fletcher-Powell kernel for n > 16, mixed
// precision: every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

FpDppLaunch fp_dpp_sym_entry_mixed(int C, bool hess) {
    return hess ? fp_dpp_entry_c<F32C, true, false, true>(C) : fp_dpp_entry_c<F32C, false, false, true>(C);
}

}  // namespace chessfad
