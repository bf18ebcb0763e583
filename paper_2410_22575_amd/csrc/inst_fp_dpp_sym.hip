// Symmetric forms of the per-call Fletcher-Powell kernel for n > 16, float64:
// every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

FpDppLaunch fp_dpp_sym_entry(int C, bool hess) {
    return hess ? fp_dpp_entry_c<F64, true, false, true>(C) : fp_dpp_entry_c<F64, false, false, true>(C);
}

}  // namespace chessfad
