// Per-call Fletcher-Powell kernels (n <= 16), mixed precision: every
// compiled chunk size and K-step count, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

FpMfmaLaunch fp_call_entry_mixed(int C, int nk, bool hess, int n) {
    return hess ? fp_call_by_steps<F32C, true, false>(C, nk, n) : fp_call_by_steps<F32C, false, false>(C, nk, n);
}

}  // namespace chessfad
