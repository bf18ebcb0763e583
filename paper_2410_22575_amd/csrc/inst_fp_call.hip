// Per-call Fletcher-Powell kernels (n <= 16), float64: every compiled chunk
// size and K-step count, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

FpMfmaLaunch fp_call_entry(int C, int nk, bool hess, int n) {
    return hess ? fp_call_by_steps<F64, true, false>(C, nk, n) : fp_call_by_steps<F64, false, false>(C, nk, n);
}

}  // namespace chessfad
