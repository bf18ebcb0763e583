// Per-call Fletcher-Powell kernels (n <= 16), float64 H.v that also stores
// the gradient and f: every compiled chunk size and K-step count.
#include "dispatch.hpp"

namespace chessfad {

FpMfmaLaunch fp_call_entry_grad(int C, int nk, int n) { return fp_call_by_steps<F64, false, true>(C, nk, n); }

}  // namespace chessfad
