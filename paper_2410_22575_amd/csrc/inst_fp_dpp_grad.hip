// Per-call Fletcher-Powell kernels for n > 16, float64 H.v with the gradient
// and f: every compiled chunk size.
#include "dispatch.hpp"

namespace chessfad {

FpDppLaunch fp_dpp_entry_grad(int C) { return fp_dpp_entry_c<F64, false, true>(C); }

}  // namespace chessfad
