// Rosenbrock: float32 hDuals with compensated sums, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch mixed_rosenbrock(int C, bool hess) {
    return hess ? plain_entry<F32C, Rosenbrock, true>(C) : plain_entry<F32C, Rosenbrock, false>(C);
}

}  // namespace chessfad
