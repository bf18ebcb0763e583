// Rosenbrock: float64, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_rosenbrock(int C, bool hess) {
    return hess ? plain_entry<F64, Rosenbrock, true>(C) : plain_entry<F64, Rosenbrock, false>(C);
}

}  // namespace chessfad
