// Plain float64 kernels for Rosenbrock, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_rosenbrock(int C, bool hess) {
    return hess ? plain_entry<Rosenbrock, true>(C) : plain_entry<Rosenbrock, false>(C);
}

}  // namespace chessfad
