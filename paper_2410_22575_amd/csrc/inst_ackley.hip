// Plain float64 kernels for Ackley, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_ackley(int C, bool hess) {
    return hess ? plain_entry<Ackley, true>(C) : plain_entry<Ackley, false>(C);
}

}  // namespace chessfad
