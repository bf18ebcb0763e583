// Ackley: float64, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_ackley(int C, bool hess) {
    return hess ? plain_entry<F64, Ackley, true>(C) : plain_entry<F64, Ackley, false>(C);
}

}  // namespace chessfad
