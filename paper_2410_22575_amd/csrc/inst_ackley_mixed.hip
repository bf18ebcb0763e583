// Ackley: float32 hDuals with compensated sums, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch mixed_ackley(int C, bool hess) {
    return hess ? plain_entry<F32C, Ackley, true>(C) : plain_entry<F32C, Ackley, false>(C);
}

}  // namespace chessfad
