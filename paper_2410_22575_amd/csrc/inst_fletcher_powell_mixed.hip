// FletcherPowell: float32 hDuals with compensated sums, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch mixed_fletcher_powell(int C, bool hess) {
    return hess ? plain_entry<F32C, FletcherPowell, true>(C) : plain_entry<F32C, FletcherPowell, false>(C);
}

}  // namespace chessfad
