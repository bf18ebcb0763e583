// FletcherPowell: float64, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_fletcher_powell(int C, bool hess) {
    return hess ? plain_entry<F64, FletcherPowell, true>(C) : plain_entry<F64, FletcherPowell, false>(C);
}

}  // namespace chessfad
