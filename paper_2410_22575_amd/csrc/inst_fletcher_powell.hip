// Plain float64 kernels for FletcherPowell, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_fletcher_powell(int C, bool hess) {
    return hess ? plain_entry<FletcherPowell, true>(C) : plain_entry<FletcherPowell, false>(C);
}

}  // namespace chessfad
