// FletcherPowell: float64, every compiled chunk size, H.v (also with the gradient) and Hessian; the L0 / L1 mappings of H.v.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_fletcher_powell(int C, bool hess) {
    return hess ? plain_entry<F64, FletcherPowell, true>(C) : plain_entry<F64, FletcherPowell, false>(C);
}

PlainLaunch grad_fletcher_powell(int C) { return plain_entry<F64, FletcherPowell, false, true>(C); }

CoarseLaunch coarse_fletcher_powell(int C, int level) {
    return level == 0 ? coarse_entry<F64, FletcherPowell, 0>(C) : coarse_entry<F64, FletcherPowell, 1>(C);
}

}  // namespace chessfad
