// FletcherPowell: float32 hDuals with compensated sums, every compiled chunk size, H.v and Hessian; the L0 / L1 mappings of H.v.
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch mixed_fletcher_powell(int C, bool hess) {
    return hess ? plain_entry<F32C, FletcherPowell, true>(C) : plain_entry<F32C, FletcherPowell, false>(C);
}

CoarseLaunch coarse_mixed_fletcher_powell(int C, int level) {
    return level == 0 ? coarse_entry<F32C, FletcherPowell, 0>(C) : coarse_entry<F32C, FletcherPowell, 1>(C);
}

}  // namespace chessfad
