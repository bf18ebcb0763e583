// Ackley: float32 hDuals with compensated sums, every compiled chunk size, H.v and Hessian; the L0 / L1 mappings of H.v
// (L1 at n = 16 on register-resident points).
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch mixed_ackley(int C, bool hess) {
    return hess ? plain_entry<F32C, Ackley, true>(C) : plain_entry<F32C, Ackley, false>(C);
}

CoarseLaunch coarse_mixed_ackley(int C, int level) {
    return level == 0 ? coarse_entry<F32C, Ackley, 0>(C) : coarse_entry<F32C, Ackley, 1>(C);
}

Row16Launch row16_mixed_ackley(int C) { return row16_entry<F32C, Ackley>(C); }

}  // namespace chessfad
