// Ackley: float64, every compiled chunk size, H.v (also with the gradient) and Hessian; the L0 / L1 mappings of H.v
// (L1 at n = 16 on register-resident points).
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_ackley(int C, bool hess) {
    return hess ? plain_entry<F64, Ackley, true>(C) : plain_entry<F64, Ackley, false>(C);
}

PlainLaunch grad_ackley(int C) { return plain_entry<F64, Ackley, false, true>(C); }

CoarseLaunch coarse_ackley(int C, int level) {
    return level == 0 ? coarse_entry<F64, Ackley, 0>(C) : coarse_entry<F64, Ackley, 1>(C);
}

Row16Launch row16_ackley(int C) { return row16_entry<F64, Ackley>(C); }

}  // namespace chessfad
