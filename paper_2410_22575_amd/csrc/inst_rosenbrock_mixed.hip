// Rosenbrock: float32 hDuals with compensated sums, every compiled chunk size, H.v and Hessian; the L0 / L1 mappings of H.v
// (L1 at n = 16 on register-resident points).
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch mixed_rosenbrock(int C, bool hess) {
    return hess ? plain_entry<F32C, Rosenbrock, true>(C) : plain_entry<F32C, Rosenbrock, false>(C);
}

CoarseLaunch coarse_mixed_rosenbrock(int C, int level) {
    return level == 0 ? coarse_entry<F32C, Rosenbrock, 0>(C) : coarse_entry<F32C, Rosenbrock, 1>(C);
}

Row16Launch row16_mixed_rosenbrock(int C) { return row16_entry<F32C, Rosenbrock>(C); }

RowsLaunch rosenbrock_rows_mixed(int C) { return rosenbrock_rows_entry<F32C>(C); }

}  // namespace chessfad
