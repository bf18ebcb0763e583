// Rosenbrock: float64, every compiled chunk size, H.v (also with the gradient) and Hessian; the L0 / L1 mappings of H.v
// (L1 at n = 16 on register-resident points).
#include "dispatch.hpp"

namespace chessfad {

PlainLaunch plain_rosenbrock(int C, bool hess) {
    return hess ? plain_entry<F64, Rosenbrock, true>(C) : plain_entry<F64, Rosenbrock, false>(C);
}

PlainLaunch grad_rosenbrock(int C) { return plain_entry<F64, Rosenbrock, false, true>(C); }

CoarseLaunch coarse_rosenbrock(int C, int level) {
    return level == 0 ? coarse_entry<F64, Rosenbrock, 0>(C) : coarse_entry<F64, Rosenbrock, 1>(C);
}

Row16Launch row16_rosenbrock(int C) { return row16_entry<F64, Rosenbrock>(C); }

RowsLaunch rosenbrock_rows(int C) { return rosenbrock_rows_entry<F64>(C); }

}  // namespace chessfad
