// Rosenbrock: symmetric kernels (SCHUNK-HESS, SC-HESS-VEC), float64 and mixed
// precision, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

SymLaunch sym_rosenbrock(int C, bool hess, bool mixed) {
    if (mixed) return hess ? sym_entry<F32C, Rosenbrock, true>(C) : sym_entry<F32C, Rosenbrock, false>(C);
    return hess ? sym_entry<F64, Rosenbrock, true>(C) : sym_entry<F64, Rosenbrock, false>(C);
}

}  // namespace chessfad
