// Ackley: symmetric kernels (SCHUNK-HESS, SC-HESS-VEC), float64 and mixed
// precision, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

SymLaunch sym_ackley(int C, bool hess, bool mixed) {
    if (mixed) return hess ? sym_entry<F32C, Ackley, true>(C) : sym_entry<F32C, Ackley, false>(C);
    return hess ? sym_entry<F64, Ackley, true>(C) : sym_entry<F64, Ackley, false>(C);
}

}  // namespace chessfad
