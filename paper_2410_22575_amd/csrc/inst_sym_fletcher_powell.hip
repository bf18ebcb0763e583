// FletcherPowell: symmetric kernels (SCHUNK-HESS, SC-HESS-VEC), float64 and mixed
// precision, every compiled chunk size, H.v and Hessian.
#include "dispatch.hpp"

namespace chessfad {

SymLaunch sym_fletcher_powell(int C, bool hess, bool mixed) {
    if (mixed) return hess ? sym_entry<F32C, FletcherPowell, true>(C) : sym_entry<F32C, FletcherPowell, false>(C);
    return hess ? sym_entry<F64, FletcherPowell, true>(C) : sym_entry<F64, FletcherPowell, false>(C);
}

}  // namespace chessfad
