// Fletcher-Powell MFMA kernels (n <= 16), float64: every compiled chunk size,
// K-step count, output kind and form (full or symmetric).
#include "dispatch.hpp"

namespace chessfad {

template <bool kHess, bool kSym>
static FpMfmaLaunch by_steps(int C, int nk) {
    switch (nk) {
        case 1: return fp_mfma_entry_c<F64, 1, kHess, kSym>(C);
        case 2: return fp_mfma_entry_c<F64, 2, kHess, kSym>(C);
        case 4: return fp_mfma_entry_c<F64, 4, kHess, kSym>(C);
        case 8: return fp_mfma_entry_c<F64, 8, kHess, kSym>(C);
        default: return nullptr;
    }
}

FpMfmaLaunch fp_mfma_entry(int C, int nk, bool hess, bool sym) {
    if (sym) return hess ? by_steps<true, true>(C, nk) : by_steps<false, true>(C, nk);
    return hess ? by_steps<true, false>(C, nk) : by_steps<false, false>(C, nk);
}

}  // namespace chessfad
