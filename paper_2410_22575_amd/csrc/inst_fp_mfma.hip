// Fletcher-Powell MFMA kernels (n <= 16), float64: every compiled chunk size,
// K-step count and output kind.
#include "dispatch.hpp"

namespace chessfad {

template <bool kHess>
static FpMfmaLaunch by_steps(int C, int nk) {
    switch (nk) {
        case 1: return fp_mfma_entry_c<F64, 1, kHess>(C);
        case 2: return fp_mfma_entry_c<F64, 2, kHess>(C);
        case 4: return fp_mfma_entry_c<F64, 4, kHess>(C);
        case 8: return fp_mfma_entry_c<F64, 8, kHess>(C);
        default: return nullptr;
    }
}

FpMfmaLaunch fp_mfma_entry(int C, int nk, bool hess) { return hess ? by_steps<true>(C, nk) : by_steps<false>(C, nk); }

}  // namespace chessfad
