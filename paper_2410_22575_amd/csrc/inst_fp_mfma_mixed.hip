// Fletcher-Powell MFMA kernels (n <= 16), float32 derivative columns, float64 values: every compiled chunk size,
// K-step count and output kind.
#include "dispatch.hpp"

namespace chessfad {

template <bool kHess>
static FpMfmaLaunch by_steps(int C, int nk) {
    switch (nk) {
        case 1: return fp_mfma_entry_c<F32C, 1, kHess>(C);
        case 2: return fp_mfma_entry_c<F32C, 2, kHess>(C);
        case 4: return fp_mfma_entry_c<F32C, 4, kHess>(C);
        case 8: return fp_mfma_entry_c<F32C, 8, kHess>(C);
        default: return nullptr;
    }
}

FpMfmaLaunch fp_mfma_entry_mixed(int C, int nk, bool hess) { return hess ? by_steps<true>(C, nk) : by_steps<false>(C, nk); }

}  // namespace chessfad
