// Fletcher-Powell MFMA kernels for any n (one point per workgroup), float64
// and mixed precision, every compiled chunk size and output kind.
#include "dispatch.hpp"

namespace chessfad {

FpRowsLaunch fp_rows_entry(int C, bool hess, bool mixed) {
    if (mixed) return hess ? fp_rows_entry_c<F32C, true>(C) : fp_rows_entry_c<F32C, false>(C);
    return hess ? fp_rows_entry_c<F64, true>(C) : fp_rows_entry_c<F64, false>(C);
}

}  // namespace chessfad
