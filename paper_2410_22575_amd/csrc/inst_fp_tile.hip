// Fletcher-Powell point-tile kernels (n <= 16), float64: every K-step count
// of the value column and both output kinds.
#include "dispatch.hpp"

namespace chessfad {

FpMfmaLaunch fp_tile_entry(int nk, bool hess) {
    return hess ? fp_tile_by_steps<F64, true>(nk) : fp_tile_by_steps<F64, false>(nk);
}

}  // namespace chessfad
