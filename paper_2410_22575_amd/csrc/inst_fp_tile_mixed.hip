// Fletcher-Powell point-tile kernels (n <= 16), mixed precision (float32
// tile): every K-step count of the value column and both output kinds.
#include "dispatch.hpp"

namespace chessfad {

FpMfmaLaunch fp_tile_entry_mixed(int nk, bool hess) {
    return hess ? fp_tile_by_steps<F32C, true>(nk) : fp_tile_by_steps<F32C, false>(nk);
}

}  // namespace chessfad
