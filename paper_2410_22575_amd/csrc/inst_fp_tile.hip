// Fletcher-Powell point-tile kernels (n <= 16), float64: every K-step count
// of the value column and both output kinds.
#include "dispatch.hpp"

namespace chessfad {

template <bool kHess>
static FpMfmaLaunch tile_by_steps(int nk) {
    switch (nk) {
        case 1: return &launch_fp_tile<1, kHess>;
        case 2: return &launch_fp_tile<2, kHess>;
        case 4: return &launch_fp_tile<4, kHess>;
        case 8: return &launch_fp_tile<8, kHess>;
        default: return nullptr;
    }
}

FpMfmaLaunch fp_tile_entry(int nk, bool hess) { return hess ? tile_by_steps<true>(nk) : tile_by_steps<false>(nk); }

}  // namespace chessfad
