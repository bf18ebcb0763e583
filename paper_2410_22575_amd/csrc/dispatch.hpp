// Kernel tables shared by the instantiation units and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "kernel_fp_call.hpp"
#include "kernel_fp_dpp.hpp"
#include "kernel_fp_mfma.hpp"
#include "kernel_fp_tile.hpp"
#include "kernel_fp_rows.hpp"
#include "kernel_plain.hpp"
#include "kernel_row16.hpp"
#include "kernel_sym.hpp"

namespace chessfad {

using PlainLaunch = hipError_t (*)(const PlainArgs&, dim3 grid, dim3 block, hipStream_t);

// Chunk sizes compiled into the library.
constexpr int kChunks[] = {1, 2, 4, 8, 16};
constexpr int kNumChunks = sizeof(kChunks) / sizeof(kChunks[0]);

template <class P, class F, int C, bool kHess, bool kGrad>
hipError_t launch_plain(const PlainArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    const size_t lds = plain_lds_bytes<P, F>(a.n, a.pstride, (int)block.x, kHess);
    hipLaunchKernelGGL((plain_kernel<P, F, C, kHess, kGrad>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <class P, class F, bool kHess, bool kGrad = false>
PlainLaunch plain_entry(int C) {
    switch (C) {
        case 1: return &launch_plain<P, F, 1, kHess, kGrad>;
        case 2: return &launch_plain<P, F, 2, kHess, kGrad>;
        case 4: return &launch_plain<P, F, 4, kHess, kGrad>;
        case 8: return &launch_plain<P, F, 8, kHess, kGrad>;
        case 16: return &launch_plain<P, F, 16, kHess, kGrad>;
        default: return nullptr;
    }
}

using CoarseLaunch = hipError_t (*)(const PlainArgs&, dim3 grid, dim3 block, size_t lds, hipStream_t);

template <class P, class F, int C, int kLevel>
hipError_t launch_coarse(const PlainArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((coarse_kernel<P, F, C, kLevel>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <class P, class F, int kLevel>
CoarseLaunch coarse_entry(int C) {
    switch (C) {
        case 1: return &launch_coarse<P, F, 1, kLevel>;
        case 2: return &launch_coarse<P, F, 2, kLevel>;
        case 4: return &launch_coarse<P, F, 4, kLevel>;
        case 8: return &launch_coarse<P, F, 8, kLevel>;
        case 16: return &launch_coarse<P, F, 16, kLevel>;
        default: return nullptr;
    }
}

// float64 H.v at n = 16 on register-resident points (the L1 mapping with a
// point's rows on one 16-lane row), Rosenbrock and Ackley.
using Row16Launch = hipError_t (*)(const Row16Args&, dim3 grid, hipStream_t);

template <class P, class F, int C>
hipError_t launch_row16(const Row16Args& a, dim3 grid, hipStream_t s) {
    if constexpr (std::is_same<F, Ackley>::value) {
        // kAckleyRow16Points points per workgroup
        const dim3 g((unsigned)((a.npts + kAckleyRow16Points - 1) / kAckleyRow16Points));
        hipLaunchKernelGGL((row16_ackley_kernel<P, C>), g, dim3(kRow16Threads), 0, s, a);
    } else {
        hipLaunchKernelGGL((row16_kernel<P, F, C>), grid, dim3(kRow16Threads), 0, s, a);
    }
    return hipGetLastError();
}

template <class P, class F>
Row16Launch row16_entry(int C) {
    switch (C) {
        case 1: return &launch_row16<P, F, 1>;
        case 2: return &launch_row16<P, F, 2>;
        case 4: return &launch_row16<P, F, 4>;
        case 8: return &launch_row16<P, F, 8>;
        case 16: return &launch_row16<P, F, 16>;
        default: return nullptr;
    }
}
Row16Launch row16_rosenbrock(int C);
Row16Launch row16_ackley(int C);
Row16Launch row16_mixed_rosenbrock(int C);
Row16Launch row16_mixed_ackley(int C);

// Rosenbrock H.v at any n on neighbour loads (L1 mapping)
using RowsLaunch = hipError_t (*)(const Row16Args&, int n, dim3 grid, hipStream_t);
template <class P, int C>
hipError_t launch_rosenbrock_rows(const Row16Args& a, int n, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((rosenbrock_rows_kernel<P, C>), grid, dim3(kRow16Threads), 0, s, a, n);
    return hipGetLastError();
}
template <class P>
RowsLaunch rosenbrock_rows_entry(int C) {
    switch (C) {
        case 1: return &launch_rosenbrock_rows<P, 1>;
        case 2: return &launch_rosenbrock_rows<P, 2>;
        case 4: return &launch_rosenbrock_rows<P, 4>;
        case 8: return &launch_rosenbrock_rows<P, 8>;
        case 16: return &launch_rosenbrock_rows<P, 16>;
        default: return nullptr;
    }
}
RowsLaunch rosenbrock_rows(int C);
RowsLaunch rosenbrock_rows_mixed(int C);

// float64 H.v that also stores the gradient and f, one per function.
PlainLaunch grad_rosenbrock(int C);
PlainLaunch grad_ackley(int C);
PlainLaunch grad_fletcher_powell(int C);

// The coarser L0 / L1 mappings of H.v, one per function and precision.
CoarseLaunch coarse_rosenbrock(int C, int level);
CoarseLaunch coarse_ackley(int C, int level);
CoarseLaunch coarse_fletcher_powell(int C, int level);
CoarseLaunch coarse_mixed_rosenbrock(int C, int level);
CoarseLaunch coarse_mixed_ackley(int C, int level);
CoarseLaunch coarse_mixed_fletcher_powell(int C, int level);

using FpMfmaLaunch = hipError_t (*)(const FpMfmaArgs&, dim3 grid, dim3 block, hipStream_t);

template <class P, int C, int NK, bool kHess, bool kSym>
hipError_t launch_fp_mfma(const FpMfmaArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    hipLaunchKernelGGL((fp_mfma_kernel<P, C, NK, kHess, kSym>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class P, int NK, bool kHess, bool kSym>
FpMfmaLaunch fp_mfma_entry_c(int C) {
    switch (C) {
        case 1: return &launch_fp_mfma<P, 1, NK, kHess, kSym>;
        case 2: return &launch_fp_mfma<P, 2, NK, kHess, kSym>;
        case 4: return &launch_fp_mfma<P, 4, NK, kHess, kSym>;
        case 8: return &launch_fp_mfma<P, 8, NK, kHess, kSym>;
        case 16: return &launch_fp_mfma<P, 16, NK, kHess, kSym>;
        default: return nullptr;
    }
}

// K steps of 4 that cover K = 2n, rounded up to 1, 2, 4 or 8.
inline int fp_mfma_steps(int n) {
    const int need = (2 * n + 3) / 4;
    return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

FpMfmaLaunch fp_mfma_entry(int C, int nk, bool hess, bool sym);

template <class P, int NK, bool kHess>
hipError_t launch_fp_tile(const FpMfmaArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    hipLaunchKernelGGL((fp_tile_kernel<P, NK, kHess>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class P, bool kHess>
FpMfmaLaunch fp_tile_by_steps(int nk) {
    switch (nk) {
        case 1: return &launch_fp_tile<P, 1, kHess>;
        case 2: return &launch_fp_tile<P, 2, kHess>;
        case 4: return &launch_fp_tile<P, 4, kHess>;
        case 8: return &launch_fp_tile<P, 8, kHess>;
        default: return nullptr;
    }
}

// The point-tile kernel (n <= 16) for a K-step count and output kind, float64
// and mixed (one translation unit each).
FpMfmaLaunch fp_tile_entry(int nk, bool hess);
FpMfmaLaunch fp_tile_entry_mixed(int nk, bool hess);

template <class P, int NK, int C, bool kHess, bool kGrad, int kN>
hipError_t launch_fp_call(const FpMfmaArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    hipLaunchKernelGGL((fp_call_kernel<P, NK, C, kHess, kGrad, kN>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class P, int NK, bool kHess, bool kGrad, int kN = 0>
FpMfmaLaunch fp_call_entry_c(int C) {
    switch (C) {
        case 1: return &launch_fp_call<P, NK, 1, kHess, kGrad, kN>;
        case 2: return &launch_fp_call<P, NK, 2, kHess, kGrad, kN>;
        case 4: return &launch_fp_call<P, NK, 4, kHess, kGrad, kN>;
        case 8: return &launch_fp_call<P, NK, 8, kHess, kGrad, kN>;
        case 16: return &launch_fp_call<P, NK, 16, kHess, kGrad, kN>;
        default: return nullptr;
    }
}

// H.v at n = 16 has an instance of its own (n a compile-time constant)
template <class P, bool kHess, bool kGrad>
FpMfmaLaunch fp_call_by_steps(int C, int nk, int n) {
    if constexpr (!kHess && !kGrad)
        if (n == 16) return fp_call_entry_c<P, 8, false, false, 16>(C);
    switch (nk) {
        case 1: return fp_call_entry_c<P, 1, kHess, kGrad>(C);
        case 2: return fp_call_entry_c<P, 2, kHess, kGrad>(C);
        case 4: return fp_call_entry_c<P, 4, kHess, kGrad>(C);
        case 8: return fp_call_entry_c<P, 8, kHess, kGrad>(C);
        default: return nullptr;
    }
}

// The per-call Fletcher-Powell kernel (n <= 16) for a chunk, K-step count and
// output kind: float64 H.v / Hessian, float64 H.v with the gradient and f, and
// mixed precision (one translation unit each).
FpMfmaLaunch fp_call_entry(int C, int nk, bool hess, int n);
FpMfmaLaunch fp_call_entry_grad(int C, int nk, int n);
FpMfmaLaunch fp_call_entry_mixed(int C, int nk, bool hess, int n);

using FpDppLaunch = hipError_t (*)(const FpDppArgs&, dim3 grid, dim3 block, size_t lds, hipStream_t);

template <class P, int C, bool kHess, bool kGrad, bool kSym>
hipError_t launch_fp_dpp(const FpDppArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((fp_dpp_kernel<P, C, kHess, kGrad, kSym>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <class P, bool kHess, bool kGrad, bool kSym = false>
FpDppLaunch fp_dpp_entry_c(int C) {
    switch (C) {
        case 1: return &launch_fp_dpp<P, 1, kHess, kGrad, kSym>;
        case 2: return &launch_fp_dpp<P, 2, kHess, kGrad, kSym>;
        case 4: return &launch_fp_dpp<P, 4, kHess, kGrad, kSym>;
        case 8: return &launch_fp_dpp<P, 8, kHess, kGrad, kSym>;
        case 16: return &launch_fp_dpp<P, 16, kHess, kGrad, kSym>;
        default: return nullptr;
    }
}

// The per-call Fletcher-Powell kernel for n > 16 (DPP lane broadcasts):
// float64 H.v / Hessian, float64 H.v with the gradient and f, mixed
// precision (one translation unit each).
FpDppLaunch fp_dpp_entry(int C, bool hess);
FpDppLaunch fp_dpp_entry_grad(int C);
FpDppLaunch fp_dpp_entry_mixed(int C, bool hess);

// Its symmetric forms: float64 and mixed precision (one translation unit each).
FpDppLaunch fp_dpp_sym_entry(int C, bool hess);
FpDppLaunch fp_dpp_sym_entry_mixed(int C, bool hess);

using FpRowsLaunch = hipError_t (*)(const FpRowsArgs&, dim3 grid, dim3 block, hipStream_t);

template <class P, int C, bool kHess>
hipError_t launch_fp_rows(const FpRowsArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    hipLaunchKernelGGL((fp_rows_kernel<P, C, kHess>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class P, bool kHess>
FpRowsLaunch fp_rows_entry_c(int C) {
    switch (C) {
        case 1: return &launch_fp_rows<P, 1, kHess>;
        case 2: return &launch_fp_rows<P, 2, kHess>;
        case 4: return &launch_fp_rows<P, 4, kHess>;
        case 8: return &launch_fp_rows<P, 8, kHess>;
        case 16: return &launch_fp_rows<P, 16, kHess>;
        default: return nullptr;
    }
}

FpRowsLaunch fp_rows_entry(int C, bool hess, bool mixed);
FpMfmaLaunch fp_mfma_entry_mixed(int C, int nk, bool hess, bool sym);

using SymLaunch = hipError_t (*)(const SymArgs&, dim3 grid, dim3 block, size_t lds, hipStream_t);

template <class P, class F, int C, bool kHess>
hipError_t launch_sym(const SymArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((sym_kernel<P, F, C, kHess>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <class P, class F, bool kHess>
SymLaunch sym_entry(int C) {
    switch (C) {
        case 1: return &launch_sym<P, F, 1, kHess>;
        case 2: return &launch_sym<P, F, 2, kHess>;
        case 4: return &launch_sym<P, F, 4, kHess>;
        case 8: return &launch_sym<P, F, 8, kHess>;
        case 16: return &launch_sym<P, F, 16, kHess>;
        default: return nullptr;
    }
}

// Symmetric vector kernels, one per function (both precisions), each in its
// own translation unit.
SymLaunch sym_rosenbrock(int C, bool hess, bool mixed);
SymLaunch sym_ackley(int C, bool hess, bool mixed);
SymLaunch sym_fletcher_powell(int C, bool hess, bool mixed);

// One per (function, precision), each defined in its own translation unit.
PlainLaunch plain_rosenbrock(int C, bool hess);
PlainLaunch plain_ackley(int C, bool hess);
PlainLaunch plain_fletcher_powell(int C, bool hess);
PlainLaunch mixed_rosenbrock(int C, bool hess);
PlainLaunch mixed_ackley(int C, bool hess);
PlainLaunch mixed_fletcher_powell(int C, bool hess);

}  // namespace chessfad
