// Fletcher-Powell parameter preparation kernels (float64 offsets E and
// float32 copies of A and B), shared by the parameter registry and the
// batched planner.
#pragma once

#include <hip/hip_runtime.h>

namespace chessfad {

// E_m = sum_j A_mj sin(alpha_j) + B_mj cos(alpha_j), one thread per m, float64
static __global__ void fp_offsets_kernel(int n, const double* A, const double* B, const double* alpha, double* E) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
        double s, c;
        sincos(alpha[j], &s, &c);
        acc += A[(size_t)m * n + j] * s;
        acc += B[(size_t)m * n + j] * c;
    }
    E[m] = acc;
}

// float32 copies of A and B (exact for the integer entries of the test
// problems); `inexact` (optional) is set to 1 if any entry rounds
static __global__ void fp_to_f32_kernel(int count, const double* A, const double* B, float* A32, float* B32,
                                        int* inexact) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const float a = (float)A[k], b = (float)B[k];
    A32[k] = a;
    B32[k] = b;
    if (inexact && ((double)a != A[k] || (double)b != B[k])) atomicOr(inexact, 1);
}

// *flag = 0 (a kernel, not a memset node)
static __global__ void fp_clear_flag_kernel(int* flag) { *flag = 0; }

}  // namespace chessfad
