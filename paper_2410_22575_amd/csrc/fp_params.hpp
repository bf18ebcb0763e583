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

// float32 copies of A and B (their entries are integers of magnitude <= 100: exact)
static __global__ void fp_to_f32_kernel(int count, const double* A, const double* B, float* A32, float* B32) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    A32[k] = (float)A[k];
    B32[k] = (float)B[k];
}

}  // namespace chessfad
