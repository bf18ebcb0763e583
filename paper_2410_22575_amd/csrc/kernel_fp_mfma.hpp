// Fletcher-Powell with its dense contraction on float64 MFMA (gfx950), n <= 16.
//
// In every call (point p, row i, chunk cs) the residual layer of f is
//   inner_m = sum_j A_mj sin(y_j) + B_mj cos(y_j),   m < n,
// one linear map applied to each hDual component of the 2n seeded values
// sin(y_j), cos(y_j).  Written as a matrix product it is
//   [A B] (n x 2n)  .  S_call (2n x (2C + 2)),
// and the S columns of many calls (and points) can share one MFMA because
// [A B] is the same for all of them.  The entries of S follow from the chain
// rule on the CHUNK-INIT seeds (k indexes the 2n rows, j its coordinate):
//   sin rows (k <  n, j = k):      d: cos x_j [j = i]     g[l]: cos x_j [j = cs+l]
//                                  h[l]: -sin x_j [j = i][j = cs+l]
//   cos rows (k >= n, j = k - n):  d: -sin x_j [j = i]    g[l]: -sin x_j [j = cs+l]
//                                  h[l]: -cos x_j [j = i][j = cs+l]
//   value column: sin x_j (sin rows), cos x_j (cos rows) - the same for every
//   call of a point, so it is contracted once per point.
//
// Mapping: a wave owns 16 consecutive points, one per MFMA column (lane % 16),
// and walks through every call (i, cs) of those points in row-major order.
// For one call and one hDual component the 16 x 16 result tile
//   D[m][point] = sum_k [A B][m][k] S_point[k][component]
// comes from NK = ceil(2n / 4) v_mfma_f64_16x16x4f64 steps over K = 2n
// (dense: every step is executed, whatever the seeds make zero).  The rest of
// f runs on the vector unit: r_m = E_m - inner_m and f = sum_m r_m * r_m,
// forming only the second-order components the output needs.  Each lane
// holds four residual rows m = 4 r + lane / 16 of its column; the sum over m
// finishes with two lane exchanges.  H.v: the chunk dot and the row sum (in
// chunk order) stay in registers; Hessian: H[p][i][cs + l] is stored.
//
// Operand layouts of v_mfma_f64_16x16x4f64 (lane l = 0..63):
//   A: lane l holds A[l % 16][l / 16];   B: lane l holds B[l / 16][l % 16];
//   D: lane l, element r holds D[4 r + l / 16][l % 16].
#pragma once

#include <stdint.h>

#include "functions.hpp"

namespace chessfad {

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct FpMfmaArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] or [npts][n][n]
    FpParams fp;
    int64_t npts;
    int n;              // <= 16
    int nc;             // chunks per row
};

constexpr int kFpMaxN = 16;
constexpr int kFpWaves = 4;                 // waves per workgroup
constexpr int kFpPointsPerWave = 16;
constexpr int kFpVStride = kFpMaxN + 1;     // padded LDS row of v

CF_DEV f64x4 mfma_f64(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

template <int C, int NK, bool kHess>
__global__ __launch_bounds__(64 * kFpWaves) void fp_mfma_kernel(FpMfmaArgs a) {
    __shared__ double vs[kHess ? 1 : kFpWaves * kFpPointsPerWave * kFpVStride];

    const int n = a.n, nc = a.nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t pbase = ((int64_t)blockIdx.x * kFpWaves + wave) * kFpPointsPerWave;
    const int64_t p = pbase + li;
    const bool live = p < a.npts;
    const double* xp = a.x + (live ? p : 0) * n;

    // [A B] operand: row m = li, column k = 4 s + lg (zero outside n x 2n)
    double aop[NK];
    // seeded sin/cos factors of coordinate jj[s] of this lane's point
    double g1[NK], g2[NK], gv[NK];
    int jj[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
        const int k = 4 * s + lg;
        const bool in = k < 2 * n;
        const int j = k < n ? k : k - n;
        aop[s] = (li < n && in) ? (k < n ? a.fp.A[li * n + k] : a.fp.B[li * n + j]) : 0.0;
        double sj = 0.0, cj = 0.0;
        if (in && live) sincos(xp[j], &sj, &cj);
        jj[s] = in ? j : -1;
        gv[s] = k < n ? sj : cj;     // value
        g1[s] = k < n ? cj : -sj;    // first-derivative factor
        g2[s] = k < n ? -sj : -cj;   // second-derivative factor
    }

    // value column, once per point: r_m = E_m - sum_k [A B][m][k] S[k][value]
    double rv[4];
    {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NK; ++s) acc = mfma_f64(aop[s], gv[s], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 4 * r + lg;
            rv[r] = m < n ? a.fp.E[m] - acc[r] : 0.0;
        }
    }

    double* vw = vs + wave * kFpPointsPerWave * kFpVStride;
    if (!kHess) {
        // stage the wave's 16 vectors (contiguous in global memory) in LDS
        const double* vg = a.v + pbase * n;
        const int64_t avail = (a.npts - pbase) * n;
        for (int idx = lane; idx < kFpPointsPerWave * n; idx += 64) {
            const int pl = idx / n, k = idx - pl * n;
            vw[pl * kFpVStride + k] = idx < avail ? vg[idx] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    for (int i = 0; i < n; ++i) {
        // d component (row derivative) of every residual, shared by the row's chunks
        f64x4 dd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NK; ++s) dd = mfma_f64(aop[s], jj[s] == i ? g1[s] : 0.0, dd);
        double rd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) rd[r] = -dd[r];

        double row = 0.0;
        for (int jc = 0; jc < nc; ++jc) {
            const int cs = jc * C;
            double dot = 0.0;
#pragma unroll
            for (int l = 0; l < C; ++l) {
                if (cs + l >= n) break;  // surplus columns of a ragged last chunk
                f64x4 ag = {0.0, 0.0, 0.0, 0.0}, ah = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < NK; ++s) {
                    const bool col = jj[s] == cs + l;
                    ag = mfma_f64(aop[s], col ? g1[s] : 0.0, ag);
                    ah = mfma_f64(aop[s], (col && jj[s] == i) ? g2[s] : 0.0, ah);
                }
                // second-order component l of r * r, summed over this lane's rows
                double h = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double rg = -ag[r], rh = -ah[r];
                    h += rv[r] * rh + rd[r] * rg + rd[r] * rg + rv[r] * rh;
                }
                h += __shfl_xor(h, 16);
                h += __shfl_xor(h, 32);
                if (kHess) {
                    if (live && lg == 0) a.out[p * n * n + (int64_t)i * n + cs + l] = h;
                } else {
                    dot += h * vw[li * kFpVStride + cs + l];
                }
            }
            row += dot;
        }
        if (!kHess && live && lg == 0) a.out[p * n + i] = row;
    }
}

}  // namespace chessfad
