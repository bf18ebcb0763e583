// Vector-ALU chunked Hessian / Hessian-vector kernel for gfx950.
//
// Work decomposition (the paper's finest GPU mapping, Sec. VI, L2): one lane
// per (point p, row i, chunk j).  A "row task" (p, i) owns nc = ceil(n / C)
// adjacent lanes; a workgroup owns `rows` consecutive row tasks of the
// flattened (p, i) index q = p * n + i, so rows of one point may span two
// workgroups and one workgroup may hold several points.  Each workgroup:
//   1. stages the coordinates of its points and, for H.v, their vectors into
//      LDS as structure-of-arrays, with the function's per-coordinate
//      transcendental tables (float64);
//   2. computes the per-point float64 island values (one task per thread);
//   3. per lane: evaluates f once on CHUNK-INIT seeds for (i, cs = j * C),
//      entirely in registers, in the precision of the policy P;
//   4. Hessian: writes H[p][i][cs .. cs + C) (columns < n only, CHUNK-HESS);
//      H.v: dots its Hessian chunk with v[p][cs .. cs + C), then the row's
//      nc partial sums are added in chunk order in float64 (CHESS-VEC).
#pragma once

#include <stdint.h>

#include "functions.hpp"

namespace chessfad {

struct PlainArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] for H.v, [npts][n][n] for the Hessian
    FpParams fp;
    int64_t npts;
    int n;              // variables
    int nc;             // chunks per row, ceil(n / C)
    int rows;           // row tasks per workgroup; blockDim.x == rows * nc
    int pstride;        // LDS stride between entries of one point (>= points per workgroup)
};

constexpr int kMaxBlock = 512;

// LDS bytes for one workgroup (host and device agree on this layout):
// doubles: red[block], t0, t1 [n][pstride]; T: xs, vs [n][pstride], isl [isl][pstride]
template <class P, class F>
__host__ __device__ inline size_t plain_lds_bytes(int n, int pstride, int block, bool hess) {
    using T = typename P::T;
    const size_t dbl = (size_t)block + (F::kTables ? 2 * (size_t)n * pstride : 0);
    const size_t tt = (size_t)n * pstride * (hess ? 1 : 2) + (size_t)F::isl_size(n) * pstride;
    return dbl * sizeof(double) + tt * sizeof(T);
}

// One workgroup's share of the launch: row tasks [blk * rows, blk * rows + rows).
// Uses the first rows * nc threads; any further threads of the workgroup
// only take part in the barriers.  `lds` holds plain_lds_bytes() bytes.
template <class P, class F, int C, bool kHess>
__device__ __forceinline__ void plain_block(const PlainArgs& a, int64_t blk, double* lds) {
    using T = typename P::T;
    const int n = a.n, nc = a.nc, ps = a.pstride;
    const int nthr = a.rows * nc;
    const int64_t nrows = a.npts * (int64_t)n;
    const int64_t q0 = blk * a.rows;
    const int64_t qlast = (q0 + a.rows < nrows ? q0 + a.rows : nrows) - 1;
    const int64_t p0 = q0 / n;
    const int npb = (int)(qlast / n - p0 + 1);  // points touched by this workgroup

    double* red = lds;
    double* t0 = red + nthr;
    double* t1 = t0 + (F::kTables ? n * ps : 0);
    T* xs = reinterpret_cast<T*>(t1 + (F::kTables ? n * ps : 0));
    T* vs = xs + n * ps;
    T* isl = vs + (kHess ? 0 : n * ps);

    // 1. stage coordinates (contiguous in global memory) into SoA LDS
    const double* xg = a.x + p0 * n;
    const double* vg = a.v + p0 * n;
    for (int idx = threadIdx.x; idx < npb * n; idx += blockDim.x) {
        const int pl = idx / n, k = idx - pl * n;
        const double xv = xg[idx];
        xs[k * ps + pl] = (T)xv;
        if (!kHess) vs[k * ps + pl] = (T)vg[idx];
        if (F::kTables) F::tables(xv, t0[k * ps + pl], t1[k * ps + pl]);
    }
    __syncthreads();
    // 2. per-point float64 island values
    const int tasks = F::isl_tasks(n);
    if (tasks) {
        for (int idx = threadIdx.x; idx < npb * tasks; idx += blockDim.x) {
            const int pl = idx / tasks, task = idx - pl * tasks;
            F::island(task, n, xg + (size_t)pl * n, t0 + pl, t1 + pl, ps, a.fp, isl + pl);
        }
        __syncthreads();
    }

    const int r = threadIdx.x / nc;
    const int j = threadIdx.x - r * nc;
    const int64_t q = q0 + r;
    const bool active = threadIdx.x < nthr && q <= qlast;
    const int64_t p = q / n;
    const int i = (int)(q - p * n);
    const int pl = (int)(p - p0);
    const int cs = j * C;

    double dot = 0.0;
    if (active) {
        PointView<T> pv{xs + pl, t0 + pl, t1 + pl, isl + pl, ps, n, i, cs};
        // 3. one f evaluation on hDual<C> seeds
        const HD<T, C> res = F::template eval<P, C>(pv, a.fp);
        if (kHess) {
            // 4a. CHUNK-HESS: H[p][i][cs + l] = second-order component l
            double* row = a.out + q * n + cs;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) row[l] = (double)res.h[l];
        } else {
            // 4b. chunk dot with v[p][cs .. cs + C)
            typename P::Dot acc;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) acc.add(res.h[l], vs[(cs + l) * ps + pl]);
            dot = acc.get();
        }
    }
    if (!kHess) {
        // row sum over the nc chunk lanes, in chunk order
        if (threadIdx.x < nthr) red[threadIdx.x] = dot;
        __syncthreads();
        if (active && j == 0) {
            double s = red[threadIdx.x];
            for (int k = 1; k < nc; ++k) s += red[threadIdx.x + k];
            a.out[q] = s;
        }
    }
}

template <class P, class F, int C, bool kHess>
__global__ __launch_bounds__(kMaxBlock) void plain_kernel(PlainArgs a) {
    extern __shared__ double lds[];
    plain_block<P, F, C, kHess>(a, blockIdx.x, lds);
}

}  // namespace chessfad
