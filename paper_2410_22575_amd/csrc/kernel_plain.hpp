// Plain float64 chunked Hessian / Hessian-vector kernel for gfx950.
//
// Work decomposition (the paper's finest GPU mapping, Sec. VI, L2): one lane
// per (point p, row i, chunk j).  A "row task" (p, i) owns nc = ceil(n / C)
// adjacent lanes; a workgroup owns `rows` consecutive row tasks of the
// flattened (p, i) index q = p * n + i, so rows of one point may span two
// workgroups and one workgroup may hold several points.  Each lane:
//   1. (cooperatively) stages the coordinates of the workgroup's points and,
//      for H.v, their vectors, into LDS as structure-of-arrays, together with
//      the function's per-coordinate transcendental tables;
//   2. evaluates f once on CHUNK-INIT seeds for (i, cs = j * C), entirely in
//      registers;
//   3. Hessian: writes H[p][i][cs .. cs + C) (columns < n only, CHUNK-HESS);
//      H.v: dots its Hessian chunk with v[p][cs .. cs + C), then the row's
//      nc partial sums are added in chunk order (CHESS-VEC) through LDS.
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
    int pstride;        // LDS stride between coordinates (>= points per workgroup)
};

constexpr int kMaxBlock = 512;

// LDS layout, in doubles: xs[n][pstride], vs[n][pstride], t0, t1 [n][pstride],
// red[blockDim].
template <class F, int C, bool kHess>
__global__ __launch_bounds__(kMaxBlock) void plain_kernel(PlainArgs a) {
    extern __shared__ double lds[];
    const int n = a.n, nc = a.nc, ps = a.pstride;
    const int64_t nrows = a.npts * (int64_t)n;
    const int64_t q0 = (int64_t)blockIdx.x * a.rows;
    const int64_t qlast = (q0 + a.rows < nrows ? q0 + a.rows : nrows) - 1;
    const int64_t p0 = q0 / n;
    const int npb = (int)(qlast / n - p0 + 1);  // points touched by this workgroup

    double* xs = lds;
    double* vs = xs + n * ps;
    double* t0 = vs + (kHess ? 0 : n * ps);
    double* t1 = t0 + (F::kTables ? n * ps : 0);
    double* red = t1 + (F::kTables ? n * ps : 0);

    // 1. stage coordinates (contiguous in global memory) into SoA LDS
    const double* xg = a.x + p0 * n;
    const double* vg = a.v + p0 * n;
    for (int idx = threadIdx.x; idx < npb * n; idx += blockDim.x) {
        const int pl = idx / n, k = idx - pl * n;
        const double xv = xg[idx];
        xs[k * ps + pl] = xv;
        if (!kHess) vs[k * ps + pl] = vg[idx];
        if (F::kTables) F::tables(xv, t0[k * ps + pl], t1[k * ps + pl]);
    }
    __syncthreads();

    const int r = threadIdx.x / nc;
    const int j = threadIdx.x - r * nc;
    const int64_t q = q0 + r;
    const bool active = q <= qlast;
    const int64_t p = q / n;
    const int i = (int)(q - p * n);
    const int pl = (int)(p - p0);
    const int cs = j * C;

    double dot = 0.0;
    if (active) {
        PointView pv{xs + pl, t0 + pl, t1 + pl, ps, n, i, cs};
        // 2. one f evaluation on hDual<C> seeds
        const HD<double, C> res = F::template eval<C>(pv, a.fp);
        if (kHess) {
            // 3a. CHUNK-HESS: H[p][i][cs + l] = second-order component l
            double* row = a.out + q * n + cs;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) row[l] = res.h[l];
        } else {
            // 3b. chunk dot with v[p][cs .. cs + C)
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) dot += res.h[l] * vs[(cs + l) * ps + pl];
        }
    }
    if (!kHess) {
        // row sum over the nc chunk lanes, in chunk order
        red[threadIdx.x] = dot;
        __syncthreads();
        if (active && j == 0) {
            double s = red[threadIdx.x];
            for (int k = 1; k < nc; ++k) s += red[threadIdx.x + k];
            a.out[q] = s;
        }
    }
}

}  // namespace chessfad
