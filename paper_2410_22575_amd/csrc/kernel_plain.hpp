// Vector-ALU chunked Hessian / Hessian-vector kernel for gfx950.
//
// Work decomposition (the paper's finest GPU mapping, Sec. VI, L2): one lane
// per (point p, row i, chunk j).  A workgroup owns `rows` consecutive row
// tasks of the flattened (p, i) index q = p * n + i, so rows of one point may
// span two workgroups and one workgroup may hold several points; its lanes
// are ordered rows fastest (lane j * rows + r).  Each workgroup:
//   1. stages the coordinates of its points and, for H.v, their vectors into
//      LDS as structure-of-arrays, with the function's per-coordinate
//      transcendental tables (float64);
//   2. computes the per-point float64 island values (one task per thread);
//   3. per lane: evaluates f once on CHUNK-INIT seeds for (i, cs = j * C),
//      entirely in registers, in the precision of the policy P;
//   4. Hessian: writes H[p][i][cs .. cs + C) (columns < n only, CHUNK-HESS);
//      H.v: dots its Hessian chunk with v[p][cs .. cs + C), then the row's
//      nc partial sums are added in chunk order in float64 (CHESS-VEC).
//      The terms of f outside the chunk run light (HD<T, 0>), as in the
//      coarse kernels: a wave's lanes share a chunk when rows >= 64.
// coarse_kernel runs the paper's coarser mappings L1 and L0 on the same
// staging.  There the lanes of a wave are at the same chunk, so the terms of
// f whose variables lie outside the chunk run on HD<T, 0> (their g and h
// components are exact zeros; see the functions' eval).
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
    int pstride;        // LDS rows per staged array (>= points per workgroup)
    double* grad = nullptr;  // kGrad kernels: [npts][n] gradient (row i's d component)
    double* fval = nullptr;  // kGrad kernels, optional: [npts] f (the value component)
    int io32 = 0;            // H.v: x, v and out are float32 (batched instances)
};

constexpr int kMaxBlock = 512;

// LDS bytes for one workgroup (host and device agree on this layout):
// doubles: red[block], t0, t1 [pstride][ks], isl [pstride][ki]; T: xs, vs
// [pstride][ks], with ks = aos_stride(n) and ki = aos_stride(isl_size(n))
template <class P, class F>
__host__ __device__ inline size_t plain_lds_bytes(int n, int pstride, int block, bool hess) {
    using T = typename P::T;
    const size_t ks = aos_stride(n), ki = aos_stride(F::isl_size(n));
    const size_t dbl = (size_t)block + (F::kTables ? 2 * ks * pstride : 0) + ki * pstride;
    const size_t tt = ks * pstride * (hess ? 1 : 2);
    return dbl * sizeof(double) + tt * sizeof(T);
}

// The points a workgroup touches, staged in LDS (layout of plain_lds_bytes).
template <typename T>
struct PlainStage {
    double* red;
    double* t0;
    double* t1;
    double* isl;
    T* xs;
    T* vs;
    int ks, ki;   // row lengths: coordinate arrays, islands
};

// Coordinates (and vectors) of the points p0 .. p0 + npb - 1, stored as XT
// in global memory, into the staging rows; then the islands.
template <class P, class F, bool kHess, typename XT>
__device__ __forceinline__ void plain_stage_points(const PlainArgs& a, const PlainStage<typename P::T>& st,
                                                   const XT* x, const XT* v, int64_t p0, int npb) {
    using T = typename P::T;
    const int n = a.n, ks = st.ks, ki = st.ki;
    const XT* xg = x + p0 * n;
    const XT* vg = v + p0 * n;
    for (int idx = threadIdx.x; idx < npb * n; idx += blockDim.x) {
        const int pl = idx / n, k = idx - pl * n;
        const double xv = (double)xg[idx];
        st.xs[pl * ks + k] = (T)xv;
        if (!kHess) st.vs[pl * ks + k] = (T)vg[idx];
        if (F::kTables) F::tables(xv, st.t0[pl * ks + k], st.t1[pl * ks + k]);
    }
    __syncthreads();
    const int tasks = F::isl_tasks(n);
    if (tasks) {
        for (int idx = threadIdx.x; idx < npb * tasks; idx += blockDim.x) {
            const int pl = idx / tasks, task = idx - pl * tasks;
            // the coordinates in float64: the staged row when it holds them
            // (an LDS read), else the input
            if constexpr (std::is_same<T, double>::value)
                F::island(task, n, st.xs + pl * ks, st.t0 + pl * ks, st.t1 + pl * ks, 1, a.fp, st.isl + pl * ki);
            else
                F::island(task, n, xg + (size_t)pl * n, st.t0 + pl * ks, st.t1 + pl * ks, 1, a.fp, st.isl + pl * ki);
        }
        __syncthreads();
    }
}

// Steps 1 and 2 for the points p0 .. p0 + npb - 1: coordinates (and vectors)
// in per-point rows with the per-coordinate tables, then the per-point
// float64 islands.  `nthr` doubles of reduction space come first.
template <class P, class F, bool kHess>
__device__ __forceinline__ PlainStage<typename P::T> plain_stage(const PlainArgs& a, int64_t p0, int npb, int nthr,
                                                                 double* lds) {
    using T = typename P::T;
    const int n = a.n, ps = a.pstride;
    PlainStage<T> st;
    const int ks = aos_stride(n), ki = aos_stride(F::isl_size(n));
    st.ks = ks;
    st.ki = ki;
    st.red = lds;
    st.t0 = st.red + nthr;
    st.t1 = st.t0 + (F::kTables ? ks * ps : 0);
    st.isl = st.t1 + (F::kTables ? ks * ps : 0);
    st.xs = reinterpret_cast<T*>(st.isl + ki * ps);
    st.vs = st.xs + ks * ps;

    // the input type is uniform: one staging loop per type
    if (a.io32)
        plain_stage_points<P, F, kHess>(a, st, reinterpret_cast<const float*>(a.x), reinterpret_cast<const float*>(a.v),
                                        p0, npb);
    else
        plain_stage_points<P, F, kHess>(a, st, a.x, a.v, p0, npb);
    return st;
}

// One workgroup's share of the launch: row tasks [blk * rows, blk * rows + rows).
// Uses the first rows * nc threads; any further threads of the workgroup
// only take part in the barriers.  `lds` holds plain_lds_bytes() bytes.
// kGrad (H.v only) also stores the gradient and f (a.grad, a.fval); it is a
// separate instantiation so that plain H.v keeps its register allocation.
template <class P, class F, int C, bool kHess, bool kGrad = false>
__device__ __forceinline__ void plain_block(const PlainArgs& a, int64_t blk, double* lds) {
    using T = typename P::T;
    const int n = a.n, nc = a.nc;
    const int nthr = a.rows * nc;
    const int64_t nrows = a.npts * (int64_t)n;
    const int64_t q0 = blk * a.rows;
    const int64_t qlast = (q0 + a.rows < nrows ? q0 + a.rows : nrows) - 1;
    const int64_t p0 = q0 / n;
    const int npb = (int)(qlast / n - p0 + 1);  // points touched by this workgroup

    // 1-2. staging and islands
    const PlainStage<T> st = plain_stage<P, F, kHess>(a, p0, npb, nthr, lds);

    // rows fastest, so that the lanes of a wave share a chunk (and the terms
    // of f outside it run light)
    const int r = threadIdx.x % a.rows;
    const int j = threadIdx.x / a.rows;
    const int64_t q = q0 + r;
    const bool active = threadIdx.x < nthr && q <= qlast;
    const int64_t p = q / n;
    const int i = (int)(q - p * n);
    const int pl = (int)(p - p0);
    const int cs = j * C;

    double dot = 0.0;
    if (active && !kHess && !kGrad) {
        PointView<T> pv{st.xs + pl * st.ks, st.t0 + pl * st.ks, st.t1 + pl * st.ks, st.isl + pl * st.ki, n, i, cs};
        // 3-4b. f on the call's seeds, its second-order part dotted with
        // v[p][cs .. cs + C)
        dot = F::template hvp<P, C>(pv, a.fp, st.vs + pl * st.ks);
    } else if (active) {
        PointView<T> pv{st.xs + pl * st.ks, st.t0 + pl * st.ks, st.t1 + pl * st.ks, st.isl + pl * st.ki, n, i, cs};
        // 3. one f evaluation on hDual<C> seeds
        const HD<T, C> res = F::template eval<P, C>(pv, a.fp);
        if (kHess) {
            // 4a. CHUNK-HESS: H[p][i][cs + l] = second-order component l
            double* row = a.out + q * n + cs;
            if (C % 2 == 0 && cs + C <= n && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
                // a whole chunk on a 16-byte boundary: 16-byte stores
                double2* row2 = reinterpret_cast<double2*>(row);
#pragma unroll
                for (int l = 0; l < C / 2; ++l)
                    row2[l] = make_double2((double)res.h[2 * l], (double)res.h[2 * l + 1]);
            } else {
#pragma unroll
                for (int l = 0; l < C; ++l)
                    if (cs + l < n) row[l] = (double)res.h[l];
            }
        } else {
            // 4b. chunk dot with v[p][cs .. cs + C)
            typename P::Dot acc;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) acc.add(res.h[l], st.vs[pl * st.ks + cs + l]);
            dot = acc.get();
            // the first-order and value components of the same call
            if (kGrad && j == 0) {
                a.grad[q] = (double)res.d;
                if (a.fval && i == 0) a.fval[p] = (double)res.v;
            }
        }
    }
    if (!kHess) {
        if (nc == 1) {
            // one chunk per row: the lane holds the row's whole sum
            if (active) st_io(a.out, q, dot, a.io32);
        } else {
            // row sum over the nc chunk lanes, in chunk order
            if (threadIdx.x < nthr) st.red[threadIdx.x] = dot;
            __syncthreads();
            if (active && j == 0) {
                double s = st.red[threadIdx.x];
                for (int k = 1; k < nc; ++k) s += st.red[threadIdx.x + k * a.rows];
                st_io(a.out, q, s, a.io32);
            }
        }
    }
}

// The paper's coarser GPU mappings of CHESS-VEC (Sec. VI), H.v only:
//   L1 (kLevel = 1): one lane per (point, row); it walks the row's chunks in
//                    order and keeps the row sum;
//   L0 (kLevel = 0): one lane per point; it walks every row and chunk.
// The workgroup stages its points as plain_block does; `rows` row tasks per
// workgroup (L0: a multiple of n, so the workgroup owns whole points).
template <class P, class F, int C, int kLevel>
__device__ __forceinline__ void coarse_block(const PlainArgs& a, int64_t blk, double* lds) {
    using T = typename P::T;
    const int n = a.n, nc = a.nc;
    const int64_t nrows = a.npts * (int64_t)n;
    const int64_t q0 = blk * a.rows;
    const int64_t qlast = (q0 + a.rows < nrows ? q0 + a.rows : nrows) - 1;
    const int64_t p0 = q0 / n;
    const int npb = (int)(qlast / n - p0 + 1);
    const PlainStage<T> st = plain_stage<P, F, false>(a, p0, npb, 0, lds);

    // the rows this lane walks: L1 one, L0 all n of its point
    const int64_t qa = kLevel == 1 ? q0 + threadIdx.x : (p0 + threadIdx.x) * n;
    const int64_t qb = kLevel == 1 ? qa + 1 : qa + n;
    if (threadIdx.x >= (kLevel == 1 ? a.rows : a.rows / n) || qa > qlast) return;
    for (int64_t q = qa; q < qb; ++q) {
        const int64_t p = q / n;
        const int i = (int)(q - p * n);
        const int pl = (int)(p - p0);
        double res = 0.0;
        for (int j = 0; j < nc; ++j) {
            const int cs = j * C;
            PointView<T> pv{st.xs + pl * st.ks, st.t0 + pl * st.ks, st.t1 + pl * st.ks, st.isl + pl * st.ki, n, i, cs};
            // f on the call's seeds, its second-order part dotted with v
            res += F::template hvp<P, C>(pv, a.fp, st.vs + pl * st.ks);
        }
        st_io(a.out, q, res, a.io32);
    }
}

template <class P, class F, int C, int kLevel>
__global__ __launch_bounds__(kMaxBlock) void coarse_kernel(PlainArgs a) {
    extern __shared__ double lds[];
    coarse_block<P, F, C, kLevel>(a, blockIdx.x, lds);
}

template <class P, class F, int C, bool kHess, bool kGrad>
__global__ __launch_bounds__(kMaxBlock) void plain_kernel(PlainArgs a) {
    extern __shared__ double lds[];
    plain_block<P, F, C, kHess, kGrad>(a, blockIdx.x, lds);
}

}  // namespace chessfad
