// Fletcher-Powell on MFMA for any n <= 512: R rows of one point per workgroup.
//
// The residual layer inner_m = sum_j A_mj sin y_j + B_mj cos y_j of every call
// is the product [A B] (n x 2n) . S_call over the derivative components of the
// seeded sin/cos values (kernel_fp_mfma.hpp lists the entries of S).  The S
// columns depend on fewer indices than the call, so each is contracted once
// per workgroup and m tile and shared by every call that uses it:
//   g column of variable k (also the d column of row k)  - factors (cos, -sin)
//   h column of row i (nonzero only for k = i)            - factors (-sin, -cos)
// as 16 x 16 MFMA tiles (16 residual rows m x 16 variables), dense over
// K = 2n in steps of 4.  The tiles, negated into r_m's components, go to LDS:
// the g columns of a block of up to kFpRowsKB variables at a time, and the
// d and h columns of the workgroup's rows.
//
// Each lane then evaluates the rest of f for whole calls (i, cs) - at most
// kFpRowsCallsPerLane of them - on the vector unit: for every residual m in
// order, the second-order components of r_m * r_m,
//   2 r_m.v r_m.h[l] [cs + l = i] + 2 r_m.d r_m.g[l],
// added into the call's running sums (two-sum compensated in float32).  The
// residual values r_m = E_m - sum_j A_mj sin x_j + B_mj cos x_j are float64
// and computed once per point.  H.v: chunk dot with v, then the row sums over
// chunks in chunk order from LDS; Hessian: H[p][i][cs + l] is stored.
//
// A workgroup owns R = fp_rows_per_block(n, nc) consecutive rows of one point
// (at most 64, and at most 512 calls), so every workgroup of a point forms
// the g columns of all n variables.
#pragma once

#include <stdint.h>

#include "kernel_fp_mfma.hpp"

namespace chessfad {

struct FpRowsArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] or [npts][n][n]
    FpParams fp;
    int64_t npts;
    int n;
    int nc;             // chunks per row
    int rows;           // rows per workgroup, fp_rows_per_block(n, nc)
    int row_blocks;     // workgroups per point, ceil(n / rows)
    double* grad = nullptr;  // H.v only, optional: [npts][n] gradient
    double* fval = nullptr;  // H.v only, optional: [npts] f
};

constexpr int kFpRowsMaxN = 512;
constexpr int kFpRowsWaves = 4;
constexpr int kFpRowsKB = 128;          // variables whose g columns are in LDS at once (a multiple of every C)
constexpr int kFpRowsMaxRows = 64;
constexpr int kFpRowsCallsPerLane = 2;
constexpr int kFpRowsMaxCalls = 64 * kFpRowsWaves * kFpRowsCallsPerLane;

// Rows per workgroup: as many as keep the calls within kFpRowsMaxCalls, at
// most kFpRowsMaxRows and n.
__host__ __device__ inline int fp_rows_per_block(int n, int nc) {
    int r = kFpRowsMaxCalls / nc;
    if (r > kFpRowsMaxRows) r = kFpRowsMaxRows;
    if (r > n) r = n;
    return r < 1 ? 1 : r;
}

// running sum: plain float64, or float32 with a two-sum low part
template <typename T>
struct RunSum;
template <>
struct RunSum<double> {
    double s = 0.0;
    CF_DEV void add(double t) { s += t; }
    CF_DEV double value() const { return s; }
};
template <>
struct RunSum<float> {
    float hi = 0.0f, lo = 0.0f;
    CF_DEV void add(float t) {
        float s, e;
        two_sum(hi, t, s, e);
        hi = s;
        lo += e;
    }
    CF_DEV float value() const { return hi + lo; }
};

// LDS of one workgroup (vv and dots are used only for H.v)
template <typename T>
struct FpRowsShared {
    double s64[kFpRowsMaxN], c64[kFpRowsMaxN], rvs[kFpRowsMaxN];
    double vv[kFpRowsMaxN];
    double dots[kFpRowsMaxCalls];
    T gk[16][kFpRowsKB];           // r_m.g of the variables of the current block
    T gi[16][kFpRowsMaxRows];      // r_m.d of the workgroup's rows (when n > kFpRowsKB)
    T hi[16][kFpRowsMaxRows];      // r_m.h of the rows' own column
};

// One workgroup's share: block blk = (point, row block).  Needs exactly
// 64 * kFpRowsWaves threads.
template <class P, int C, bool kHess>
__device__ __forceinline__ void fp_rows_block(const FpRowsArgs& a, int64_t blk, FpRowsShared<typename P::T>& sh) {
    using T = typename P::T;
    using V = typename MfmaTile<T>::V;
    constexpr int Q = kFpRowsCallsPerLane;

    const int n = a.n, nc = a.nc;
    const int64_t p = blk / a.row_blocks;
    const int r0 = (int)(blk - p * a.row_blocks) * a.rows;
    const int nrows = (r0 + a.rows <= n ? a.rows : n - r0);
    const int ncalls = nrows * nc;
    const double* xp = a.x + p * n;

    // per-point prologue (float64): sin/cos of the coordinates, the vector,
    // then the residual values
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        double s, c;
        sincos(xp[t], &s, &c);
        sh.s64[t] = s;
        sh.c64[t] = c;
        if (!kHess) sh.vv[t] = a.v[p * n + t];
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        const double* Am = a.fp.A + (size_t)m * n;
        const double* Bm = a.fp.B + (size_t)m * n;
        double acc = Am[0] * sh.s64[0];
        acc = acc + Bm[0] * sh.c64[0];
        for (int j = 1; j < n; ++j) {
            acc = acc + Am[j] * sh.s64[j];
            acc = acc + Bm[j] * sh.c64[j];
        }
        sh.rvs[m] = a.fp.E[m] - acc;
    }
    if (!kHess && a.fval && r0 == 0) {
        __syncthreads();
        if (threadIdx.x == 0) {
            // the value component of f = sum_m r_m * r_m, in order
            double f = sh.rvs[0] * sh.rvs[0];
            for (int m = 1; m < n; ++m) f += sh.rvs[m] * sh.rvs[m];
            a.fval[p] = f;
        }
    }

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int mtiles = (n + 15) / 16;
    const int nk = (2 * n + 3) / 4;
    const int kblocks = (n + kFpRowsKB - 1) / kFpRowsKB;
    const bool gi_in_gk = kblocks == 1;  // every row's d column is a column of the one g block
    const int rtiles = (nrows + 15) / 16;
    const T zero = T(0);

    // the lane's calls (i, cs)
    int ci[Q], ccs[Q];
    bool cval[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int cl = threadIdx.x + q * (int)blockDim.x;
        cval[q] = cl < ncalls;
        const int rr = cval[q] ? cl / nc : 0;
        ci[q] = r0 + rr;
        ccs[q] = cval[q] ? (cl - rr * nc) * C : 0;
    }
    RunSum<T> fh[Q][C];
    RunSum<T> fd[Q];  // first-order component (row's first chunk, when asked for)
    const bool want_grad = !kHess && a.grad != nullptr;

    // -r_m components of S columns col0 .. col0 + 15 (variables or rows) for
    // the residual rows of m tile mt: the g/d column (h = false) or the h
    // column (h = true) of each
    // Up to kJ tiles of one m tile share each K step's [A B] operand load and
    // run as independent accumulation chains.
    constexpr int kJ = 2;
    auto tiles = [&](int mt, int count, const int (&col0)[kJ], const bool (&h)[kJ], V (&acc)[kJ]) {
#pragma unroll
        for (int t = 0; t < kJ; ++t) acc[t] = V{zero, zero, zero, zero};
        const int m_op = mt * 16 + li;      // A-operand row of this lane
        for (int s = 0; s < nk; ++s) {
            const int k = 4 * s + lg;
            T aop = zero;
            int j = -1;
            if (k < 2 * n) {
                j = k < n ? k : k - n;
                if (m_op < n) aop = k < n ? fp_a<T>(a.fp, (size_t)m_op * n + k) : fp_b<T>(a.fp, (size_t)m_op * n + j);
            }
            const double sj = j >= 0 ? sh.s64[j] : 0.0, cj = j >= 0 ? sh.c64[j] : 0.0;
#pragma unroll
            for (int t = 0; t < kJ; ++t) {
                if (t < count) {
                    const int var = col0[t] + li;   // B-operand column of this lane
                    T b = zero;
                    if (j == var) b = (T)(h[t] ? (k < n ? -sj : -cj) : (k < n ? cj : -sj));
                    acc[t] = mfma16(aop, b, acc[t]);
                }
            }
        }
    };
    for (int mt = 0; mt < mtiles; ++mt) {
        for (int kb = 0; kb < kblocks; ++kb) {
            const int kbase = kb * kFpRowsKB;
            const int kcount = n - kbase < kFpRowsKB ? n - kbase : kFpRowsKB;
            const int ktiles = (kcount + 15) / 16;
            const int rt_tasks = kb == 0 ? (gi_in_gk ? rtiles : 2 * rtiles) : 0;
            const int ntasks = ktiles + rt_tasks;
            // MFMA phase: the block's g columns, and (first block) the rows' h
            // (and d) columns; the wave's tasks kJ at a time
            __syncthreads();  // the previous phase has finished reading LDS
            for (int t0 = wave; t0 < ntasks; t0 += kFpRowsWaves * kJ) {
                int col0[kJ], count = 0;
                bool hcol[kJ];
                T* dst[kJ];
                int dcol[kJ];
#pragma unroll
                for (int u = 0; u < kJ; ++u) {
                    const int t = t0 + u * kFpRowsWaves;
                    col0[u] = 0;
                    hcol[u] = false;
                    dst[u] = nullptr;
                    dcol[u] = 0;
                    if (t < ntasks) {
                        count = u + 1;
                        if (t < ktiles) {
                            col0[u] = kbase + 16 * t;
                            dst[u] = &sh.gk[0][0];
                            dcol[u] = 16 * t;
                        } else {
                            const int w = t - ktiles;
                            hcol[u] = gi_in_gk || w >= rtiles;
                            const int rt = w < rtiles ? w : w - rtiles;
                            col0[u] = r0 + 16 * rt;
                            dst[u] = hcol[u] ? &sh.hi[0][0] : &sh.gi[0][0];
                            dcol[u] = 16 * rt;
                        }
                    }
                }
                V acc[kJ];
                tiles(mt, count, col0, hcol, acc);
#pragma unroll
                for (int u = 0; u < kJ; ++u) {
                    if (u < count) {
                        const int stride = dst[u] == &sh.gk[0][0] ? kFpRowsKB : kFpRowsMaxRows;
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            dst[u][MfmaTile<T>::row(r, lg) * stride + dcol[u] + li] = -acc[u][r];
                    }
                }
            }
            __syncthreads();
            // vector phase: every call whose chunk lies in this block takes the
            // second-order components of r_m * r_m for the tile's residuals
            const int mcount = n - mt * 16 < 16 ? n - mt * 16 : 16;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = ci[q], cs = ccs[q], il = i - r0;
                if (cval[q] && cs / kFpRowsKB == kb) {
                for (int mm = 0; mm < mcount; ++mm) {
                    const T rd = gi_in_gk ? sh.gk[mm][i - kbase] : sh.gi[mm][il];
                    const T* gm = &sh.gk[mm][cs - kbase];
                    if (want_grad && cs == 0) {
                        const T rv = (T)sh.rvs[mt * 16 + mm];
                        fd[q].add(rv * rd + rd * rv);
                    }
#pragma unroll
                    for (int l = 0; l < C; ++l) {
                        if (cs + l < n) {
                            const T rg = gm[l];
                            if (cs + l == i) {
                                const T rv = (T)sh.rvs[mt * 16 + mm], rh = sh.hi[mm][il];
                                fh[q][l].add(rv * rh + rd * rg + rd * rg + rv * rh);
                            } else {
                                fh[q][l].add(rd * rg + rd * rg);
                            }
                        }
                    }
                }
                }
            }
        }
    }

    // per call: store the Hessian chunk, or its dot with v
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = ci[q], cs = ccs[q];
        if (!cval[q]) {
        } else if (kHess) {
            double* row = a.out + p * n * n + (int64_t)i * n + cs;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) row[l] = (double)fh[q][l].value();
        } else {
            typename P::Dot dot;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) dot.add(fh[q][l].value(), (T)sh.vv[cs + l]);
            sh.dots[threadIdx.x + q * blockDim.x] = dot.get();
            if (want_grad && cs == 0) a.grad[p * n + i] = (double)fd[q].value();
        }
    }
    if (!kHess) {
        __syncthreads();
        for (int t = threadIdx.x; t < nrows; t += blockDim.x) {
            double s = sh.dots[t * nc];
            for (int jc = 1; jc < nc; ++jc) s += sh.dots[t * nc + jc];
            a.out[p * n + r0 + t] = s;
        }
    }
}

template <class P, int C, bool kHess>
__global__ __launch_bounds__(64 * kFpRowsWaves) void fp_rows_kernel(FpRowsArgs a) {
    __shared__ FpRowsShared<typename P::T> sh;
    fp_rows_block<P, C, kHess>(a, blockIdx.x, sh);
}

}  // namespace chessfad
