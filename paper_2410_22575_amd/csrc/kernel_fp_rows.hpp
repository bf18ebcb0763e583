// Fletcher-Powell on MFMA for any n <= 512: R rows of one point per workgroup.
//
// The residual layer inner_m = sum_j A_mj sin y_j + B_mj cos y_j of every call
// is the product [A B] (n x 2n) . S_call over the derivative components of the
// seeded sin/cos values (kernel_fp_mfma.hpp lists the entries of S).  The S
// columns depend on fewer indices than the call, so each is contracted once
// per workgroup and m tile and shared by every call that uses it:
//   g column of variable k (also the d column of row k)  - factors (cos, -sin)
//   h column of row i (nonzero only for k = i)            - factors (-sin, -cos)
// as 16 x 16 MFMA tiles (16 residual rows m x 16 variables).  A tile's
// columns are nonzero only in the K entries of their own 16 variables (sin
// and cos part), so a tile contracts those 32 entries in 8 steps of 4; the
// other K steps of the dense product add exact zeros and are not executed
// (at n <= 16 the two coincide).  The tiles, negated into r_m's components,
// go to LDS.
//
// The workgroup takes its calls (i, cs) in passes over blocks of up to
// kFpRowsKB variables: a pass holds the calls of every row of the workgroup
// whose chunk lies in the block (at most kFpRowsCallsPerLane per lane, all
// lanes busy), and per m tile it forms the g columns of the block, the d
// columns of the rows (from the block when there is one pass) and the h
// columns of the rows whose own variable lies in the block.  Each lane then
// evaluates the rest of f for its calls on the vector unit: for every
// residual m in order, the second-order components of r_m * r_m,
//   2 r_m.d r_m.g[l], and on the row's own column
//   r_m.v r_m.h + r_m.d r_m.g + r_m.d r_m.g + r_m.v r_m.h (the product rule),
// added into the call's running sums (in float32 the 16 residuals of an m
// tile are summed plainly and each tile's partial enters a two-sum
// compensated running sum); the own column runs in a sum of its own (two-sum
// per term in float32), which replaces entry l = i - cs at the end.  The residual values r_m = E_m - sum_j A_mj sin x_j + B_mj cos x_j are
// float64 and computed once per point.  H.v: chunk dot with v, then the row
// sums over chunks in chunk order, pass after pass; Hessian: H[p][i][cs + l]
// is stored.
//
// Within a pass a lane takes kFpRowsCallsPerLane calls of one chunk (rows
// t, t + slot, ...) and reads each g entry once for all of them; consecutive
// lanes take consecutive rows, so the lanes of a wave read the same g entries
// (LDS broadcast) and consecutive d and h entries.
#pragma once

#include <stdint.h>

#include <type_traits>

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
    int rows;           // rows per workgroup, fp_rows_per_block(n, C)
    int row_blocks;     // workgroups per point, ceil(n / rows)
    double* grad = nullptr;  // H.v only, optional: [npts][n] gradient
    double* fval = nullptr;  // H.v only, optional: [npts] f
};

constexpr int kFpRowsMaxN = 512;
constexpr int kFpRowsWaves = 4;
constexpr int kFpRowsKB = 128;          // variables of one pass (a multiple of 16 and of every C)
constexpr int kFpRowsMaxRows = 64;
constexpr int kFpRowsCallsPerLane = 2;
constexpr int kFpRowsMaxCalls = 64 * kFpRowsWaves * kFpRowsCallsPerLane;

// Chunks per pass: all of a row's when they span at most kFpRowsKB variables.
__host__ __device__ inline int fp_rows_pass_chunks(int n, int C) {
    const int nc = (n + C - 1) / C;
    return nc < kFpRowsKB / C ? nc : kFpRowsKB / C;
}

// Rows per workgroup: as many as keep a pass's calls within kFpRowsMaxCalls,
// at most kFpRowsMaxRows and n.
__host__ __device__ inline int fp_rows_per_block(int n, int C) {
    const int cpp = fp_rows_pass_chunks(n, C);
    int r = kFpRowsMaxCalls / cpp;
    if (r > kFpRowsMaxRows) r = kFpRowsMaxRows;
    if (r > n) r = n;
    // a lane takes kFpRowsCallsPerLane rows of one chunk: the chunks' row
    // slots must fit the workgroup's lanes
    while (r > 1 && cpp * ((r + kFpRowsCallsPerLane - 1) / kFpRowsCallsPerLane) > 64 * kFpRowsWaves) --r;
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
    double dots[kFpRowsMaxCalls];  // a pass's chunk dots, [chunk][row]
    double rowsum[kFpRowsMaxRows];  // H.v row sums over the passes so far
    T gk[16][kFpRowsKB];           // r_m.g of the variables of the current pass
    T gi[16][kFpRowsMaxRows];      // r_m.d of the workgroup's rows (more than one pass)
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
    const int cpp = fp_rows_pass_chunks(n, C);
    const int npass = (nc + cpp - 1) / cpp;
    const bool one_pass = npass == 1;   // every row's d column is a column of gk
    const int rtiles = (nrows + 15) / 16;
    const T zero = T(0);
    const bool want_grad = !kHess && a.grad != nullptr;

    // -r_m components of S columns col0 .. col0 + 15 (variables or rows) for
    // the residual rows of m tile mt: the g/d columns (h = false) or the h
    // columns (h = true).  Column col0 + c is nonzero only in the two K
    // entries of its own variable (the sin part and the cos part of [A B]), so
    // the tile contracts the 2 x 16 entries of its columns' variables - four K
    // steps over A, then four over B - and no other K step, whose products are
    // all exact zeros.  The eight A-operand values are loaded before the first
    // MFMA.  The lane's B-operand entry of its own column col0 + li lies in K
    // step u_own of each half (4 u + lg = li); every other entry is zero.
    const bool b_lane = ((li - lg) & 3) == 0;
    const int u_own = (li - lg) >> 2;
    auto tile = [&](int mt, int col0, bool h) {
        const int m_op = mt * 16 + li;      // A-operand row of this lane
        T aop[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = col0 + 4 * u + lg;   // variable of this K entry
            const bool ok = m_op < n && kk < n;
            const size_t idx = ok ? (size_t)m_op * n + kk : 0;
            aop[u] = ok ? fp_a<T>(a.fp, idx) : zero;
            aop[4 + u] = ok ? fp_b<T>(a.fp, idx) : zero;
        }
        const int var = col0 + li;
        const bool on = b_lane && var < n;
        const double sj = sh.s64[on ? var : 0], cj = sh.c64[on ? var : 0];
        const T b0 = on ? (T)(h ? -sj : cj) : zero;     // sin part
        const T b1 = on ? (T)(h ? -cj : -sj) : zero;    // cos part
        V acc = V{zero, zero, zero, zero};
#pragma unroll
        for (int s = 0; s < 8; ++s) acc = mfma16(aop[s], (s & 3) == u_own ? (s < 4 ? b0 : b1) : zero, acc);
        return acc;
    };

    for (int pass = 0; pass < npass; ++pass) {
        const int jc0 = pass * cpp;                       // first chunk of the pass
        const int ncp = nc - jc0 < cpp ? nc - jc0 : cpp;  // chunks in the pass
        const int kbase = jc0 * C;                        // first variable of the pass
        const int kcount = n - kbase < ncp * C ? n - kbase : ncp * C;
        const int ktiles = (kcount + 15) / 16;
        const int pcalls = nrows * ncp;

        // the lane's calls of this pass: one chunk jc0 + jl, and rows t, t + slot,
        // ... of it, so that the lane reads each g entry once for all its
        // calls; a lane takes as few calls as keep every call of the pass on
        // some lane (slot = ceil(nrows / ceil(pcalls / lanes)))
        const int per_lane = (pcalls + (int)blockDim.x - 1) / (int)blockDim.x;
        const int slot = (nrows + per_lane - 1) / per_lane;
        const int lane_jl = threadIdx.x / slot;
        const bool lane_on = lane_jl < ncp;
        const int jl = lane_on ? lane_jl : 0;
        const int t0 = threadIdx.x - lane_jl * slot;
        const int cs_lane = (jc0 + jl) * C;
        int ci[Q], clo[Q], cdi[Q];
        bool cval[Q], cown[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int t = t0 + q * slot;
            cval[q] = lane_on && t < nrows;
            ci[q] = r0 + (cval[q] ? t : 0);
            cdi[q] = jl * nrows + (cval[q] ? t : 0);   // the call's slot in dots, [chunk][row]
            clo[q] = ci[q] - cs_lane;
            cown[q] = cval[q] && clo[q] >= 0 && clo[q] < C;
        }
        RunSum<T> fh[Q][C];
        RunSum<T> fo[Q];  // the row's own column (product rule in full)
        RunSum<T> fd[Q];  // first-order component (row's first chunk, when asked for)

        for (int mt = 0; mt < mtiles; ++mt) {
            // MFMA phase: the pass's g columns, the rows' d columns (more than
            // one pass) and the h columns of the rows whose own variable lies
            // in the pass; one tile per wave at a time
            const int gtasks = one_pass ? 0 : rtiles;
            const int ntasks = ktiles + gtasks + rtiles;
            __syncthreads();  // the previous phase has finished reading LDS
            for (int t = wave; t < ntasks; t += kFpRowsWaves) {
                T* dst;
                int col0, dcol, stride;
                bool hcol = false;
                if (t < ktiles) {
                    col0 = kbase + 16 * t;
                    dst = &sh.gk[0][0];
                    dcol = 16 * t;
                    stride = kFpRowsKB;
                } else {
                    const int w = t - ktiles;
                    hcol = w >= gtasks;
                    const int rt = hcol ? w - gtasks : w;
                    col0 = r0 + 16 * rt;
                    dst = hcol ? &sh.hi[0][0] : &sh.gi[0][0];
                    dcol = 16 * rt;
                    stride = kFpRowsMaxRows;
                    if (hcol && (col0 + 16 <= kbase || col0 >= kbase + kcount)) continue;
                }
                const V acc = tile(mt, col0, hcol);
#pragma unroll
                for (int r = 0; r < 4; ++r) dst[MfmaTile<T>::row(r, lg) * stride + dcol + li] = -acc[r];
            }
            __syncthreads();
            // vector phase: the second-order components of r_m * r_m for the
            // tile's residuals
            const int mcount = n - mt * 16 < 16 ? n - mt * 16 : 16;
            // NQ calls per lane (NQ = per_lane, uniform over the workgroup)
            auto valu = [&](auto nq) {
                constexpr int NQ = decltype(nq)::value;
                // float32: the tile's residuals are summed plainly and the
                // tile's partial enters the compensated running sum (blocked
                // compensation, one two-sum per 16 terms); float64: term by term
                constexpr bool kTile = sizeof(T) == sizeof(float);
                T part[NQ][C];
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int l = 0; l < C; ++l) part[q][l] = zero;
                const int csl = cs_lane - kbase;
                for (int mm = 0; mm < mcount; ++mm) {
                    const T* gm = &sh.gk[mm][csl];
                    T rd[NQ], rd2[NQ];
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        rd[q] = one_pass ? sh.gk[mm][ci[q]] : sh.gi[mm][ci[q] - r0];
                        rd2[q] = rd[q] + rd[q];   // (2 r.d) r.g = r.d r.g + r.d r.g exactly
                    }
#pragma unroll
                    for (int l = 0; l < C; ++l) {
                        const T g = gm[l];
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            const T pr2 = rd2[q] * g;
                            if constexpr (kTile)
                                part[q][l] += pr2;
                            else
                                fh[q][l].add(pr2);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        if (cown[q]) {
                            const T rv = (T)sh.rvs[mt * 16 + mm], rh = sh.hi[mm][ci[q] - r0], rg = gm[clo[q]];
                            fo[q].add(rv * rh + rd[q] * rg + rd[q] * rg + rv * rh);
                        }
                        if (want_grad && cs_lane == 0 && cval[q]) {
                            const T rv = (T)sh.rvs[mt * 16 + mm];
                            fd[q].add(rv * rd[q] + rd[q] * rv);
                        }
                    }
                }
                if constexpr (kTile) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int l = 0; l < C; ++l) fh[q][l].add(part[q][l]);
                }
            };
            static_assert(Q == 2, "the vector phase takes one or two calls per lane");
            if (lane_on) {
                if (per_lane == 1)
                    valu(std::integral_constant<int, 1>{});
                else
                    valu(std::integral_constant<int, 2>{});
            }
        }

        // per call: store the Hessian chunk, or its dot with v
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (!cval[q]) continue;
            const int i = ci[q], cs = cs_lane;
            T hv[C];
#pragma unroll
            for (int l = 0; l < C; ++l) hv[l] = cown[q] && l == clo[q] ? fo[q].value() : fh[q][l].value();
            if (kHess) {
                double* row = a.out + p * n * n + (int64_t)i * n + cs;
#pragma unroll
                for (int l = 0; l < C; ++l)
                    if (cs + l < n) row[l] = (double)hv[l];
            } else {
                typename P::Dot dot;
#pragma unroll
                for (int l = 0; l < C; ++l)
                    if (cs + l < n) dot.add(hv[l], (T)sh.vv[cs + l]);
                sh.dots[cdi[q]] = dot.get();
                if (want_grad && cs == 0) a.grad[p * n + i] = (double)fd[q].value();
            }
        }
        if (!kHess) {
            // row sums over the pass's chunks, in chunk order, continuing the
            // previous passes' sums (the next pass writes dots only after
            // two more barriers)
            __syncthreads();
            for (int t = threadIdx.x; t < nrows; t += blockDim.x) {
                double s = pass == 0 ? sh.dots[t] : sh.rowsum[t];
                for (int jl = pass == 0 ? 1 : 0; jl < ncp; ++jl) s += sh.dots[jl * nrows + t];
                if (pass + 1 < npass)
                    sh.rowsum[t] = s;
                else
                    a.out[p * n + r0 + t] = s;
            }
        }
    }
}

template <class P, int C, bool kHess>
__global__ __launch_bounds__(64 * kFpRowsWaves) void fp_rows_kernel(FpRowsArgs a) {
    __shared__ FpRowsShared<typename P::T> sh;
    fp_rows_block<P, C, kHess>(a, blockIdx.x, sh);
}

}  // namespace chessfad
