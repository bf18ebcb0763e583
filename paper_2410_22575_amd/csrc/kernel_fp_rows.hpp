// Fletcher-Powell on MFMA for any n <= 512: one point per workgroup, calls as
// matrix columns.
//
// The residual layer inner_m = sum_j A_mj sin y_j + B_mj cos y_j of every call
// is the product [A B] (n x 2n) . S_call (2n x (2C + 1)) over the derivative
// components (d, g[l], h[l]) of the seeded sin/cos values (see
// kernel_fp_mfma.hpp for the entries of S).  Here a wave takes 16 calls of
// one point as the 16 MFMA columns and walks the 16-row tiles of m and the
// K = 2n steps of 4; each step loads one [A B] operand per lane and feeds it
// to all component tiles of the pass (dense: every step runs).  Per m tile
// the vector unit forms r_m = E_m - inner_m and the second-order components
// of r_m * r_m and adds them into the call's running f.h[l]; after the last
// tile the four lane groups are summed with two lane exchanges.
//
// A workgroup owns R consecutive rows of one point (R = 64 / nc when nc <= 64,
// else 1): it stages the point's sin/cos(x_j) (float64), its vector and the
// float64 residual values r_m = E_m - sum_j A_mj sin x_j + B_mj cos x_j in
// LDS, its four waves take the R * nc calls 16 at a time, and the row sums
// over chunks (H.v) are formed in chunk order from LDS.  Per m tile the d
// tile is formed first; the g and h tiles follow LB at a time (LB = 8 in
// float32, 4 in float64) to bound the accumulator registers.
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
    int rows;           // rows per workgroup
    int row_blocks;     // workgroups per point, ceil(n / rows)
};

constexpr int kFpRowsMaxN = 512;
constexpr int kFpRowsWaves = 4;
constexpr int kFpRowsMaxCalls = 512;  // rows * nc <= max(64, nc) <= 512

// running sum: plain float64, or float32 with a two-sum low part
template <typename T>
struct RunSum;
template <>
struct RunSum<double> {
    double s = 0.0;
    CF_DEV void add(double t) { s += t; }
    CF_DEV double lane_total() {
        double h = s;
        h += __shfl_xor(h, 16);
        h += __shfl_xor(h, 32);
        return h;
    }
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
    CF_DEV float lane_total() {
        float h = hi, l = lo;
#pragma unroll
        for (int x = 16; x <= 32; x *= 2) {
            const float oh = __shfl_xor(h, x), ol = __shfl_xor(l, x);
            float s, e;
            two_sum(h, oh, s, e);
            h = s;
            l += e + ol;
        }
        return h + l;
    }
};

// LDS of one workgroup (vv and dots are used only for H.v)
struct FpRowsShared {
    double s64[kFpRowsMaxN], c64[kFpRowsMaxN], rvs[kFpRowsMaxN];
    double vv[kFpRowsMaxN];
    double dots[kFpRowsMaxCalls];
};

// One workgroup's share: block blk = (point, row block).  Needs exactly
// 64 * kFpRowsWaves threads.
template <class P, int C, bool kHess>
__device__ __forceinline__ void fp_rows_block(const FpRowsArgs& a, int64_t blk, FpRowsShared& sh) {
    using T = typename P::T;
    using V = typename MfmaTile<T>::V;
    constexpr int LBMAX = sizeof(T) == sizeof(double) ? 4 : 8;
    constexpr int LB = C < LBMAX ? C : LBMAX;
    double* s64 = sh.s64;
    double* c64 = sh.c64;
    double* rvs = sh.rvs;
    double* vv = sh.vv;
    double* dots = sh.dots;

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
        s64[t] = s;
        c64[t] = c;
        if (!kHess) vv[t] = a.v[p * n + t];
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        const double* Am = a.fp.A + (size_t)m * n;
        const double* Bm = a.fp.B + (size_t)m * n;
        double acc = Am[0] * s64[0];
        acc = acc + Bm[0] * c64[0];
        for (int j = 1; j < n; ++j) {
            acc = acc + Am[j] * s64[j];
            acc = acc + Bm[j] * c64[j];
        }
        rvs[m] = a.fp.E[m] - acc;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int mtiles = (n + 15) / 16;
    const int nk = (2 * n + 3) / 4;
    const int groups = (ncalls + 15) / 16;
    const T zero = T(0);

    for (int grp = wave; grp < groups; grp += kFpRowsWaves) {
        const int cl = grp * 16 + li;          // this lane's call within the workgroup
        const bool valid = cl < ncalls;
        const int i = valid ? r0 + cl / nc : -1;
        const int cs = valid ? (cl - (cl / nc) * nc) * C : -8192;

        RunSum<T> fh[C];
        for (int mt = 0; mt < mtiles; ++mt) {
            const int m_op = mt * 16 + li;     // A-operand row of this lane
            // [A B] operand and seeded sin/cos factors of K step s
            auto operands = [&](int s, T& aop, T& g1, T& g2, int& jm) {
                const int k = 4 * s + lg;
                const bool in = k < 2 * n;
                const int j = k < n ? k : k - n;
                aop = g1 = g2 = zero;
                if (in) {
                    if (m_op < n) aop = k < n ? fp_a<T>(a.fp, (size_t)m_op * n + k) : fp_b<T>(a.fp, (size_t)m_op * n + j);
                    const double sj = s64[j], cj = c64[j];
                    g1 = (T)(k < n ? cj : -sj);
                    g2 = (T)(k < n ? -sj : -cj);
                }
                jm = in ? j : -1;
            };
            V ad = {zero, zero, zero, zero};
            for (int s = 0; s < nk; ++s) {
                T aop, g1, g2;
                int jm;
                operands(s, aop, g1, g2, jm);
                ad = mfma16(aop, jm == i ? g1 : zero, ad);
            }
            T rv[4], rd[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = mt * 16 + MfmaTile<T>::row(r, lg);
                rv[r] = m < n ? (T)rvs[m] : zero;
                rd[r] = -ad[r];
            }
#pragma unroll
            for (int lb = 0; lb < C; lb += LB) {
                V ag[LB], ah[LB];
#pragma unroll
                for (int l = 0; l < LB; ++l) ag[l] = ah[l] = V{zero, zero, zero, zero};
                for (int s = 0; s < nk; ++s) {
                    T aop, g1, g2;
                    int jm;
                    operands(s, aop, g1, g2, jm);
#pragma unroll
                    for (int l = 0; l < LB; ++l) {
                        const bool col = jm == cs + lb + l;
                        ag[l] = mfma16(aop, col ? g1 : zero, ag[l]);
                        ah[l] = mfma16(aop, (col && jm == i) ? g2 : zero, ah[l]);
                    }
                }
                // second-order components of r_m * r_m for this lane's rows m
                // (rows m >= n have rv = rd = rg = rh = 0 and add nothing)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
#pragma unroll
                    for (int l = 0; l < LB; ++l) {
                        const T rg = -ag[l][r], rh = -ah[l][r];
                        fh[lb + l].add(rv[r] * rh + rd[r] * rg + rd[r] * rg + rv[r] * rh);
                    }
                }
            }
        }
        T h[C];
#pragma unroll
        for (int l = 0; l < C; ++l) h[l] = fh[l].lane_total();

        if (valid && lg == 0) {
            if (kHess) {
                double* row = a.out + p * n * n + (int64_t)i * n + cs;
#pragma unroll
                for (int l = 0; l < C; ++l)
                    if (cs + l < n) row[l] = (double)h[l];
            } else {
                typename P::Dot dot;
#pragma unroll
                for (int l = 0; l < C; ++l)
                    if (cs + l < n) dot.add(h[l], (T)vv[cs + l]);
                dots[cl] = dot.get();
            }
        }
    }
    if (!kHess) {
        __syncthreads();
        for (int t = threadIdx.x; t < nrows; t += blockDim.x) {
            double s = dots[t * nc];
            for (int jc = 1; jc < nc; ++jc) s += dots[t * nc + jc];
            a.out[p * n + r0 + t] = s;
        }
    }
}

template <class P, int C, bool kHess>
__global__ __launch_bounds__(64 * kFpRowsWaves) void fp_rows_kernel(FpRowsArgs a) {
    __shared__ FpRowsShared sh;
    fp_rows_block<P, C, kHess>(a, blockIdx.x, sh);
}

}  // namespace chessfad
