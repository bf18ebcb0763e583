// H.v at n = 16 for Rosenbrock and Ackley: the paper's L1 mapping
// (Sec. VI: one lane per (point p, row i), the lane walks the row's chunks in
// order and keeps the row sum), with a point's 16 rows on one 16-lane row of
// the wave.  Lane 16 r + i of a workgroup holds coordinate i of its point:
// x_i and v_i come from one coalesced load (the flattened index q = 16 p + i
// is the lane's own), its table values from its own sin and cos.  A call
// (i, cs) reads the other coordinates' values from their lanes:
//   - Rosenbrock's terms in x_i need x and v of lanes i - 1 and i + 1 (DPP
//     row shifts; at the row's ends the lane's own value, the clamped index
//     of the LDS kernels, whose terms there carry a zero row seed);
//   - Ackley's chunk slots need x_k, the table value -2 pi sin(2 pi x_k) and
//     v_k of lanes k = cs .. cs + C - 1: DPP row broadcasts (row_newbcast:k)
//     inside the FMAs, and the point's two sums over its coordinates are
//     butterflies over the row (row rotations by 8, 4, 2, 1, whose adds give
//     every lane the same value: each step adds a pair in both of its lanes).
// Ackley's kernel runs a wave's 16 points in four such passes and forms each
// point's island in four lanes instead of all sixteen of its row (see
// row16_ackley_kernel).  Nothing is staged in LDS and no lane waits at a
// barrier.  The calls'
// arithmetic is that of the functions' hvp (Rosenbrock: the same row_terms;
// Ackley: the slots' second-order components h_k = F'' S.d S.g_k +
// G'' C.d C.g_k with S.g_k = 2 x_k, C.g_k = -2 pi sin(2 pi x_k), then
// h_k v_k, and the own term), in the same order; only the summation order
// inside Ackley's two sums differs.  Precision policies as the LDS kernels:
// F64 in float64 throughout; F32C with float32 hDual components (x, v and the
// table values rounded where used), float64 islands and a float64 chunk dot
// of the float32 values.
#pragma once

#include <stdint.h>

#include "functions.hpp"

namespace chessfad {

// dot += v_k h_k over the chunk's slots k = cs + l, l = 0 .. C - 1 in order,
// with h_k = x_k (2 F'' S.d) + t1_k (G'' C.d) in T; x_k, t1_k and v_k are read
// from lane k of this lane's 16-lane row (v_k as float64)
template <typename T, int C, int CS>
struct AckleyRow16Slots;

#include "dpp_ackley_row16.inc"

constexpr int kRow16Threads = 256;   // 16 points per workgroup

struct Row16Args {
    const double* x;    // [npts][16]
    const double* v;    // [npts][16]
    double* out;        // [npts][16]
    int64_t npts;
};

// DPP on the two 32-bit halves of a double, or on a float (ctrl: the DPP
// control code); lanes whose source lies outside the row keep `own`
template <int kCtrl>
__device__ __forceinline__ double row16_dpp(double src, double own) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(own), __double2loint(src), kCtrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(own), __double2hiint(src), kCtrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int kCtrl>
__device__ __forceinline__ float row16_dpp(float src, float own) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(own), __float_as_int(src), kCtrl, 0xf, 0xf, false));
}
constexpr int kDppRowShl1 = 0x101;   // lane i reads lane i + 1
constexpr int kDppRowShr1 = 0x111;   // lane i reads lane i - 1
constexpr int kDppRowRor = 0x120;    // + r: lane i reads lane (i - r) mod 16

// sum of a value over the lanes of the 16-lane row, the same in every lane
__device__ __forceinline__ double row16_sum(double a) {
    a += row16_dpp<kDppRowRor + 8>(a, a);
    a += row16_dpp<kDppRowRor + 4>(a, a);
    a += row16_dpp<kDppRowRor + 2>(a, a);
    a += row16_dpp<kDppRowRor + 1>(a, a);
    return a;
}

template <class P, int C>
__device__ __forceinline__ double row16_rosenbrock(double xd, double vd, int i) {
    using T = typename P::T;
    const T xi = (T)xd, vi = (T)vd;
    const T xm = row16_dpp<kDppRowShr1>(xi, xi), xp = row16_dpp<kDppRowShl1>(xi, xi);
    const T vm = row16_dpp<kDppRowShr1>(vi, vi), vp = row16_dpp<kDppRowShl1>(vi, vi);
    double res = 0.0;
    static_for<16 / C>([&](auto jc) {
        constexpr int cs = decltype(jc)::value * C;
        HD<T, 2> tm, tp;
        Rosenbrock::row_terms_at<T, C>(i, 16, cs, xm, xi, xp, tm, tp);
        typename P::Dot acc;
        acc.add(tm.h[0], vm);
        acc.add(tm.h[1], vi);
        acc.add(tp.h[0], vi);
        acc.add(tp.h[1], vp);
        res += acc.get();
    });
    return res;
}

// the calls of row i of one point from its coordinate's x, v and table values
// and the point's island (F', F'', G', G'' of its two sums: isl[1], isl[2],
// isl[4], isl[5] of Ackley::outer)
template <class P, int C>
__device__ __forceinline__ double row16_ackley_calls(double xd, double vd, double t0d, double t1d, double f1d,
                                                     double f2, double g1d, double g2, int i) {
    using T = typename P::T;
    const T xi = (T)xd, t0 = (T)t0d, t1 = (T)t1d, vi = (T)vd;
    const T f1 = (T)f1d, g1 = (T)g1d;
    // the row seed's first-order parts S.d = 2 x_i, C.d = t1_i through F'' and
    // G'' (formed in float64, then rounded); the own term's second-order parts
    // S.h = 2, C.h = -4 pi^2 t0_i
    const T f2d = (T)(f2 * (double)(T(2) * xi)), g2d = (T)(g2 * (double)t1);
    const T own = f1 * T(2) + g1 * (T(-kTwoPi * kTwoPi) * t0);
    double res = 0.0;
    static_for<16 / C>([&](auto jc) {
        constexpr int cs = decltype(jc)::value * C;
        double dot = 0.0;
        AckleyRow16Slots<T, C, cs>::run(dot, xi, t1, (double)vi, f2d + f2d, g2d);
        if (i >= cs && i < cs + C) dot += (double)own * (double)vi;
        res += dot;
    });
    return res;
}

// Ackley: a wave takes 16 points in four passes of four (one point per 16-lane
// row).  The first sweep loads each pass's x and v, forms the table values and
// the point's two sums (row butterflies), and lane (lg, i) keeps the sums of
// point 4 (i / 4) + lg of its row; after it every lane forms the island of one
// point, four lanes per point rather than all sixteen of its row.  The second
// sweep takes each pass's island from lane 4 s of the row and runs the calls.
// The arithmetic is the same as with the island formed in every lane.
constexpr int kAckleyRow16Passes = 4;
constexpr int kAckleyRow16Points = (kRow16Threads / 64) * 4 * kAckleyRow16Passes;   // per workgroup

template <class P, int C>
__global__ __launch_bounds__(kRow16Threads) void row16_ackley_kernel(Row16Args a) {
    constexpr int kPasses = kAckleyRow16Passes;
    const int lane = threadIdx.x & 63, i = lane & 15, lg = lane >> 4;
    const int64_t pw = ((int64_t)blockIdx.x * (kRow16Threads / 64) + (threadIdx.x >> 6)) * (4 * kPasses);
    double xs[kPasses], vs[kPasses], t0s[kPasses], t1s[kPasses];
    double ss = 0.0, cs = 0.0;
#pragma unroll
    for (int s = 0; s < kPasses; ++s) {
        const int64_t q = (pw + 4 * s + lg) * 16 + i;
        // whole points only: a lane past the end belongs to a point past the end
        const bool live = q < a.npts * 16;
        xs[s] = live ? __builtin_nontemporal_load(a.x + q) : 0.5;
        vs[s] = live ? __builtin_nontemporal_load(a.v + q) : 0.0;
        Ackley::tables(xs[s], t0s[s], t1s[s]);
        const double sx = row16_sum(xs[s] * xs[s]), sc = row16_sum(t0s[s]);
        if ((i >> 2) == s) {
            ss = sx;
            cs = sc;
        }
    }
    // the islands in float64 from the float64 inputs
    double isl[6];
    Ackley::outer(16, ss, cs, isl, 1);
#pragma unroll
    for (int s = 0; s < kPasses; ++s) {
        const double f1 = __shfl(isl[1], 4 * s, 16), f2 = __shfl(isl[2], 4 * s, 16);
        const double g1 = __shfl(isl[4], 4 * s, 16), g2 = __shfl(isl[5], 4 * s, 16);
        const double r = row16_ackley_calls<P, C>(xs[s], vs[s], t0s[s], t1s[s], f1, f2, g1, g2, i);
        const int64_t q = (pw + 4 * s + lg) * 16 + i;
        if (q < a.npts * 16) __builtin_nontemporal_store(r, a.out + q);
    }
}

// Rosenbrock's H.v for any n in the same L1 mapping (one lane per (point,
// row i), consecutive lanes consecutive rows): a call (i, cs) needs x and v of
// rows i - 1, i, i + 1 only, so each lane loads those three itself (the
// neighbours' loads hit the lines its neighbour lanes fetch; HBM bytes stay
// those of x, v and the result) - no LDS staging, no barrier.  The index is
// clamped at the point's ends as in the LDS kernels (those terms carry a zero
// row seed).  Every chunk's call is evaluated, in order, by the same
// row_terms code.
template <class P, int C>
__global__ __launch_bounds__(kRow16Threads) void rosenbrock_rows_kernel(Row16Args a, int n) {
    using T = typename P::T;
    const int64_t q = (int64_t)blockIdx.x * kRow16Threads + threadIdx.x;
    if (q >= a.npts * n) return;
    const int i = (int)(q % n);
    const int64_t qm = i > 0 ? q - 1 : q, qp = i + 1 < n ? q + 1 : q;
    const T xm = (T)a.x[qm], xi = (T)a.x[q], xp = (T)a.x[qp];
    const T vm = (T)a.v[qm], vi = (T)a.v[q], vp = (T)a.v[qp];
    const int nc = (n + C - 1) / C;
    double res = 0.0;
    for (int j = 0; j < nc; ++j) {
        HD<T, 2> tm, tp;
        Rosenbrock::row_terms_at<T, C>(i, n, j * C, xm, xi, xp, tm, tp);
        typename P::Dot acc;
        acc.add(tm.h[0], vm);
        acc.add(tm.h[1], vi);
        acc.add(tp.h[0], vi);
        acc.add(tp.h[1], vp);
        res += acc.get();
    }
    a.out[q] = res;
}

// Rosenbrock (one point per 16-lane row)
template <class P, class F, int C>
__global__ __launch_bounds__(kRow16Threads) void row16_kernel(Row16Args a) {
    const int64_t q = (int64_t)blockIdx.x * kRow16Threads + threadIdx.x;
    const int i = threadIdx.x & 15;
    // whole points only: a lane past the end belongs to a point past the end
    const bool live = q < a.npts * 16;
    // every element is read and written once: streaming (non-temporal) accesses
    const double xi = live ? __builtin_nontemporal_load(a.x + q) : 0.5;
    const double vi = live ? __builtin_nontemporal_load(a.v + q) : 0.0;
    const double r = row16_rosenbrock<P, C>(xi, vi, i);
    if (live) __builtin_nontemporal_store(r, a.out + q);
}

}  // namespace chessfad
