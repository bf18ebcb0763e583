// Symmetric chunked Hessian / Hessian-vector kernel (vector ALU), gfx950.
//
// SCHUNK-HESS (Sec. III.B) and SC-HESS-VEC (Sec. VI) evaluate f only for the
// chunks of a row that start at the row's own chunk b = i / C or after it:
// n (n / C + 1) / 2 calls per point when C divides n (Sec. V) instead of
// n ceil(n / C).  An entry H(i, s) of a later chunk stands in for its mirror
// H(s, i), which no call evaluates:
//   Hessian: the lane writes it to both places;
//   H.v:     it adds H(i, s) v[s] to r(i), as every entry does, and
//            H(i, s) v[i] to r(s).
// Inside a row's own chunk every row evaluates its entries itself, so no
// product is counted twice.
//
// Work decomposition: a workgroup owns `ppb` whole points.  The calls of one
// point are the pairs (b, cn), b <= cn < nc, times the C rows i = b C + ii of
// row block b; one lane per (pair, point, ii), ii fastest and then points, so
// the C lanes of a pair are adjacent and aligned within a wave, and the lanes
// of a wave mostly share a pair (and its chunk cs: the terms of f outside the
// chunk run light).  The workgroup loops over its ppb * C * nc (nc + 1) / 2
// calls in strides of blockDim.x.
//
// H.v reductions, all in LDS and in a fixed order (bitwise reproducible):
//   own(i, cn)  the lane's chunk dot (as in CHESS-VEC), one slot per call,
//               at the call's index within its point
//   mir(b, s)   sum over the C rows of block b of H(i, s) v[i], formed with a
//               reduce-scatter across the pair's C lanes (lane ii ends up with
//               column s = cn C + ii); column s has s / C slots, b < s / C
//   r(k) = sum_{cn >= k / C} own(k, cn) + sum_{b < k / C} mir(b, k).
// Per point that is C nc (nc + 1) / 2 + C nc (nc - 1) / 2 = C nc^2 doubles.
// The mirror products are formed in float64 also under the mixed policy
// (float32 h times float32 v is exact in float64).
#pragma once

#include <stdint.h>

#include "functions.hpp"

namespace chessfad {

struct SymArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] for H.v, [npts][n][n] for the Hessian
    FpParams fp;
    int64_t npts;
    int n;
    int nc;             // ceil(n / C)
    int ppb;            // points per workgroup
    int pstride;        // LDS rows per staged array (>= ppb)
};

constexpr int kSymThreads = 256;
// LDS ceiling for one workgroup of the symmetric kernel
constexpr size_t kSymMaxLds = 64 * 1024;

// Slots of one point's H.v partial sums (C nc^2 doubles, own sums first).
template <int C>
__host__ __device__ inline int sym_slots(int nc) { return C * nc * nc; }

// Index of pair (b, cn), b <= cn, in the order b = 0, 1, ..., cn = b, ..., nc - 1.
__host__ __device__ inline int sym_pair(int b, int cn, int nc) { return b * nc - b * (b - 1) / 2 + (cn - b); }

// Offset of column s's mirror slots within the mirror part of a point.
template <int C>
__host__ __device__ inline int sym_mir_off(int s) {
    const int sb = s / C;
    return C * (sb * (sb - 1) / 2) + (s - sb * C) * sb;
}

// LDS bytes (host and device agree on this layout):
// doubles: partial sums [ppb][C nc^2] (H.v), t0, t1 [pstride][ks],
// isl [pstride][ki]; T: xs, vs [pstride][ks] (per-point rows, aos_stride)
template <class P, class F>
__host__ __device__ inline size_t sym_lds_bytes(int n, int C, int ppb, int pstride, bool hess) {
    using T = typename P::T;
    const int nc = (n + C - 1) / C;
    const size_t red = hess ? 0 : (size_t)ppb * C * nc * nc;
    const size_t ks = aos_stride(n), ki = aos_stride(F::isl_size(n));
    const size_t dbl = red + (F::kTables ? 2 * ks * pstride : 0) + ki * pstride;
    const size_t tt = ks * pstride * (hess ? 1 : 2);
    return dbl * sizeof(double) + tt * sizeof(T);
}

// Sum m[l] over the C adjacent lanes of a pair and leave column l = ii in
// lane ii: at half-width h a lane keeps the half of its columns selected by
// bit h of ii and adds the partner's copy of that half.
template <int C>
CF_DEV double pair_reduce_scatter(double (&m)[C], int ii) {
#pragma unroll
    for (int h = C / 2; h >= 1; h /= 2) {
        const bool up = (ii & h) != 0;
#pragma unroll
        for (int k = 0; k < h; ++k) {
            const double keep = up ? m[k + h] : m[k];
            const double send = up ? m[k] : m[k + h];
            m[k] = keep + __shfl_xor(send, h);
        }
    }
    return m[0];
}

template <class P, class F, int C, bool kHess>
__global__ __launch_bounds__(kSymThreads) void sym_kernel(SymArgs a) {
    using T = typename P::T;
    extern __shared__ double lds[];
    const int n = a.n, nc = a.nc, ps = a.pstride, ppb = a.ppb;
    const int per_point = C * (nc * (nc + 1) / 2);
    const int slots = sym_slots<C>(nc);
    const int64_t p0 = (int64_t)blockIdx.x * ppb;
    const int npb = (int)(a.npts - p0 < ppb ? a.npts - p0 : ppb);

    double* red = lds;  // per point: own sums [per_point], then mirror sums
    double* t0 = red + (kHess ? 0 : (size_t)ppb * slots);
    const int ks = aos_stride(n), ki = aos_stride(F::isl_size(n));
    double* t1 = t0 + (F::kTables ? ks * ps : 0);
    double* isl = t1 + (F::kTables ? ks * ps : 0);
    T* xs = reinterpret_cast<T*>(isl + ki * ps);
    T* vs = xs + ks * ps;

    // 1. stage coordinates (and vectors) in per-point rows, with the
    //    per-coordinate tables
    const double* xg = a.x + p0 * n;
    const double* vg = a.v + p0 * n;
    for (int idx = threadIdx.x; idx < npb * n; idx += blockDim.x) {
        const int pl = idx / n, k = idx - pl * n;
        const double xv = xg[idx];
        xs[pl * ks + k] = (T)xv;
        if (!kHess) vs[pl * ks + k] = (T)vg[idx];
        if (F::kTables) F::tables(xv, t0[pl * ks + k], t1[pl * ks + k]);
    }
    __syncthreads();
    // 2. per-point float64 island values
    const int tasks = F::isl_tasks(n);
    if (tasks) {
        for (int idx = threadIdx.x; idx < npb * tasks; idx += blockDim.x) {
            const int pl = idx / tasks, task = idx - pl * tasks;
            if constexpr (std::is_same<T, double>::value)
                F::island(task, n, xs + pl * ks, t0 + pl * ks, t1 + pl * ks, 1, a.fp, isl + pl * ki);
            else
                F::island(task, n, xg + (size_t)pl * n, t0 + pl * ks, t1 + pl * ks, 1, a.fp, isl + pl * ki);
        }
        __syncthreads();
    }

    // 3. the calls; every lane runs the same number of iterations, so the
    //    pair reductions always see all lanes of the wave
    const int total = npb * per_point;  // a multiple of C: pairs never straddle the end
    for (int base = 0; base < total; base += blockDim.x) {
        // t -> (pair, point, ii), ii fastest and then points: the lanes of a
        // wave share a pair (b, cn) across points, so they share the chunk
        // cs and f's terms outside it run light
        const int t = base + threadIdx.x;
        const bool in_range = t < total;
        const int tt = in_range ? t : 0;
        const int ii = tt % C;
        const int rest = tt / C;
        const int pair0 = rest / npb;
        const int pl = rest - pair0 * npb;
        const int local = pair0 * C + ii;
        int pair = pair0;
        int b = 0;
        while (pair >= nc - b) {
            pair -= nc - b;
            ++b;
        }
        const int cn = b + pair;
        const int i = b * C + ii, cs = cn * C;
        const bool active = in_range && i < n;
        const bool mirrored = cn > b;

        double m[C];
#pragma unroll
        for (int l = 0; l < C; ++l) m[l] = 0.0;
        if (active && !kHess && F::kRowTerms) {
            // H.v of a function whose calls reach their second-order part
            // through a few terms: those terms alone, component by component
            PointView<T> pv{xs + pl * ks, t0 + pl * ks, t1 + pl * ks, isl + pl * ki, n, i, cs};
            T h[C];
            if constexpr (F::kRowTerms) F::template hrow<P, C>(pv, a.fp, h);
            typename P::Dot acc;
#pragma unroll
            for (int l = 0; l < C; ++l)
                if (cs + l < n) acc.add(h[l], vs[pl * ks + cs + l]);
            red[(size_t)pl * slots + local] = acc.get();
            if (mirrored) {
                const double vi = (double)vs[pl * ks + i];
#pragma unroll
                for (int l = 0; l < C; ++l) m[l] = cs + l < n ? (double)h[l] * vi : 0.0;
            }
        } else if (active) {
            PointView<T> pv{xs + pl * ks, t0 + pl * ks, t1 + pl * ks, isl + pl * ki, n, i, cs};
            const HD<T, C> res = F::template eval<P, C>(pv, a.fp);
            if (kHess) {
                double* Hp = a.out + (p0 + pl) * (int64_t)n * n;
                double* row = Hp + (int64_t)i * n + cs;
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
                if (mirrored) {
#pragma unroll
                    for (int l = 0; l < C; ++l)
                        if (cs + l < n) Hp[(int64_t)(cs + l) * n + i] = (double)res.h[l];
                }
            } else {
                typename P::Dot acc;
#pragma unroll
                for (int l = 0; l < C; ++l)
                    if (cs + l < n) acc.add(res.h[l], vs[pl * ks + cs + l]);
                red[(size_t)pl * slots + local] = acc.get();
                if (mirrored) {
                    const double vi = (double)vs[pl * ks + i];
#pragma unroll
                    for (int l = 0; l < C; ++l) m[l] = cs + l < n ? (double)res.h[l] * vi : 0.0;
                }
            }
        }
        if (!kHess) {
            const double s = pair_reduce_scatter<C>(m, ii);
            if (in_range && mirrored && cs + ii < n)
                red[(size_t)pl * slots + per_point + sym_mir_off<C>(cs + ii) + b] = s;
        }
    }

    // 4. H.v: r(k) from the row's own calls, in chunk order, then the
    //    mirror sums of the row blocks before it
    if (!kHess) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < npb * n; idx += blockDim.x) {
            const int pl = idx / n, k = idx - pl * n, kb = k / C, kk = k - kb * C;
            const double* rp = red + (size_t)pl * slots;
            const double* ok = rp + sym_pair(kb, kb, nc) * C + kk;  // pairs (kb, cn) are adjacent
            double s = ok[0];
            for (int cn = kb + 1; cn < nc; ++cn) s += ok[(cn - kb) * C];
            const double* mk = rp + per_point + sym_mir_off<C>(k);
            for (int b = 0; b < kb; ++b) s += mk[b];
            a.out[(p0 + pl) * n + k] = s;
        }
    }
}

}  // namespace chessfad
