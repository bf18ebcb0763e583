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
// For one hDual component the 16 x 16 result tile
//   D[m][point] = sum_k [A B][m][k] S_point[k][component]
// comes from v_mfma_f64_16x16x4f64 steps over K = 2n, four K entries per
// step.  The value column is dense (all NK = ceil(2n / 4) steps).  A d, g or
// h column of variable k is nonzero only in K entries k and n + k, which lie
// in two steps; only those two are executed (the others would add exact
// zeros).  Each column of S depends on fewer indices than the call, so each
// tile is contracted once for all the calls that share it:
//   value        depends on the point only        - once per point
//   d            on the row i                     - once per row
//   g[l]         on the variable k = cs + l       - once per variable
//   h[l]         nonzero only for k = i (the second-order part of a seeded
//                sin/cos needs both seeds on one coordinate) - once per row;
//                the other h columns of S are zero and are not contracted.
// Every component of every call is therefore the same sum of the same
// products as when the call contracts its own columns.  The rest of f runs on
// the vector unit, per call: r_m = E_m - inner_m and f = sum_m r_m * r_m,
// forming only the second-order components the output needs (with the zero
// h columns, the terms r_m.v r_m.h[l] drop out).  Each lane
// holds four residual rows m = 4 r + lane / 16 of its column; the sum over m
// finishes with two lane exchanges.  H.v: the chunk dot and the row sum (in
// chunk order) stay in registers; Hessian: H[p][i][cs + l] is stored.
//
// Symmetric form (kSym, SCHUNK-HESS / SC-HESS-VEC): row i walks only the
// chunks from its own chunk i / C onwards.  An entry H(i, s) of a later chunk
// is also stored at H(s, i) (Hessian), or adds H(i, s) v[i] to r(s) through a
// per-point float64 accumulator in LDS (H.v).  Rows run in increasing order,
// so r(s) has all its mirror terms (from rows before s's chunk) by the time
// row s is finished.
//
// Precision policies: F64 runs every step in float64 (v_mfma_f64_16x16x4f64);
// F32C runs the derivative columns on v_mfma_f32_16x16x4f32 with float32
// seeded factors and [A B], keeps the value column and the residual values
// r_m in float64 (their difference E_m - inner_m cancels), sums each lane's
// four residuals in float32 and forms the chunk dot in float64.
//
// Operand layouts (lane l = 0..63), both instructions:
//   A: lane l holds A[l % 16][l / 16];   B: lane l holds B[l / 16][l % 16];
//   D (f64): lane l, element r holds D[4 r + l / 16][l % 16];
//   D (f32): lane l, element r holds D[4 (l / 16) + r][l % 16].
#pragma once

#include <stdint.h>

#include "functions.hpp"

namespace chessfad {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct FpMfmaArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] or [npts][n][n]
    FpParams fp;
    int64_t npts;
    int n;              // <= 16
    int nc;             // chunks per row
    double* grad = nullptr;  // H.v only, optional: [npts][n] gradient
    double* fval = nullptr;  // H.v only, optional: [npts] f
};

constexpr int kFpMaxN = 16;
constexpr int kFpWaves = 4;                 // waves per workgroup
constexpr int kFpPointsPerWave = 16;
constexpr int kFpVStride = kFpMaxN + 1;     // padded LDS row of v

CF_DEV f64x4 mfma16(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
CF_DEV f32x4 mfma16(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// MFMA accumulator type and the residual row held in element r of lane group lg
template <typename T>
struct MfmaTile;
template <>
struct MfmaTile<double> {
    using V = f64x4;
    static CF_DEV int row(int r, int lg) { return 4 * r + lg; }
};
template <>
struct MfmaTile<float> {
    using V = f32x4;
    static CF_DEV int row(int r, int lg) { return 4 * lg + r; }
};

// Both members of each lane pair (l, l ^ 16) or (l, l ^ 32), from the gfx950
// row swaps: v_permlane16_swap exchanges the odd 16-lane rows of its first
// operand with the even rows of its second, v_permlane32_swap the upper half
// of the first with the lower half of the second.  With both operands equal
// to x, lane l gets x from the lower member of its pair in .first and from
// the upper member in .second.
template <int X>
CF_DEV void lane_pair(unsigned x, unsigned& first, unsigned& second) {
    if constexpr (X == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        first = r[0];
        second = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        first = r[0];
        second = r[1];
    }
}
template <int X>
CF_DEV double pair_sum(double h) {
    unsigned l0, l1, h0, h1;
    lane_pair<X>((unsigned)__double2loint(h), l0, l1);
    lane_pair<X>((unsigned)__double2hiint(h), h0, h1);
    return __hiloint2double((int)h0, (int)l0) + __hiloint2double((int)h1, (int)l1);
}
template <int X>
CF_DEV void pair_floats(float x, float& first, float& second) {
    unsigned a, b;
    lane_pair<X>(__float_as_uint(x), a, b);
    first = __uint_as_float(a);
    second = __uint_as_float(b);
}

// Sum over the residual rows of one lane and then across the four lane
// groups: plain float64, or float32 with two-sum compensation.  Every lane
// ends with the same total.
CF_DEV double row_sum4(const double (&t)[4]) {
    double h = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) h += t[r];
    h = pair_sum<16>(h);
    return pair_sum<32>(h);
}
template <int X>
CF_DEV void pair_two_sum(float& hi, float& lo) {
    float h0, h1, l0, l1, s, e;
    pair_floats<X>(hi, h0, h1);
    pair_floats<X>(lo, l0, l1);
    two_sum(h0, h1, s, e);
    hi = s;
    lo = e + (l0 + l1);
}
CF_DEV float row_sum4(const float (&t)[4]) {
    float hi = t[0], lo = 0.0f;
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        float s, e;
        two_sum(hi, t[r], s, e);
        hi = s;
        lo += e;
    }
    pair_two_sum<16>(hi, lo);
    pair_two_sum<32>(hi, lo);
    return hi + lo;
}

template <class P, int C, int NK, bool kHess, bool kSym>
__global__ __launch_bounds__(64 * kFpWaves) void fp_mfma_kernel(FpMfmaArgs a) {
    using T = typename P::T;
    using V = typename MfmaTile<T>::V;
    __shared__ T vs[kHess ? 1 : kFpWaves * kFpPointsPerWave * kFpVStride];
    // mirror sums of the symmetric H.v, one row of kFpVStride per point
    // (float64: one array per lane group, which adds its four residuals' part)
    constexpr int kMirGroups = sizeof(T) == sizeof(double) ? 4 : 1;
    __shared__ double msum[(kSym && !kHess) ? kFpWaves * kMirGroups * kFpPointsPerWave * kFpVStride : 1];

    const int n = a.n, nc = a.nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t pbase = ((int64_t)blockIdx.x * kFpWaves + wave) * kFpPointsPerWave;
    const int64_t p = pbase + li;
    const bool live = p < a.npts;
    const double* xp = a.x + (live ? p : 0) * n;

    // [A B] operand: row m = li, column k = 4 s + lg (zero outside n x 2n)
    double aop64[NK];
    T aop[NK];
    // seeded sin/cos factors of coordinate jj[s] of this lane's point
    T g1[NK], g2[NK];
    double gv[NK];
    int jj[NK];
    // n = 2 NK with NK even: the cos half's step s holds the coordinates of
    // the sin half's step s - NK / 2, so their sin and cos are reused
    const bool halves = NK % 2 == 0 && n == 2 * NK;
    double ssv[NK], csv[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
        const int k = 4 * s + lg;
        const bool in = k < 2 * n;
        const int j = k < n ? k : k - n;
        aop64[s] = (li < n && in) ? (k < n ? a.fp.A[li * n + k] : a.fp.B[li * n + j]) : 0.0;
        aop[s] = (T)aop64[s];
        double sj = 0.0, cj = 0.0;
        if (halves && s >= NK / 2) {
            sj = ssv[s >= NK / 2 ? s - NK / 2 : 0];
            cj = csv[s >= NK / 2 ? s - NK / 2 : 0];
        } else if (in && live) {
            sincos(xp[j], &sj, &cj);
        }
        ssv[s] = sj;
        csv[s] = cj;
        jj[s] = in ? j : -1;
        gv[s] = k < n ? sj : cj;          // value
        g1[s] = (T)(k < n ? cj : -sj);    // first-derivative factor
        g2[s] = (T)(k < n ? -sj : -cj);   // second-derivative factor
    }

    // value column in float64, once per point: r_m = E_m - sum_k [A B][m][k] S[k][value]
    // (rows of the f64 tile: m = 4 r + lg; rv[] is indexed like the T tile)
    T rv[4];
    {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NK; ++s) acc = mfma16(aop64[s], gv[s], acc);
        double r64[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 4 * r + lg;
            r64[r] = m < n ? a.fp.E[m] - acc[r] : 0.0;
        }
        if constexpr (sizeof(T) == sizeof(double)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) rv[r] = (T)r64[r];
        } else {
            // move row 4 r' + lg' of the f64 layout to element r of lane group lg
            // (f32 layout row 4 lg + r): row m lives in lane group m % 4, element m / 4
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 4 * lg + r;
                const int src = (m & 3) * 16 + li;
                double val = 0.0;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const double got = __shfl(r64[rr], src);
                    if (rr == (m >> 2)) val = got;
                }
                rv[r] = (T)val;
            }
        }
    }

    T* vw = vs + wave * kFpPointsPerWave * kFpVStride;
    double* mwave = msum + ((kSym && !kHess) ? wave * kMirGroups * kFpPointsPerWave * kFpVStride : 0);
    // this lane's mirror array: its lane group's (float64) or the wave's
    double* mw = mwave + (kMirGroups == 4 ? lg * kFpPointsPerWave * kFpVStride : 0);
    if (!kHess) {
        // stage the wave's 16 vectors (contiguous in global memory) in LDS
        const double* vg = a.v + pbase * n;
        const int64_t avail = (a.npts - pbase) * n;
        for (int idx = lane; idx < kFpPointsPerWave * n; idx += 64) {
            const int pl = idx / n, k = idx - pl * n;
            vw[pl * kFpVStride + k] = (T)(idx < avail ? vg[idx] : 0.0);
        }
        if (kSym)
            for (int idx = lane; idx < kMirGroups * kFpPointsPerWave * kFpVStride; idx += 64) mwave[idx] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    const T zero = T(0);
    // g column of every variable k: the same in every call whose chunk holds
    // k, whatever the row, so it is contracted once here (r_m.g = -inner_m.g)
    constexpr int KMAX = 2 * NK;  // n <= 2 NK
    T rg[KMAX][4];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        V ag = {zero, zero, zero, zero};
        if (k < n) {
            // only the steps holding K entries k (sin) and n + k (cos) have a
            // nonzero B operand; the others would add exact zeros
            const int s_cos = (n + k) >> 2;
#pragma unroll
            for (int s = 0; s < NK; ++s)
                if (s == (k >> 2) || s == s_cos) ag = mfma16(aop[s], jj[s] == k ? g1[s] : zero, ag);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) rg[k][r] = -ag[r];
    }

    constexpr int KCH = (KMAX + C - 1) / C;  // chunks that can hold a variable
    for (int i = 0; i < n; ++i) {
        // d column (row derivative), shared by the row's chunks, and the one
        // nonzero h column (the row's own variable)
        V dd = {zero, zero, zero, zero}, ah = {zero, zero, zero, zero};
        const int s_sin = i >> 2, s_cos = (n + i) >> 2;   // the steps holding K entries i and n + i
#pragma unroll
        for (int s = 0; s < NK; ++s) {
            if (s == s_sin || s == s_cos) {
                dd = mfma16(aop[s], jj[s] == i ? g1[s] : zero, dd);
                ah = mfma16(aop[s], jj[s] == i ? g2[s] : zero, ah);
            }
        }
        T rd[4], rh[4], rd2[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            rd[r] = -dd[r];
            rh[r] = -ah[r];
            rd2[r] = -(dd[r] + dd[r]);   // 2 r.d, exact: rd2 rg = rd rg + rd rg, one rounding each way
        }
        if (!kHess && !kSym && (a.grad || a.fval)) {
            // first-order (and, once, value) component of f = sum_m r_m * r_m
            T t[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) t[r] = rv[r] * rd[r] + rd[r] * rv[r];
            const T gd = row_sum4(t);
            if (a.grad && live && lg == 0) a.grad[p * n + i] = (double)gd;
            if (a.fval && i == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) t[r] = rv[r] * rv[r];
                const T fv = row_sum4(t);
                if (live && lg == 0) a.fval[p] = (double)fv;
            }
        }

        double row = 0.0;
        const int own = i / C;
        // float64 H.v sums each lane's residual rows into the chunk dots and
        // adds the four lane groups once per row (the same products, summed
        // over m and the columns in another order); in the symmetric form
        // each lane group also keeps its part of the mirror terms.  The
        // Hessian and the float32 symmetric form form every entry first.  In float32
        // the lane's four-row partial is a plain sum and its chunk dot is
        // float64; the lanes' dots meet in float64.
        constexpr bool kLaneDot = !kHess && (!kSym || sizeof(T) == sizeof(double));
        double lane_row = 0.0;
        // fixed trip counts (no early exit) so that rg is indexed statically
#pragma unroll
        for (int jc = 0; jc < KCH; ++jc) {
            if (jc < nc && (!kSym || jc >= own)) {
                const bool mirrored = kSym && jc > own;
                typename P::Dot dot;   // the row's chunk dot, or (float32 lane dots) the lane's
                double lane_dot = 0.0;
#pragma unroll
                for (int l = 0; l < C; ++l) {
                    const int k = jc * C + l;
                    // surplus columns of a ragged last chunk are skipped
                    if (k < KMAX && k < n) {
                        // second-order component l of r * r for this lane's
                        // rows (independent terms: a chain through one
                        // accumulator is slower)
                        T t[4];
                        if (kLaneDot) {
                            // every entry here, the row's own one too: its two
                            // r.v r.h products are added after the chunk.
                            // r.d r.g + r.d r.g = (2 r.d) r.g exactly (doubling
                            // is exact), so one product forms both
#pragma unroll
                            for (int r = 0; r < 4; ++r) t[r] = rd2[r] * rg[k][r];
                        } else if (k == i) {
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                t[r] = rv[r] * rh[r] + rd[r] * rg[k][r] + rd[r] * rg[k][r] + rv[r] * rh[r];
                        } else {
#pragma unroll
                            for (int r = 0; r < 4; ++r) t[r] = rd2[r] * rg[k][r];
                        }
                        if constexpr (kLaneDot && sizeof(T) == sizeof(double)) {
                            const double tl = (t[0] + t[1]) + (t[2] + t[3]);
                            lane_dot += tl * (double)vw[li * kFpVStride + k];
                            // symmetric form: the lane group's part of H(i, k) v[i] for r(k)
                            if (mirrored) mw[li * kFpVStride + k] += tl * (double)vw[li * kFpVStride + i];
                        } else if constexpr (kLaneDot) {
                            // the lane's four residuals summed plainly, the
                            // chunk dot compensated (blocked compensation)
                            const float tl = (t[0] + t[1]) + (t[2] + t[3]);
                            dot.add(tl, vw[li * kFpVStride + k]);
                        } else {
                            // summed over all residual rows
                            const T h = row_sum4(t);
                            if (kHess) {
                                if (live && lg == 0) {
                                    a.out[p * n * n + (int64_t)i * n + k] = (double)h;
                                    if (mirrored) a.out[p * n * n + (int64_t)k * n + i] = (double)h;
                                }
                            } else {
                                dot.add(h, vw[li * kFpVStride + k]);
                                if (mirrored && lg == 0)
                                    mw[li * kFpVStride + k] += (double)h * (double)vw[li * kFpVStride + i];
                            }
                        }
                    }
                }
                if constexpr (kLaneDot && sizeof(T) == sizeof(double)) {
                    if (jc == own) {
                        // the own entry's r.v r.h + ... + r.v r.h: its remaining products
                        double o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = rv[r] * rh[r] + rv[r] * rh[r];
                        lane_dot += ((o[0] + o[1]) + (o[2] + o[3])) * (double)vw[li * kFpVStride + i];
                    }
                    lane_row += lane_dot;
                } else if constexpr (kLaneDot) {
                    if (jc == own) {
                        T o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = rv[r] * rh[r] + rv[r] * rh[r];
                        dot.add((o[0] + o[1]) + (o[2] + o[3]), vw[li * kFpVStride + i]);
                    }
                    lane_row += dot.get();
                }
                else if (!kHess)
                    row += dot.get();
            }
        }
        if constexpr (kLaneDot) row = pair_sum<32>(pair_sum<16>(lane_row));
        if (kSym && !kHess) {
            // r(i)'s mirror terms, from the rows of earlier row blocks (all done)
            double mir = mwave[li * kFpVStride + i];
#pragma unroll
            for (int g = 1; g < kMirGroups; ++g) mir += mwave[(g * kFpPointsPerWave + li) * kFpVStride + i];
            row += mir;
        }
        if (!kHess && live && lg == 0) a.out[p * n + i] = row;
    }
}

}  // namespace chessfad
