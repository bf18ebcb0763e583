// Fletcher-Powell, n <= 16: all second-order components of a point as one
// 16 x 16 MFMA tile - the closed form 2 (J^T J + diag(D^T r)), kept as a
// comparison for the chunked method (CHESSFAD_OPT_FP_MFMA = 3); it makes no
// per-call evaluation.
//
// The hDual evaluation of one call (point p, row i, chunk cs) has two layers:
// the residuals r_m = E_m - sum_j A_mj sin(y_j) + B_mj cos(y_j) and
// f = sum_m r_m * r_m.  On the CHUNK-INIT seeds every seeded sin/cos has
// its first-order parts on one coordinate only, so the residual layer gives,
// with J_mj = B_mj sin x_j - A_mj cos x_j,
//   r_m.v    = E_m - sum_j A_mj sin x_j + B_mj cos x_j   (the same in every call)
//   r_m.d    = J_mi                                       (the row's column)
//   r_m.g[l] = J_m,cs+l                                   (the chunk's columns)
//   r_m.h[l] = [cs + l = i] (A_mi sin x_i + B_mi cos x_i)
// and the product rule for r_m * r_m, summed over m, gives the second-order
// component l of the call
//   f.h[l] = sum_m 2 r_m.d r_m.g[l] + [cs + l = i] sum_m 2 r_m.v r_m.h[l].
// Over all calls of a point the first sum is entry (i, cs + l) of J^T J (times
// two, which is exact), one 16 x 16 x 16 product: four v_mfma_f64_16x16x4f64
// steps with J in both operands.  So a wave forms every (row, chunk) block of
// a point at once; the chunk size only names which block of the tile a call
// is, and the results do not depend on it.  The second sum (the row's own
// entry) runs on the vector unit.
//
// Mapping: a wave owns 16 consecutive points.
//   1. Value column, once per point, as in the per-call kernel: lane
//      (li = point, lg) contracts [A B] against its point's sin/cos values on
//      MFMA (D[m][point], m = 4 r + lg); the sin/cos values and r_m go to LDS.
//   2. Per point (the wave's 16 in turn): lane (li, lg) forms J[4 s + lg][li],
//      s < 4, from its column's A, B entries (held in registers for all
//      points) and the point's sin/cos of x_li; four MFMA steps give
//      D[4 r + lg][li] = sum_m J_m,4r+lg J_m,li.
//   3. H.v: (H v)_i = 2 (sum_k D[k][i] v_k + o_i v_i), o_i = sum_m r_m.v r_m.h(i):
//      lane (li = i, lg) takes its four k = 4 r + lg and its four m = 4 s + lg,
//      and the four lane groups are added with two lane exchanges.  D is
//      symmetric (J_mk J_mi = J_mi J_mk), so column i of D is row i of H.
//      Hessian: entry (4 r + lg, li) is 2 (D + [on the diagonal] o) and is stored.
// Operand layouts as in the per-call kernel (lane l = 0..63):
//   A: lane l holds A[l % 16][l / 16];   B: lane l holds B[l / 16][l % 16];
//   D: lane l, element r holds D[4 r + l / 16][l % 16].
// With A = B = J[4 s + lg][li] both operands are the same register: A[i][m] =
// J[m][i] and B[m][k] = J[m][k].
//
// Precision policies: F64 runs everything in float64.  F32C rounds J to
// float32 once and runs the tile on v_mfma_f32_16x16x4f32 (the sum over the
// n <= 16 residuals is one plain float32 block, as in the rows kernel's
// blocked compensation, whose blocks are 16 residuals); the value column, the
// residual values, the own entries and the dot with v stay in float64.  The
// f32 tile's D layout is row 4 lg + r in element r (MfmaTile<float>::row).
#pragma once

#include "kernel_fp_mfma.hpp"

namespace chessfad {

template <class Prec, int NK, bool kHess>
__global__ __launch_bounds__(64 * kFpWaves) void fp_tile_kernel(FpMfmaArgs a) {
    using T = typename Prec::T;
    using V = typename MfmaTile<T>::V;
    constexpr int P = kFpPointsPerWave, S = kFpVStride;
    // per wave: sin and cos of every (point, coordinate), r_m of every
    // (point, residual), v of every (point, coordinate); entries of index
    // n .. 15 are zero
    __shared__ double sins[kFpWaves * P * S], coss[kFpWaves * P * S], rvs[kFpWaves * P * S];
    __shared__ double vs[kHess ? 1 : kFpWaves * P * S];

    const int n = a.n;
    // the wave index is the same in every lane: keep it (and the point loop) scalar
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int64_t pbase = ((int64_t)blockIdx.x * kFpWaves + wave) * P;
    const int64_t p = pbase + li;
    const bool live = p < a.npts;
    const double* xp = a.x + (live ? p : 0) * n;
    double* sw = sins + wave * P * S;
    double* cw = coss + wave * P * S;
    double* rw = rvs + wave * P * S;
    double* vw = vs + (kHess ? 0 : wave * P * S);

    // every global load of the prologue is issued first, so that their
    // latencies overlap: this lane's coordinates, the [A B] operands of the
    // value column, its four vector entries, and its column of A and B
    const bool halves = NK % 2 == 0 && n == 2 * NK;
    double xv[NK], aop[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
        const int k = 4 * s + lg;
        const bool in = k < 2 * n;
        const int j = k < n ? k : k - n;
        aop[s] = (li < n && in) ? (k < n ? a.fp.A[li * n + k] : a.fp.B[li * n + j]) : 0.0;
        xv[s] = (in && live && !(halves && s >= NK / 2)) ? xp[j] : 0.0;
    }
    double vreg[4];
    if (!kHess) {
        // the wave's 16 vectors are contiguous in global memory
        const double* vg = a.v + pbase * n;
        const int64_t avail = (a.npts - pbase) * n;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int idx = lane + 64 * t;
            vreg[t] = (idx < P * n && idx < avail) ? vg[idx] : 0.0;
        }
    }
    double am[4], bm[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int m = 4 * s + lg;
        const bool in = m < n && li < n;
        am[s] = in ? a.fp.A[m * n + li] : 0.0;
        bm[s] = in ? a.fp.B[m * n + li] : 0.0;
    }

    // 1. value column: lane (point li) contracts its sin/cos values
    {
        double ssv[NK], csv[NK];
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NK; ++s) {
            const int k = 4 * s + lg;
            const bool in = k < 2 * n;
            const int j = k < n ? k : k - n;
            double sj = 0.0, cj = 0.0;
            if (halves && s >= NK / 2) {
                sj = ssv[s >= NK / 2 ? s - NK / 2 : 0];
                cj = csv[s >= NK / 2 ? s - NK / 2 : 0];
            } else if (in && live) {
                sincos(xv[s], &sj, &cj);
            }
            ssv[s] = sj;
            csv[s] = cj;
            acc = mfma16(aop[s], k < n ? sj : cj, acc);
            // the lane of sin row k = j stores coordinate j's pair
            if (k < n) {
                sw[li * S + j] = sj;
                cw[li * S + j] = cj;
            }
        }
        // coordinates n .. 15 and residuals n .. 15 read as zeros
        for (int j = n + lg; j < P; j += 4) {
            sw[li * S + j] = 0.0;
            cw[li * S + j] = 0.0;
        }
        double fsum = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 4 * r + lg;
            const double rm = m < n ? a.fp.E[m] - acc[r] : 0.0;
            rw[li * S + m] = rm;
            fsum += rm * rm;
        }
        if (!kHess && a.fval) {
            fsum = pair_sum<32>(pair_sum<16>(fsum));
            if (live && lg == 0) a.fval[p] = fsum;
        }
    }
    if (!kHess) {
        // v in LDS, zero-padded to 16 entries per point
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int idx = lane + 64 * t;
            if (idx < P * n) {
                const int pl = idx / n, k = idx - pl * n;
                vw[pl * S + k] = vreg[t];
            }
        }
        for (int idx = lane; idx < P * (P - n); idx += 64) {
            const int pl = idx / (P - n), k = n + idx - pl * (P - n);
            vw[pl * S + k] = 0.0;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // 2. the point loop; am, bm: this lane's entries of A and B (column li,
    // rows m = 4 s + lg)
    const int ms = (n + 3) >> 2;   // K steps that hold a residual
    const int np = a.npts - pbase < P ? (int)(a.npts - pbase) : P;
    for (int pt = 0; pt < np; ++pt) {
        const double sj = sw[pt * S + li], cj = cw[pt * S + li];
        double jv[4];
        V d = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            jv[s] = bm[s] * sj - am[s] * cj;
            // float32 policy: J rounded once from float64
            if (s < ms) d = mfma16((T)jv[s], (T)jv[s], d);
        }
        // own entry: sum over this lane's residuals of r_m.v r_m.h(li)
        double o = 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) o += rw[pt * S + 4 * s + lg] * (am[s] * sj + bm[s] * cj);
        const int64_t q = pbase + pt;
        if constexpr (kHess) {
            o = pair_sum<32>(pair_sum<16>(o));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = MfmaTile<T>::row(r, lg);
                const double h = i == li ? (double)d[r] + o : (double)d[r];
                if (i < n && li < n) a.out[(q * n + i) * n + li] = h + h;
            }
        } else {
            double part = o * vw[pt * S + li];
#pragma unroll
            for (int r = 0; r < 4; ++r) part += (double)d[r] * vw[pt * S + MfmaTile<T>::row(r, lg)];
            const double row = pair_sum<32>(pair_sum<16>(part));
            if (lg == 0 && li < n) a.out[q * n + li] = row + row;
            if (a.grad) {
                // first-order component: sum_m 2 r_m.v r_m.d
                double g = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s) g += rw[pt * S + 4 * s + lg] * jv[s];
                g = pair_sum<32>(pair_sum<16>(g));
                if (lg == 0 && li < n) a.grad[q * n + li] = g + g;
            }
        }
    }
}

}  // namespace chessfad
