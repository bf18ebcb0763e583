// Fletcher-Powell, n <= 16: the chunked method per call on the vector unit,
// its operands shared across lanes by DPP row broadcasts.
//
// One call (point p, row i, chunk cs) evaluates f = sum_m r_m * r_m on the
// CHUNK-INIT seeds.  The residual layer r_m = E_m - sum_j A_mj sin(y_j) +
// B_mj cos(y_j) gives, with J_mk = B_mk sin x_k - A_mk cos x_k and
// D_mk = A_mk sin x_k + B_mk cos x_k (chain rule of sin and cos on seeds whose
// first-order parts sit on one coordinate each):
//   r_m.v    = E_m - sum_j A_mj sin x_j + B_mj cos x_j   (the same in every call)
//   r_m.d    = J_mi                                       (the row's variable)
//   r_m.g[l] = J_m,cs+l                                   (the chunk's variables)
//   r_m.h[l] = [cs + l = i] D_mi
// and the product rule of the square, summed over m, gives the call's
// second-order components
//   f.h[l] = sum_m 2 r_m.d r_m.g[l] + [cs + l = i] sum_m 2 r_m.v r_m.h[l].
//
// Mapping (the paper's L1: one lane per (point, row), walking the row's
// chunks in order): a point's 16 lanes form one 16-lane row of the wave, lane
// i the row variable i (lanes i >= n carry zeros).  Lane k holds the
// residual-layer column of its own variable, J_mk for m < 16 - which is r.d
// in the calls of row k and r.g in every call whose chunk holds k - and r_k.v.
// A call's g components are the columns of the lanes cs .. cs + C - 1 of the
// same row: DPP row_newbcast reads them inside the FMA (v_fmac_f64_dpp), so
// the product rule runs at one instruction per product with no LDS traffic.
// Per call and residual m the lane forms the C products r_m.d r_m.g[l]; the
// row's own entry adds sum_m r_m.v D_mi (r_m.v broadcast from lane m); then
// the call's terms h[l] v[cs + l] (v broadcast from lane cs + l) are added to
// the row sum column by column, chunk by chunk in order.  The doubling of the product rule is applied once to
// the row's sum (doubling is exact, so this equals doubling every term).
//
// The value column r_m.v is the one dense contraction, [A B] . [sin x; cos x]
// over K = 2n for every point: it runs on MFMA (v_mfma_f64_16x16x4f64, a wave's
// 16 points as the columns) in a prologue, which stages sin x, cos x, r.v and v
// of the wave's points in LDS.  The wave then takes its points four at a time
// (one per 16-lane row).  A and B are staged per workgroup.
//
// Precision policies: F64 runs everything in float64.  F32C rounds J to
// float32 once and forms the C-component products and their sum over the
// n <= 16 residuals in float32 (v_fmac_f32_dpp: one plain float32 block, the
// block size of the rows kernel's compensated sums); r.v, the own entry
// sum_m r.v D, the chunk dot with v and the row sums stay in float64.
#pragma once

#include "kernel_fp_mfma.hpp"

namespace chessfad {

// acc[l] += J[m] (lane cs + l of this lane's 16-lane row) * J[m] (own lane),
// m = 0 .. 15 in order, l = 0 .. C - 1
template <typename T, int C, int CS>
struct DppChunkProducts;
// dot += v (lane cs + l) * h[l], l = 0 .. C - 1 in order
template <int C, int CS>
struct DppChunkDot;
// acc[l] += g[u] (lane cs + l of this lane's 16-lane row) * d[u] (own lane),
// u = 0 .. 3 in order, l = 0 .. C - 1
template <typename T, int C, int CS>
struct DppRowProducts;

#include "dpp_blocks.inc"

constexpr int kFpCallRows = 4;  // points per wave in one pass (one per 16-lane row)

// Waves per SIMD the register budget is cut for: four (128 VGPRs; the
// value column's MFMA results stay in VGPRs), except float64 calls of 16
// columns (and of 8 in the n = 16 instance), whose product sums and J values
// need more (three waves).
template <class Prec, int C, int kN>
constexpr int fp_call_min_waves() {
    return std::is_same<typename Prec::T, double>::value && (C == 16 || (kN && C == 8)) ? 3 : 4;
}

// kN = 16: the instance for n = 16 (n and the chunk count are constants, so
// the bounds guards and index divisions fold); kN = 0: n from the arguments.
template <class Prec, int NK, int C, bool kHess, bool kGrad, int kN>
__global__ __launch_bounds__(64 * kFpWaves, (fp_call_min_waves<Prec, C, kN>())) void fp_call_kernel(FpMfmaArgs a) {
    using T = typename Prec::T;
    constexpr int P = kFpPointsPerWave, S = kFpVStride;
    // per wave: sin x, cos x, r.v and v of each (point, coordinate or
    // residual); entries n .. 15 are zero
    __shared__ double sins[kFpWaves * P * S], coss[kFpWaves * P * S], rvs[kFpWaves * P * S];
    __shared__ double vs[kHess ? 1 : kFpWaves * P * S];
    // A and B as [m][k], zero outside n x n
    __shared__ double as[16 * S], bs[16 * S];

    const int n = kN ? kN : a.n, nc = kN ? (kN + C - 1) / C : a.nc;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int64_t pbase = ((int64_t)blockIdx.x * kFpWaves + wave) * P;
    double* sw = sins + wave * P * S;
    double* cw = coss + wave * P * S;
    double* rw = rvs + wave * P * S;
    double* vw = vs + (kHess ? 0 : wave * P * S);

    {
        const int m = threadIdx.x >> 4, k = threadIdx.x & 15;
        const bool in = m < n && k < n;
        as[m * S + k] = in ? a.fp.A[m * n + k] : 0.0;
        bs[m * S + k] = in ? a.fp.B[m * n + k] : 0.0;
    }

    // 1. value column: lane (li = point, lg) contracts its point's sin/cos
    // values against [A B] (row m = li, column 4 s + lg of [A B])
    {
        const int64_t p = pbase + li;
        const bool live = p < a.npts;
        const double* xp = a.x + (live ? p : 0) * n;
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
                cf_sincos(xv[s], &sj, &cj);
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
        if (kGrad && a.fval) {
            fsum = pair_sum<32>(pair_sum<16>(fsum));
            if (live && lg == 0) a.fval[p] = fsum;
        }
        if (!kHess) {
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
    }
    __syncthreads();

    // 2. the calls: lane (lg, li) is row i = li of point 4 pass + lg
    const int np = a.npts - pbase < P ? (int)(a.npts - pbase) : P;
    for (int pass = 0; pass * kFpCallRows < np; ++pass) {
        const int pt = pass * kFpCallRows + lg;
        const int64_t q = pbase + pt;
        const bool live = pt < np && li < n;
        const double s = sw[pt * S + li], c = cw[pt * S + li];
        const double rv = rw[pt * S + li];   // r_m.v of m = li
        // this lane's variable's column of the residual layer, and D for the
        // row's own second-order part
        T jm[16];
        double dm[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const double am = as[m * S + li], bm = bs[m * S + li];
            jm[m] = (T)(bm * s - am * c);
            dm[m] = am * s + bm * c;
        }
        // the own entry's sum_m r_m.v r_m.h, undoubled
        double own = 0.0;
        dpp_row_dot(own, rv, dm);
        const double vi = kHess ? 0.0 : vw[pt * S + li];
        double row = 0.0;
        static_for<16 / C>([&](auto jcc) {
            constexpr int jc = decltype(jcc)::value;
            constexpr int cs = jc * C;
            if (jc < nc) {
                // the call (i, cs): products r_m.d r_m.g[l] summed over m
                T h[C];
#pragma unroll
                for (int l = 0; l < C; ++l) h[l] = T(0);
                DppChunkProducts<T, C, cs>::run(h, jm);
                double h64[C];
#pragma unroll
                for (int l = 0; l < C; ++l) h64[l] = (double)h[l];
                if constexpr (kHess) {
                    // CHUNK-HESS: H[p][i][cs + l] = 2 (products + [own] r.v r.h)
#pragma unroll
                    for (int l = 0; l < C; ++l) {
                        if (cs + l == li) h64[l] += own;
                        h64[l] += h64[l];
                    }
                    if (live) {
                        double* dst = a.out + (q * n + li) * n + cs;
                        if (C % 2 == 0 && cs + C <= n && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                            double2* d2 = reinterpret_cast<double2*>(dst);
#pragma unroll
                            for (int l = 0; l < C / 2; ++l) d2[l] = make_double2(h64[2 * l], h64[2 * l + 1]);
                        } else {
#pragma unroll
                            for (int l = 0; l < C; ++l)
                                if (cs + l < n) dst[l] = h64[l];
                        }
                    }
                } else {
                    // the call's terms h[l] v[cs + l] (v of lane cs + l) added
                    // to the row sum column by column, in order
                    DppChunkDot<C, cs>::run(row, vi, h64);
                }
            }
        });
        if constexpr (!kHess) {
            row += own * vi;
            if (live) a.out[q * n + li] = row + row;
            if (kGrad) {
                // first-order component: sum_m 2 r_m.v r_m.d
                double jd[16];
#pragma unroll
                for (int m = 0; m < 16; ++m) jd[m] = (double)jm[m];
                double g = 0.0;
                dpp_row_dot(g, rv, jd);
                if (live) a.grad[q * n + li] = g + g;
            }
        }
    }
}

}  // namespace chessfad
