// Fletcher-Powell, 16 < n <= 512: the chunked method per call on the vector
// unit, the chunk's components shared across lanes by DPP row broadcasts.
//
// The call (point p, row i, chunk cs) evaluates f = sum_m r_m * r_m on the
// CHUNK-INIT seeds.  With J_mk = B_mk sin x_k - A_mk cos x_k and
// D_mk = A_mk sin x_k + B_mk cos x_k (the chain rule of sin and cos on seeds
// whose first-order parts sit on one coordinate each) the residual layer
// r_m = E_m - sum_j A_mj sin(y_j) + B_mj cos(y_j) has the components
//   r_m.v = E_m - sum_j A_mj sin x_j + B_mj cos x_j,  r_m.d = J_mi,
//   r_m.g[l] = J_m,cs+l,  r_m.h[l] = [cs + l = i] D_mi,
// and the product rule of the square, summed over the n residuals, gives
//   f.h[l] = sum_m 2 r_m.d r_m.g[l] + [cs + l = i] sum_m 2 r_m.v r_m.h[l].
//
// Mapping: the variables are taken in blocks of 16 and a workgroup's 256
// lanes form 16 rows of 16 lanes.  A lane row is one (point, row block ib):
// lane t holds row i = 16 ib + t and walks its calls in order - the column
// blocks kb and within each the chunks cs = 16 kb + jC (the paper's L1
// mapping, one lane per (point, row)).  In column block kb lane t also holds
// the residual-layer column of variable 16 kb + t, so the call's g components
// J_m,cs+l are the values of lanes jC + l of the same lane row, which
// v_fmac_*_dpp (row_newbcast) reads inside the multiply-add: the product rule
// costs one instruction per product.  Per call and residual the lane forms
// its own r_m.d = J_mi and its column's J_m,16kb+t from A, B (global memory,
// cached: they are shared by every point) and the point's sin x, cos x (LDS),
// then the C products.  The row's own second-order part,
// sum_m r_m.v D_mi, is formed once per row and added in the call that holds
// column i.  H.v: each call's chunk dot with v (v of lane jC + l), the row's
// sum over its calls in order; Hessian: H[p][i][cs + l] is stored.
//
// The value column r_m.v is computed once per point per workgroup (float64)
// and staged in LDS with sin x, cos x and v.  A workgroup holds ppw points
// (16, 4 or 1), each on 16 / ppw lane rows, and the row blocks of its points
// are split over `rsplit` workgroups: few large points still fill the GPU.
//
// Precision policies: F64 runs everything in float64.  F32C forms J from the
// float32 copies of A and B (exact: small integers) and float32 sin, cos,
// sums each call's products over 16 residuals in plain float32 and adds each
// 16-residual partial into a two-sum compensated running sum; r.v, the own
// part, the chunk dot with v (a float32 x float32 product is exact in
// float64) and the row sums stay in float64.
#pragma once

#include <stdint.h>

#include "kernel_fp_call.hpp"

namespace chessfad {

struct FpDppArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] for H.v, [npts][n][n] for the Hessian
    FpParams fp;
    int64_t npts;
    int n;              // 17 .. 512 (any n <= 512 works)
    int nb;             // blocks of 16 variables, ceil(n / 16)
    int ppw;            // points per workgroup: 16, 4 or 1
    int rsplit;         // workgroups per point group (each takes every rsplit-th row block slot)
    double* grad = nullptr;  // H.v only, optional: [npts][n] gradient
    double* fval = nullptr;  // H.v only, optional: [npts] f
};

constexpr int kFpDppThreads = 256;
constexpr int kFpDppMaxStage = 2048;  // ppw * 16 nb: LDS of 4 float64 rows per point = 64 KiB

// LDS bytes of one workgroup: sin x, cos x, r.v and v, ppw rows of 16 nb each
__host__ __device__ inline size_t fp_dpp_lds_bytes(int nb, int ppw) { return (size_t)4 * ppw * 16 * nb * sizeof(double); }

// A and B (float64, or the float32 copies) at element offset `idx`: a
// uniform base and a 32-bit offset, the addressing of a scalar-base load
template <typename T>
CF_DEV const T* fp_a_base(const FpParams& p);
template <>
CF_DEV const double* fp_a_base<double>(const FpParams& p) { return p.A; }
template <>
CF_DEV const float* fp_a_base<float>(const FpParams& p) { return p.A32; }
template <typename T>
CF_DEV const T* fp_b_base(const FpParams& p);
template <>
CF_DEV const double* fp_b_base<double>(const FpParams& p) { return p.B; }
template <>
CF_DEV const float* fp_b_base<float>(const FpParams& p) { return p.B32; }
template <typename T>
CF_DEV T ld_at(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (size_t)(idx * (uint32_t)sizeof(T)));
}

// Per-call accumulation of the C products over the residuals: float64
// directly; float32 in 16-residual blocks added into a two-sum running sum.
template <class Prec, int C>
struct DppCallSum;
template <int C>
struct DppCallSum<F64, C> {
    double acc[C];
    CF_DEV DppCallSum() {
#pragma unroll
        for (int l = 0; l < C; ++l) acc[l] = 0.0;
    }
    CF_DEV double (&block())[C] { return acc; }
    CF_DEV void close_block() {}
    CF_DEV double value(int l) const { return acc[l]; }
};
template <int C>
struct DppCallSum<F32C, C> {
    float blk[C], hi[C], lo[C];
    CF_DEV DppCallSum() {
#pragma unroll
        for (int l = 0; l < C; ++l) blk[l] = hi[l] = lo[l] = 0.0f;
    }
    CF_DEV float (&block())[C] { return blk; }
    CF_DEV void close_block() {
#pragma unroll
        for (int l = 0; l < C; ++l) {
            float s, e;
            two_sum(hi[l], blk[l], s, e);
            hi[l] = s;
            lo[l] += e;
            blk[l] = 0.0f;
        }
    }
    CF_DEV double value(int l) const { return (double)hi[l] + (double)lo[l]; }
};

template <class Prec, int C, bool kHess, bool kGrad>
__global__ __launch_bounds__(kFpDppThreads) void fp_dpp_kernel(FpDppArgs a) {
    using T = typename Prec::T;
    extern __shared__ double lds[];
    const int n = a.n, nb = a.nb, ppw = a.ppw, n16 = 16 * nb;
    double* sins = lds;
    double* coss = sins + ppw * n16;
    double* rvs = coss + ppw * n16;
    double* vs = rvs + ppw * n16;
    const int64_t pg = blockIdx.x / a.rsplit;
    const int rpart = (int)(blockIdx.x - pg * a.rsplit);
    const int64_t p0 = pg * ppw;

    // 1. sin x, cos x and v of the workgroup's points (zeros past n and npts)
    for (int idx = threadIdx.x; idx < ppw * n16; idx += kFpDppThreads) {
        const int ps = idx / n16, k = idx - ps * n16;
        const int64_t p = p0 + ps;
        const bool live = p < a.npts && k < n;
        double s = 0.0, c = 0.0;
        if (live) sincos(a.x[p * n + k], &s, &c);
        sins[idx] = s;
        coss[idx] = c;
        if (!kHess) vs[idx] = live ? a.v[p * n + k] : 0.0;
    }
    __syncthreads();
    // 2. the value column r_m.v (float64), points fastest so that neighbouring
    // lanes read the same row of A and B
    for (int idx = threadIdx.x; idx < ppw * n16; idx += kFpDppThreads) {
        const int m = idx / ppw, ps = idx - m * ppw;
        const int64_t p = p0 + ps;
        double r = 0.0;
        if (m < n && p < a.npts) {
            const double* Am = a.fp.A + (size_t)m * n;
            const double* Bm = a.fp.B + (size_t)m * n;
            const double* sp = sins + ps * n16;
            const double* cp = coss + ps * n16;
            double acc = Am[0] * sp[0];
            acc = acc + Bm[0] * cp[0];
            for (int j = 1; j < n; ++j) {
                acc = acc + Am[j] * sp[j];
                acc = acc + Bm[j] * cp[j];
            }
            r = a.fp.E[m] - acc;
        }
        rvs[ps * n16 + m] = r;
    }
    __syncthreads();
    if (kGrad && a.fval && rpart == 0 && (int)threadIdx.x < ppw) {
        const int64_t p = p0 + threadIdx.x;
        if (p < a.npts) {
            const double* rp = rvs + threadIdx.x * n16;
            double f = rp[0] * rp[0];
            for (int m = 1; m < n; ++m) f += rp[m] * rp[m];
            a.fval[p] = f;
        }
    }

    // 3. the calls: lane row d = (point slot, row-block slot), lane t
    const int d = threadIdx.x >> 4, t = threadIdx.x & 15;
    const int rbw = 16 / ppw;
    const int ps = d / rbw, rs = d - ps * rbw;
    const int64_t p = p0 + ps;
    const bool pt_live = p < a.npts;
    const double* sp = sins + ps * n16;
    const double* cp = coss + ps * n16;
    const double* rp = rvs + ps * n16;
    const double* vp = vs + (kHess ? 0 : ps * n16);
    for (int ib = rpart * rbw + rs; ib < nb; ib += a.rsplit * rbw) {
        const int i = 16 * ib + t;
        const bool row_live = pt_live && i < n;
        const int ia = i < n ? i : 0;   // an in-range column for the loads of padded lanes
        const double si64 = sp[i], ci64 = cp[i];
        const T si = (T)si64, ci = (T)ci64;
        // the row's own second-order part sum_m r_m.v D_mi (and, for the
        // gradient, its first-order part sum_m r_m.v J_mi), float64
        // (sin and cos are staged as zeros past n, which masks padded rows)
        double own = 0.0, gd = 0.0;
        for (int m = 0; m < n; ++m) {
            const double am = ld_at(a.fp.A, (uint32_t)(m * n + ia)), bm = ld_at(a.fp.B, (uint32_t)(m * n + ia));
            const double rv = rp[m];
            own += rv * (am * si64 + bm * ci64);
            if (kGrad) gd += rv * (bm * si64 - am * ci64);
        }
        if (kGrad && row_live) a.grad[p * n + i] = gd + gd;
        const double vi = kHess ? 0.0 : vp[i];
        double row = 0.0;
        for (int kb = 0; kb < nb; ++kb) {
            const int k = 16 * kb + t;
            const int ka = k < n ? k : 0;
            const T sk = (T)sp[k], ck = (T)cp[k];
            const double vk = kHess ? 0.0 : vp[k];
            static_for<16 / C>([&](auto jcc) {
                constexpr int jc = decltype(jcc)::value;
                constexpr int cl = jc * C;   // the chunk's first lane in the row
                const int cs = 16 * kb + cl;
                if (cs >= n) return;
                // the call (i, cs): products r_m.d r_m.g[l] over the residuals
                DppCallSum<Prec, C> sum;
                const T* Ab = fp_a_base<T>(a.fp);
                const T* Bb = fp_b_base<T>(a.fp);
                // J_mi and J_m,k of four residuals; padded lanes have zero
                // sin and cos, so their J entries are zero; residuals past n
                // (the last group) are zero
                auto group = [&](int m0, bool tail) {
                    T g[4], dd[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int m = tail && m0 + u >= n ? n - 1 : m0 + u;
                        const uint32_t mo = (uint32_t)(m * n);
                        const T ai = ld_at(Ab, mo + ia), bi = ld_at(Bb, mo + ia);
                        const T ak = ld_at(Ab, mo + ka), bk = ld_at(Bb, mo + ka);
                        dd[u] = bi * si - ai * ci;
                        g[u] = bk * sk - ak * ck;
                        if (tail && m0 + u >= n) dd[u] = g[u] = T(0);
                    }
                    DppRowProducts<T, C, cl>::run(sum.block(), g, dd);
                };
                int m0 = 0, groups = 0;
                for (; m0 + 4 <= n; m0 += 4) {
                    group(m0, false);
                    // float32: a block of 16 residuals enters the running sum
                    if (++groups == 4) {
                        sum.close_block();
                        groups = 0;
                    }
                }
                if (m0 < n) group(m0, true);
                sum.close_block();
                double h[C];
#pragma unroll
                for (int l = 0; l < C; ++l) h[l] = sum.value(l);
                if constexpr (kHess) {
                    // CHUNK-HESS: H[p][i][cs + l] = 2 (products + [cs + l = i] own)
#pragma unroll
                    for (int l = 0; l < C; ++l) {
                        if (cs + l == i) h[l] += own;
                        h[l] += h[l];
                    }
                    if (row_live) {
                        double* dst = a.out + ((size_t)p * n + i) * n + cs;
#pragma unroll
                        for (int l = 0; l < C; ++l)
                            if (cs + l < n) dst[l] = h[l];
                    }
                } else {
                    // the chunk dot with v (v of lane cl + l), the row sum in call order
                    double dot = 0.0;
                    DppChunkDot<C, cl>::run(dot, vk, h);
                    row += dot;
                }
            });
        }
        if constexpr (!kHess) {
            row += own * vi;
            if (row_live) a.out[p * n + i] = row + row;
        }
    }
}

}  // namespace chessfad
