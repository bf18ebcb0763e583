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
// lanes form 16 lane rows of 16 lanes.  A lane row is one (point, row block
// ib, column block kb) pair: lane t holds row i = 16 ib + t and the calls of
// that row whose chunks lie in kb, cs = 16 kb + jC, in order (the paper's L1
// mapping, one lane per (point, row), with the row's column blocks spread
// over lane rows).  In the pair the lane also holds the residual-layer
// column of variable 16 kb + t, so the call's g components J_m,cs+l are the
// values of lanes jC + l of the same lane row, which v_fmac_*_dpp
// (row_newbcast) reads inside the multiply-add: the product rule costs one
// instruction per product.  A round gives the lane rows kbg column blocks of
// rb row blocks of ppw points (ppw rb kbg <= 16); the residuals are taken in
// tiles of 16, and per tile the workgroup forms the J entries of the round's
// row and column blocks in LDS once, each from A, B and the point's
// sin x, cos x, so that every call reads its r_m.d = J_mi and r_m.g = J_m,k
// there.  The row's own second-order part, sum_m r_m.v D_mi, is formed once
// per row after the value column (float64, m in order, from the row's column
// of A and B, loads coalesced across the rows) and added in the call that
// holds column i.  H.v: each call's terms h[l] v[cs + l] (v of lane jC + l)
// are added to the row's partial of the pair column by column in order; the
// row's partials of its column blocks are summed in block order through
// LDS.  Hessian: H[p][i][cs + l] is stored per call.
//
// The value column r_m.v is computed once per point per workgroup (float64,
// a lane row per residual) and staged in LDS with sin x, cos x and v.  The row-block rounds of a point
// group are split over `rsplit` workgroups: few large points still fill the
// GPU.
//
// Precision policies: F64 runs everything in float64.  F32C forms J from the
// float32 copies of A and B (exact: small integers) and float32 sin, cos,
// sums each call's products over 16 residuals in plain float32 and adds each
// 16-residual partial into a two-sum compensated running sum; r.v, the own
// part, the chunk dot with v (a float32 x float32 product is exact in
// float64) and the row sums stay in float64.
#pragma once

#include <stdint.h>

#include <type_traits>

#include "kernel_fp_call.hpp"

namespace chessfad {

struct FpDppArgs {
    const double* x;    // [npts][n]
    const double* v;    // [npts][n] (H.v only)
    double* out;        // [npts][n] for H.v, [npts][n][n] for the Hessian
    FpParams fp;
    int64_t npts;
    int n;              // any n <= 512 (the library runs it for n > 16)
    int nb;             // blocks of 16 variables, ceil(n / 16)
    int ppw;            // points per workgroup
    int rb;             // row blocks per round
    int kbg;            // column blocks per round
    int rsplit;         // workgroups per point group (each takes a range of row-block rounds)
    double* grad = nullptr;  // H.v only, optional: [npts][n] gradient
    double* fval = nullptr;  // H.v only, optional: [npts] f
    int io32 = 0;            // H.v: x, v and out are float32 (batched instances)
};

constexpr int kFpDppThreads = 256;
constexpr int kFpDppTile = 16;   // residuals per J tile (MT x 16 lanes = the workgroup's 256 threads)

// LDS of one workgroup, in doubles (host and device agree): per point sin x,
// cos x, r.v, v (16 nb each); the row partials of a round (16 x 16), the
// rows' running sums and own parts (ppw x rb x 16 each); the D tile of the
// round's row blocks, [point][row-block slot][residual][lane] (float64);
// then the J tile, [point][block slot][residual][lane] of T.  The symmetric
// form keeps sin x, cos x, v, r.v (whose space then holds the running
// results), the row and the mirror partials of a round (16 x 16 each) and
// the J tile.
__host__ __device__ inline size_t fp_dpp_lds_doubles(int nb, int ppw, int rb, bool sym = false) {
    if (sym) return (size_t)4 * ppw * 16 * nb + 512;
    return (size_t)4 * ppw * 16 * nb + 256 + (size_t)ppw * rb * 16;
}
template <typename T>
__host__ __device__ inline size_t fp_dpp_lds_bytes(int nb, int ppw, int rb, int kbg, bool sym = false) {
    return fp_dpp_lds_doubles(nb, ppw, rb, sym) * sizeof(double) +
           (size_t)ppw * (kbg + rb) * kFpDppTile * 16 * sizeof(T);
}

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

// A and B at R offsets, all loads in flight together: T = float reads the
// float32 copies; T = double reads them too when they are exact (the same
// values in half the bytes), else the float64 arrays.
template <typename T, int R>
CF_DEV void fp_ab_loads(const FpParams& fp, const T* Ab, const T* Bb, const uint32_t (&o)[R], T (&av)[R],
                        T (&bv)[R]) {
    if (std::is_same<T, double>::value && fp.ab32) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bv[r] = (T)ld_at(fp.B32, o[r]);
            av[r] = (T)ld_at(fp.A32, o[r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bv[r] = ld_at(Bb, o[r]);
            av[r] = ld_at(Ab, o[r]);
        }
    }
}

// Per-call accumulation of the C products over the residuals: float64
// directly; float32 in 16-residual blocks (one J tile) added into a two-sum
// running sum.
template <class Prec, int C>
struct DppCallSum;
template <int C>
struct DppCallSum<F64, C> {
    double acc[C];
    CF_DEV void reset() {
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
    CF_DEV void reset() {
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

// sin x, cos x and v of the points p0 .. p0 + ppw - 1 (zeros past n and
// npts), from x and v stored as XT.
template <bool kHess, typename XT>
__device__ __forceinline__ void fp_dpp_stage(const FpDppArgs& a, const XT* x, const XT* v, int64_t p0, double* sins,
                                             double* coss, double* vs) {
    const int n = a.n, n16 = 16 * a.nb;
    for (int idx = threadIdx.x; idx < a.ppw * n16; idx += kFpDppThreads) {
        const int ps = idx / n16, k = idx - ps * n16;
        const int64_t p = p0 + ps;
        const bool live = p < a.npts && k < n;
        double s = 0.0, c = 0.0;
        if (live) sincos((double)x[p * n + k], &s, &c);
        sins[idx] = s;
        coss[idx] = c;
        if (!kHess) vs[idx] = live ? (double)v[p * n + k] : 0.0;
    }
}

// The value column r_m.v = E_m - sum_j A_mj sin x_j + B_mj cos x_j (float64)
// of the points p0 .. p0 + ppw - 1 from their staged sin x and cos x: a lane
// row per (point, residual), lane t summing the terms j = t, t + 16, ... in
// order, then the 16 partial sums in a fixed tree; zeros past n and npts.
__device__ __forceinline__ void fp_dpp_value_column(const FpDppArgs& a, int64_t p0, const double* sins,
                                                    const double* coss, double* rvs) {
    const int n = a.n, n16 = 16 * a.nb;
    for (int task = threadIdx.x >> 4; task < a.ppw * n16; task += kFpDppThreads / 16) {
        const int ps = task / n16, m = task - ps * n16, t = threadIdx.x & 15;
        const int64_t p = p0 + ps;
        const bool on = m < n && p < a.npts;
        const double* sp = sins + ps * n16;
        const double* cp = coss + ps * n16;
        double acc = 0.0;
        if (on && a.fp.ab32) {
            // the exact float32 copies: the same values, half the bytes
            const float* Am = a.fp.A32 + (size_t)m * n;
            const float* Bm = a.fp.B32 + (size_t)m * n;
#pragma unroll 4
            for (int j = t; j < n; j += 16) acc += (double)Am[j] * sp[j] + (double)Bm[j] * cp[j];
        } else if (on) {
            const double* Am = a.fp.A + (size_t)m * n;
            const double* Bm = a.fp.B + (size_t)m * n;
#pragma unroll 4
            for (int j = t; j < n; j += 16) acc += Am[j] * sp[j] + Bm[j] * cp[j];
        }
#pragma unroll
        for (int w = 8; w >= 1; w >>= 1) acc += __shfl_xor(acc, w, 16);
        if (t == 0) rvs[ps * n16 + m] = on ? a.fp.E[m] - acc : 0.0;
    }
}

// One workgroup: point group pg, row-block rounds [ibr0, ibr1).
//
// A lane row (16 lanes) d is (point slot ps, row-block slot ibs, column-
// block slot kbs); in round (ibr, kgr) it holds the calls of rows
// i = 16 ib + t, ib = ibr rb + ibs, whose chunks lie in column block
// kb = kgr kbg + kbs.  Per tile of 16 residuals the workgroup forms the J
// entries the round needs - columns of its kbg column blocks and rb row
// blocks - in LDS once, each from A, B and the point's sin, cos; every lane
// then reads its own r.d = J_mi and its column's J_m,16kb+t, and the calls'
// C products r.d r.g[l] take the chunk columns from the lanes that hold them
// (DPP).  After the last tile: the Hessian chunk of each call is stored, or
// each call's terms h[l] v[cs + l] are added to the row's partial; the
// partials of a row's column blocks are summed in block order through LDS.
//
// kSym: the symmetric forms SC-HESS-VEC and SCHUNK-HESS (Sec. III.B,
// Sec. VI).  Only the calls whose chunk is the row's own chunk or lies right
// of it are evaluated: the pairs kb >= ib (a row-block group's rounds start
// at the column group that holds its first row block).  In the diagonal pair
// lane t counts its calls jc >= t / C and mirrors jc > t / C; right of the
// diagonal every call is counted and mirrored.  A mirrored entry H(i, s)
// stands for H(s, i) too: the Hessian stores it twice; H.v adds H(i, s) v_i
// to the result of column s, summed over the pair's 16 rows by recursive
// halving across the lane row (lane c ends with column 16 kb + c).  After a
// round the pairs' row partials and mirror partials are added, pair by pair
// in lane-row order, to a running result per (point, variable) in LDS; a
// point group is one workgroup (no split), and the result is written after
// its last round.
template <class Prec, int C, bool kHess, bool kGrad, bool kSym = false>
__device__ __forceinline__ void fp_dpp_block(const FpDppArgs& a, int64_t pg, int ibr0, int ibr1, double* lds) {
    static_assert(!(kSym && kGrad), "the symmetric form has no gradient output");
    using T = typename Prec::T;
    constexpr int MT = kFpDppTile;
    const int n = a.n, nb = a.nb, ppw = a.ppw, rb = a.rb, kbg = a.kbg, n16 = 16 * nb;
    const int nslots = kbg + rb;
    double* sins = lds;
    double* coss = sins + ppw * n16;
    double* rvs = coss + ppw * n16;
    double* vs = rvs + ppw * n16;
    double* part = vs + ppw * n16;            // [16 lane rows][16]
    double* rowsum = part + 256;              // [ppw][rb][16]; kSym: the mirror partials [16 lane rows][16]
    T* jt = reinterpret_cast<T*>(kSym ? rowsum + 256 : rowsum + ppw * rb * 16);   // [ppw][nslots][MT][16]
    double* mirp = rowsum;
    // after the prologue: the rows' own parts (kSym H.v: the running results,
    // started at own_i v_i)
    double* sacc = rvs;
    const int64_t p0 = pg * ppw;

    // 1. sin x, cos x and v of the workgroup's points (zeros past n and npts);
    // the input type is uniform: one loop per type
    if (a.io32)
        fp_dpp_stage<kHess>(a, reinterpret_cast<const float*>(a.x), reinterpret_cast<const float*>(a.v), p0, sins,
                            coss, vs);
    else
        fp_dpp_stage<kHess>(a, a.x, a.v, p0, sins, coss, vs);
    __syncthreads();
    // 2. the value column r_m.v (float64)
    fp_dpp_value_column(a, p0, sins, coss, rvs);
    __syncthreads();
    if (kGrad && a.fval && ibr0 == 0 && (int)threadIdx.x < ppw) {
        const int64_t p = p0 + threadIdx.x;
        if (p < a.npts) {
            const double* rp = rvs + threadIdx.x * n16;
            double f = rp[0] * rp[0];
            for (int m = 1; m < n; ++m) f += rp[m] * rp[m];
            a.fval[p] = f;
        }
    }
    {
        // the own parts own_i = sum_m r_m.v D_mi, D_mi = A_mi sin x_i +
        // B_mi cos x_i, of the rows of this workgroup's rounds (float64, m in
        // order; kGrad: also the gradient 2 sum_m r_m.v J_mi, stored here),
        // held in registers until every thread has read r.v; their space then
        // keeps own_i (kSym H.v: starts the running results at own_i v_i)
        constexpr int kMaxTasks = 8;   // ppw 16 nb <= 2048 (the LDS limit)
        const int r0 = 16 * ibr0 * rb, r1 = 16 * ibr1 * rb < n16 ? 16 * ibr1 * rb : n16;
        const int nr = r1 - r0;
        double ownr[kMaxTasks];
#pragma unroll
        for (int k = 0; k < kMaxTasks; ++k) {
            const int task = threadIdx.x + k * kFpDppThreads;
            ownr[k] = 0.0;
            if (task < ppw * nr) {
                const int ps = task / nr, i = r0 + task - ps * nr;
                if (i < n) {
                    const double s = sins[ps * n16 + i], c = coss[ps * n16 + i];
                    const double* rp = rvs + ps * n16;
                    double own = 0.0, gr = 0.0;
                    if (a.fp.ab32) {
                        const float* Ai = a.fp.A32 + i;
                        const float* Bi = a.fp.B32 + i;
#pragma unroll 4
                        for (int m = 0; m < n; ++m) {
                            const double am = (double)Ai[(size_t)m * n], bm = (double)Bi[(size_t)m * n];
                            own += rp[m] * (am * s + bm * c);
                            if (kGrad) gr += rp[m] * (bm * s - am * c);
                        }
                    } else {
                        const double* Ai = a.fp.A + i;
                        const double* Bi = a.fp.B + i;
#pragma unroll 4
                        for (int m = 0; m < n; ++m) {
                            const double am = Ai[(size_t)m * n], bm = Bi[(size_t)m * n];
                            own += rp[m] * (am * s + bm * c);
                            if (kGrad) gr += rp[m] * (bm * s - am * c);
                        }
                    }
                    ownr[k] = kSym && !kHess ? own * vs[ps * n16 + i] : own;
                    if (kGrad && p0 + ps < a.npts) a.grad[(p0 + ps) * n + i] = gr + gr;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxTasks; ++k) {
            const int task = threadIdx.x + k * kFpDppThreads;
            if (task < ppw * nr) {
                const int ps = task / nr;
                sacc[ps * n16 + r0 + task - ps * nr] = ownr[k];
            }
        }
    }

    // 3. the rounds
    const int d = threadIdx.x >> 4, t = threadIdx.x & 15;
    const int per_pt = rb * kbg;
    const bool lr_on = d < ppw * per_pt;
    const int ps = lr_on ? d / per_pt : 0;
    const int ibs = lr_on ? (d - ps * per_pt) / kbg : 0;
    const int kbs = lr_on ? d - ps * per_pt - ibs * kbg : 0;
    const int64_t p = p0 + ps;
    const double* vp = vs + (kHess ? 0 : ps * n16);
    const T* Ab = fp_a_base<T>(a.fp);
    const T* Bb = fp_b_base<T>(a.fp);
    const T* jk = jt + ((size_t)(ps * nslots + kbs) * MT) * 16 + t;          // this lane's column's entries
    const T* ji = jt + ((size_t)(ps * nslots + kbg + ibs) * MT) * 16 + t;    // this lane's row's entries
    const int kgr_n = (nb + kbg - 1) / kbg;
    const int tiles = (n + MT - 1) / MT;
    DppCallSum<Prec, C> sums[16 / C];

    for (int ibr = ibr0; ibr < ibr1; ++ibr) {
        const int ib = ibr * rb + ibs;
        const int i = 16 * ib + t;
        const bool row_live = lr_on && p < a.npts && ib < nb && i < n;
        for (int kgr = kSym ? (ibr * rb) / kbg : 0; kgr < kgr_n; ++kgr) {
            const int kb = kgr * kbg + kbs;
            const bool pair_on = lr_on && ib < nb && kb < nb && (!kSym || kb >= ib);
            // a round whose row blocks all lie in its column group forms no
            // row slots: a row's entries are its column slot's
            const bool alias = ibr * rb >= kgr * kbg && ibr * rb + rb <= kgr * kbg + kbg;
            const int nform = alias ? kbg : nslots;
            const T* jr = alias ? jt + ((size_t)(ps * nslots + ibr * rb + ibs - kgr * kbg) * MT) * 16 + t : ji;
#pragma unroll
            for (int jc = 0; jc < 16 / C; ++jc) sums[jc].reset();
            for (int mt = 0; mt < tiles; ++mt) {
                __syncthreads();   // the previous tile has been read
                // the round's J entries of this tile, J_mk = B_mk sin x_k -
                // A_mk cos x_k: entry [q][u][tt] of q = (point, block slot) is
                // thread 16 u + tt's in step q (MT x 16 = 256 threads)
                {
                    const int u = threadIdx.x >> 4, tt = threadIdx.x & 15;
                    const int m = mt * MT + u;
                    const bool m_on = m < n;
                    const uint32_t mrow = (uint32_t)((m_on ? m : 0) * n);
                    // eight (or four) block slots at a time, their A and B
                    // loads (from clamped, in-range offsets) all in flight
                    // together and shared by the points; sin and cos are zero
                    // past n, and blocks past nb and residuals past n are masked
                    auto form = [&](int b0, auto rc) {
                        constexpr int R = decltype(rc)::value;
                        T bv[R], av[R];
                        int col[R];
                        bool on[R];
                        uint32_t o[R];
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int bs = b0 + r < nform ? b0 + r : nform - 1;
                            const int blk = bs < kbg ? kgr * kbg + bs : ibr * rb + (bs - kbg);
                            on[r] = m_on && blk < nb;
                            col[r] = on[r] ? 16 * blk + tt : 0;
                            o[r] = mrow + (uint32_t)(col[r] < n ? col[r] : n - 1);
                        }
                        fp_ab_loads<T, R>(a.fp, Ab, Bb, o, av, bv);
                        for (int qs = 0; qs < ppw; ++qs) {
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                const int sc = qs * n16 + col[r];
                                const T jv = bv[r] * (T)sins[sc] - av[r] * (T)coss[sc];
                                if (b0 + r < nform) jt[(qs * nslots + b0 + r) * (MT * 16) + threadIdx.x] = on[r] ? jv : T(0);
                            }
                        }
                    };
                    for (int b0 = 0; b0 < nform;) {
                        if (nform - b0 > 4) {
                            form(b0, std::integral_constant<int, 8>{});
                            b0 += 8;
                        } else {
                            form(b0, std::integral_constant<int, 4>{});
                            b0 += 4;
                        }
                    }
                }
                __syncthreads();
                if (pair_on) {
#pragma unroll
                    for (int ug = 0; ug < MT / 4; ++ug) {
                        T g[4], dd[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            g[u] = jk[(4 * ug + u) * 16];
                            dd[u] = jr[(4 * ug + u) * 16];
                        }
                        static_for<16 / C>([&](auto jcc) {
                            constexpr int jc = decltype(jcc)::value;
                            DppRowProducts<T, C, jc * C>::run(sums[jc].block(), g, dd);
                        });
                    }
#pragma unroll
                    for (int jc = 0; jc < 16 / C; ++jc) sums[jc].close_block();
                }
            }
            // the calls of the pair (kSym: calls jc >= tc counted, jc > tc mirrored)
            double prt = 0.0;
            if (pair_on) {
                const int tc = kSym && kb == ib ? t / C : -1;
                const double vk = kHess ? 0.0 : vp[16 * kb + t];
                double w[kSym && !kHess ? 16 : 1];   // kSym H.v: mirror terms h v_i per column 16 kb + c
#pragma unroll
                for (int c = 0; c < (kSym && !kHess ? 16 : 1); ++c) w[c] = 0.0;
                static_for<16 / C>([&](auto jcc) {
                    constexpr int jc = decltype(jcc)::value;
                    constexpr int cl = jc * C;   // the chunk's first lane in the row
                    const int cs = 16 * kb + cl;
                    if (cs >= n) return;
                    double h[C];
#pragma unroll
                    for (int l = 0; l < C; ++l) h[l] = sums[jc].value(l);
                    if constexpr (kHess) {
                        if (jc < tc) return;
                        if (kSym && jc > tc && row_live) {
                            // SCHUNK-HESS: the mirror image H[p][cs + l][i]
#pragma unroll
                            for (int l = 0; l < C; ++l)
                                if (cs + l < n) a.out[((size_t)p * n + cs + l) * n + i] = h[l] + h[l];
                        }
                        // CHUNK-HESS: H[p][i][cs + l] = 2 (products + [cs + l = i] own)
                        if (kb == ib) {
                            const double own = sacc[ps * n16 + i];
#pragma unroll
                            for (int l = 0; l < C; ++l)
                                if (cs + l == i) h[l] += own;
                        }
                        if (row_live) {
                            double* dst = a.out + ((size_t)p * n + i) * n + cs;
#pragma unroll
                            for (int l = 0; l < C; ++l)
                                if (cs + l < n) dst[l] = h[l] + h[l];
                        }
                    } else if constexpr (!kSym && std::is_same<T, double>::value) {
                        // the call's terms h[l] v[cs + l] (v of lane cl + l)
                        // added to the row's partial column by column, in order
                        DppChunkDot<C, cl>::run(prt, vk, h);
                    } else if constexpr (!kSym) {
                        // float calls: the chunk dot first, then one add (fewer
                        // live registers than the float64 form)
                        double dot = 0.0;
                        DppChunkDot<C, cl>::run(dot, vk, h);
                        prt += dot;
                    } else {
                        // a counted call's chunk dot with v (v of lane cl + l)
                        double dot = 0.0;
                        DppChunkDot<C, cl>::run(dot, vk, h);
                        if (jc >= tc) prt += dot;
                        const double vi = vp[i];   // zero past n
#pragma unroll
                        for (int l = 0; l < C; ++l) w[cl + l] = jc > tc ? h[l] * vi : 0.0;
                    }
                });
                if constexpr (kSym && !kHess) {
                    // recursive halving over the lane row: at step s the lanes
                    // with bit s set keep the upper half of their live entries
                    // and receive it from lane t ^ s, so lane t ends with
                    // column t's sum
#pragma unroll
                    for (int s = 8; s >= 1; s >>= 1) {
                        const bool up = (t & s) != 0;
#pragma unroll
                        for (int j = 0; j < s; ++j) {
                            const double send = up ? w[j] : w[j + s];
                            const double keep = up ? w[j + s] : w[j];
                            w[j] = keep + __shfl_xor(send, s, 16);
                        }
                    }
                    mirp[d * 16 + t] = w[0];
                }
            }
            if constexpr (kSym && !kHess) {
                // the round's row and mirror partials into the running
                // results, pair by pair in lane-row order
                part[d * 16 + t] = prt;
                __syncthreads();
                if ((int)threadIdx.x < ppw * 16) {
                    const int ms = threadIdx.x >> 4;
                    double* ap = sacc + ms * n16 + t;
                    for (int e = 0; e < per_pt; ++e) {
                        const int ibe = ibr * rb + e / kbg, kbe = kgr * kbg + e % kbg;
                        if (ibe >= nb || kbe >= nb || kbe < ibe) continue;
                        ap[16 * ibe] += part[(ms * per_pt + e) * 16 + t];
                        ap[16 * kbe] += mirp[(ms * per_pt + e) * 16 + t];
                    }
                }
            } else if constexpr (!kHess) {
                // the row's partials over the round's column blocks, in block order
                part[d * 16 + t] = prt;
                __syncthreads();
                if (lr_on && kbs == 0) {
                    double* rs = rowsum + (ps * rb + ibs) * 16 + t;
                    double acc = kgr == 0 ? 0.0 : *rs;
                    for (int b = 0; b < kbg; ++b) acc += part[(d + b) * 16 + t];
                    *rs = acc;
                }
            }
        }
        if constexpr (!kHess && !kSym) {
            __syncthreads();
            if (row_live && kbs == 0) {
                const double own = sacc[ps * n16 + i];
                const double row = rowsum[(ps * rb + ibs) * 16 + t] + own * vp[i];
                st_io(a.out, p * n + i, row + row, a.io32);
            }
        }
    }
    if constexpr (kSym && !kHess) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < ppw * n16; idx += kFpDppThreads) {
            const int pe = idx / n16, ie = idx - pe * n16;
            if (ie < n && p0 + pe < a.npts) st_io(a.out, (p0 + pe) * n + ie, sacc[idx] + sacc[idx], a.io32);
        }
    }
}

// The row-block rounds [ibr0, ibr1) of workgroup rpart of a point group (a
// point group's rounds split over rsplit workgroups).
__host__ __device__ inline void fp_dpp_rounds(int nb, int rb, int rsplit, int rpart, int& ibr0, int& ibr1) {
    const int ibr_n = (nb + rb - 1) / rb;
    const int per = (ibr_n + rsplit - 1) / rsplit;
    ibr0 = rpart * per;
    ibr1 = ibr0 + per < ibr_n ? ibr0 + per : ibr_n;
}

// kSym: a point group is one workgroup (rsplit = 1).
template <class Prec, int C, bool kHess, bool kGrad, bool kSym>
__global__ __launch_bounds__(kFpDppThreads) void fp_dpp_kernel(FpDppArgs a) {
    extern __shared__ double lds[];
    const int64_t pg = blockIdx.x / a.rsplit;
    int ibr0, ibr1;
    fp_dpp_rounds(a.nb, a.rb, a.rsplit, (int)(blockIdx.x - pg * a.rsplit), ibr0, ibr1);
    fp_dpp_block<Prec, C, kHess, kGrad, kSym>(a, pg, ibr0, ibr1, lds);
}

}  // namespace chessfad
