// Fletcher-Powell, 16 < n <= 512: the symmetric forms SC-HESS-VEC and
// SCHUNK-HESS (Sec. III.B, Sec. VI) on the per-call kernel with DPP lane
// broadcasts.
//
// The calls are the full form's (kernel_fp_dpp.hpp) whose chunk is the row's
// own chunk or lies right of it; for row i = 16 ib + t they sit in the column
// blocks kb >= ib.  An entry of a chunk right of the row's own one also
// stands for its mirror image: H.v adds h v_i to the result of its column,
// the Hessian stores it at [column][i] as well.
//
// Mapping: a point's (row block, column block) pairs kb >= ib, taken row by
// row (nb (nb + 1) / 2 of them), are cut into passes of q pairs; a workgroup
// runs each pass for its ppw points at once, lane row (point ps, pair q')
// holding lane t's row of that pair as in the full form.  Per tile of 16
// residuals the workgroup forms in LDS the J entries of each pair's column
// block (slot q'), plus the row block of the pass's first pair when that
// row's diagonal pair lies in an earlier pass (slot q); every other pair's
// row block is the column block of its own row's diagonal pair, in the same
// pass.  The own part sum_m r_m.v D_mi of each row is formed once in the
// prologue (float64, residuals in order).  H.v: after a pass each pair's row
// partials (the chunk dots with v of the counted calls) and mirror partials
// (the mirrored entries times v_i, summed over the pair's 16 rows by
// recursive halving, lane c ending with column 16 kb + c) are added, pair by
// pair in pass order, to one LDS accumulator per (point, variable) that
// starts at own_i v_i.  A point group is one workgroup: the result is
// written once, after the last pass.
//
// Precision policies as in the full form.
#pragma once

#include <stdint.h>

#include "kernel_fp_dpp.hpp"

namespace chessfad {

__host__ __device__ inline int fp_sym_pairs(int nb) { return nb * (nb + 1) / 2; }

// LDS of one workgroup (host and device agree): per point sin x, cos x, v,
// r.v and the accumulator (16 nb doubles each); the row and mirror partials
// of a pass (16 x 16 doubles each); the J tile [point][slot][residual][lane]
// of T with q + 1 slots; the pair table (ib << 8 | kb, 16 bits each).
template <typename T>
__host__ __device__ inline size_t fp_sym_lds_bytes(int nb, int ppw, int q) {
    return ((size_t)5 * ppw * 16 * nb + 512) * sizeof(double) +
           (size_t)ppw * (q + 1) * kFpDppTile * 16 * sizeof(T) +
           (((size_t)fp_sym_pairs(nb) * sizeof(uint16_t) + 7) & ~(size_t)7);
}

template <class Prec, int C, bool kHess>
__device__ __forceinline__ void fp_sym_block(const FpDppArgs& a, int64_t pg, double* lds) {
    using T = typename Prec::T;
    constexpr int MT = kFpDppTile;
    const int n = a.n, nb = a.nb, ppw = a.ppw, Q = a.q, n16 = 16 * nb;
    const int npairs = fp_sym_pairs(nb);
    double* sins = lds;
    double* coss = sins + ppw * n16;
    double* vs = coss + ppw * n16;
    double* rvs = vs + ppw * n16;
    double* acc = rvs + ppw * n16;   // H.v: running results; Hessian: own parts
    double* part = acc + ppw * n16;  // [16 lane rows][16]
    double* mirp = part + 256;       // [16 lane rows][16]
    T* jt = reinterpret_cast<T*>(mirp + 256);   // [ppw][Q + 1][MT][16]
    uint16_t* pairs = reinterpret_cast<uint16_t*>(jt + (size_t)ppw * (Q + 1) * MT * 16);
    const int64_t p0 = pg * ppw;

    // 1. sin x, cos x and v of the workgroup's points; the pair table
    if (a.io32)
        fp_dpp_stage<kHess>(a, reinterpret_cast<const float*>(a.x), reinterpret_cast<const float*>(a.v), p0, sins,
                            coss, vs);
    else
        fp_dpp_stage<kHess>(a, a.x, a.v, p0, sins, coss, vs);
    for (int f = threadIdx.x; f < npairs; f += kFpDppThreads) {
        int ib = 0, r = f;
        while (r >= nb - ib) {
            r -= nb - ib;
            ++ib;
        }
        pairs[f] = (uint16_t)(ib << 8 | (ib + r));
    }
    __syncthreads();
    // 2. the value column r_m.v (float64)
    fp_dpp_value_column(a, p0, sins, coss, rvs);
    __syncthreads();
    // 3. the own part of every row, own_i = sum_m r_m.v D_mi with
    // D_mi = A_mi sin x_i + B_mi cos x_i (float64, m in order); the
    // accumulator starts at own_i v_i (H.v) or holds own_i (Hessian)
    for (int task = threadIdx.x; task < ppw * n16; task += kFpDppThreads) {
        const int ps = task / n16, i = task - ps * n16;
        double own = 0.0;
        if (i < n) {
            const double s = sins[task], c = coss[task];
            const double* rp = rvs + ps * n16;
            const double* Ai = a.fp.A + i;
            const double* Bi = a.fp.B + i;
#pragma unroll 8
            for (int m = 0; m < n; ++m) own += rp[m] * (Ai[(size_t)m * n] * s + Bi[(size_t)m * n] * c);
        }
        acc[task] = kHess ? own : own * vs[task];
    }

    // 4. the passes
    const int d = threadIdx.x >> 4, t = threadIdx.x & 15;
    const bool lr_on = d < ppw * Q;
    const int ps = lr_on ? d / Q : 0;
    const int qd = lr_on ? d - ps * Q : 0;
    const int64_t p = p0 + ps;
    const double* vp = vs + ps * n16;
    const T* Ab = fp_a_base<T>(a.fp);
    const T* Bb = fp_b_base<T>(a.fp);
    const int tiles = (n + MT - 1) / MT;
    const int npass = (npairs + Q - 1) / Q;
    const T* jk = jt + ((size_t)(ps * (Q + 1) + qd) * MT) * 16 + t;   // this lane's column's entries
    DppCallSum<Prec, C> sums[16 / C];

    for (int pass = 0; pass < npass; ++pass) {
        const int f0 = pass * Q;
        const bool pair_on = lr_on && f0 + qd < npairs;
        const int pr = pairs[pair_on ? f0 + qd : f0];
        const int ib = pr >> 8, kb = pr & 0xff, dq = kb - ib;
        // the row's entries: the slot of its diagonal pair, or slot Q
        const T* ji = jt + ((size_t)(ps * (Q + 1) + (dq <= qd ? qd - dq : Q)) * MT) * 16 + t;
        const int pr0 = pairs[f0];
        const int row0 = (pr0 >> 8) != (pr0 & 0xff) ? pr0 >> 8 : -1;   // slot Q's block, if any pair reads it
#pragma unroll
        for (int jc = 0; jc < 16 / C; ++jc) sums[jc].reset();
        for (int mt = 0; mt < tiles; ++mt) {
            __syncthreads();   // the previous tile has been read
            // the pass's J entries of this tile, J_mk = B_mk sin x_k - A_mk cos x_k:
            // entry [e][u][tt] of e = (point, slot) is thread 16 u + tt's
            {
                const int u = threadIdx.x >> 4, tt = threadIdx.x & 15;
                const int m = mt * MT + u;
                const bool m_on = m < n;
                const uint32_t mrow = (uint32_t)((m_on ? m : 0) * n);
                // eight slots at a time, their A and B loads all in flight
                // together and shared by the points
                for (int b0 = 0; b0 <= Q; b0 += 8) {
                    T bv[8], av[8];
                    int col[8];
                    bool on[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const int sl = b0 + r <= Q ? b0 + r : Q;
                        const int blk = sl < Q ? (f0 + sl < npairs ? pairs[f0 + sl] & 0xff : -1) : row0;
                        on[r] = m_on && blk >= 0;
                        col[r] = on[r] ? 16 * blk + tt : 0;
                        const uint32_t o = mrow + (uint32_t)(col[r] < n ? col[r] : n - 1);
                        bv[r] = ld_at(Bb, o);
                        av[r] = ld_at(Ab, o);
                    }
                    for (int es = 0; es < ppw; ++es) {
#pragma unroll
                        for (int r = 0; r < 8; ++r) {
                            const int sc = es * n16 + col[r];
                            const T jv = bv[r] * (T)sins[sc] - av[r] * (T)coss[sc];
                            if (b0 + r <= Q) jt[(es * (Q + 1) + b0 + r) * (MT * 16) + threadIdx.x] = on[r] ? jv : T(0);
                        }
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
                        dd[u] = ji[(4 * ug + u) * 16];
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
        // the calls of the pair: in the diagonal pair lane t's calls jc >= t / C
        // are counted (its own chunk and those right of it) and jc > t / C
        // mirrored; right of the diagonal every call is both
        if (pair_on) {
            const int i = 16 * ib + t;
            const int tc = dq == 0 ? t / C : -1;
            const bool row_live = p < a.npts && i < n;
            if constexpr (kHess) {
                const double own = acc[ps * n16 + i];
                static_for<16 / C>([&](auto jcc) {
                    constexpr int jc = decltype(jcc)::value;
                    const int cs = 16 * kb + jc * C;
                    if (!row_live || jc < tc) return;
                    double* dst = a.out + ((size_t)p * n + i) * n + cs;
#pragma unroll
                    for (int l = 0; l < C; ++l) {
                        double h = sums[jc].value(l);
                        if (cs + l == i) h += own;
                        if (cs + l < n) dst[l] = h + h;
                    }
                    if (jc == tc) return;
#pragma unroll
                    for (int l = 0; l < C; ++l) {
                        const double h = sums[jc].value(l);
                        if (cs + l < n) a.out[((size_t)p * n + cs + l) * n + i] = h + h;
                    }
                });
            } else {
                const double vk = vp[16 * kb + t];   // zero past n
                const double vi = vp[i];
                double prt = 0.0, w[16];
                static_for<16 / C>([&](auto jcc) {
                    constexpr int jc = decltype(jcc)::value;
                    constexpr int cl = jc * C;   // the chunk's first lane in the row
                    double h[C];
#pragma unroll
                    for (int l = 0; l < C; ++l) h[l] = sums[jc].value(l);
                    double dot = 0.0;
                    DppChunkDot<C, cl>::run(dot, vk, h);
                    if (jc >= tc) prt += dot;
#pragma unroll
                    for (int l = 0; l < C; ++l) w[cl + l] = jc > tc ? h[l] * vi : 0.0;
                });
                // recursive halving over the row's lanes: at step s the lanes
                // with bit s set keep the upper half of their live entries and
                // receive it from lane t ^ s, so lane t ends with column t
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
                part[d * 16 + t] = prt;
                mirp[d * 16 + t] = w[0];
            }
        }
        if constexpr (!kHess) {
            // the pass's partials into the accumulator, pair by pair in order
            __syncthreads();
            if ((int)threadIdx.x < ppw * 16) {
                const int ms = threadIdx.x >> 4;
                double* ap = acc + ms * n16 + t;
                for (int qq = 0; qq < Q && f0 + qq < npairs; ++qq) {
                    const int prq = pairs[f0 + qq];
                    const int dd = (ms * Q + qq) * 16 + t;
                    ap[16 * (prq >> 8)] += part[dd];
                    ap[16 * (prq & 0xff)] += mirp[dd];
                }
            }
        }
    }
    if constexpr (!kHess) {
        __syncthreads();
        for (int task = threadIdx.x; task < ppw * n16; task += kFpDppThreads) {
            const int ps2 = task / n16, i = task - ps2 * n16;
            const int64_t pp = p0 + ps2;
            if (i < n && pp < a.npts) st_io(a.out, pp * n + i, acc[task] + acc[task], a.io32);
        }
    }
}

template <class Prec, int C, bool kHess>
__global__ __launch_bounds__(kFpDppThreads) void fp_sym_kernel(FpDppArgs a) {
    extern __shared__ double lds[];
    fp_sym_block<Prec, C, kHess>(a, blockIdx.x, lds);
}

}  // namespace chessfad
