// C ABI of the chunked Hessian library (declared in include/chessfad.h):
// single-instance entry points, the Fletcher-Powell parameter registry,
// options, status strings, and the host services shared with the batched
// planner (tuned chunk table, operation-count model).
//
// Host side only: every argument check happens before anything is enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "chessfad.h"
#include "dispatch.hpp"
#include "fp_params.hpp"
#include "runtime.hpp"

using namespace chessfad;

namespace {
thread_local std::string g_hip_error;
std::mutex g_tune_mu;
int g_tuned[2][3][2][CHESSFAD_MAX_N + 1];  // autotuned chunk per (form, func, precision, n); 0 = none
int g_tuned_map[2][3][CHESSFAD_MAX_N + 1];  // autotuned mapping of H.v per precision (1 or 2); 0 = none
int g_opt_fp_mfma = 1;                   // CHESSFAD_OPT_FP_MFMA
int g_opt_batch_graph = 1;               // CHESSFAD_OPT_BATCH_GRAPH
int g_opt_mapping = 2;                   // CHESSFAD_OPT_MAPPING
int g_opt_fp_points = 0;                 // CHESSFAD_OPT_FP_POINTS
int g_opt_fp_blocks = 0;                 // CHESSFAD_OPT_FP_BLOCKS
int g_opt_batch_tune = 1;                // CHESSFAD_OPT_BATCH_TUNE
}  // namespace

namespace chessfad {

int hip_fail(hipError_t e) {
    g_hip_error = hipGetErrorString(e);
    return CHESSFAD_E_HIP;
}

int check_func_n(int func_id, int n) {
    if (func_id < CHESSFAD_ROSENBROCK || func_id > CHESSFAD_FLETCHER_POWELL) return CHESSFAD_E_FUNC;
    if (n < 1 || n > CHESSFAD_MAX_N) return CHESSFAD_E_N;
    if (func_id == CHESSFAD_ROSENBROCK && n < 2) return CHESSFAD_E_N;
    return CHESSFAD_OK;
}

int resolve_chunk(int func_id, int n, int precision, int max_chunk, bool sym) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const int t = g_tuned[sym][func_id][precision][n];
        if (t > 0 && t <= max_chunk) return t;
    }
    int c = 1;
    if (sym) {
        // Sec. V: the symmetric form needs (3/2) n (2n + 2c + n/c + 1) M
        // multiplications, smallest near c = sqrt(n / 2); ties go to the
        // larger chunk
        double best = 1e300;
        for (int k = 0; k < kNumChunks; ++k) {
            const int ck = kChunks[k];
            if (ck > n || ck > max_chunk) break;
            const double cost = 2.0 * ck + (double)n / ck;
            if (cost <= best) {
                best = cost;
                c = ck;
            }
        }
        return c;
    }
    // full form: the largest compiled chunk <= min(4, n, max_chunk); for
    // Fletcher-Powell above 16 variables (the rows kernel, whose work per
    // point does not grow with the chunk while its workgroups per point
    // shrink) the largest one <= min(n, max_chunk)
    const int cap = func_id == CHESSFAD_FLETCHER_POWELL && n > kFpMaxN ? 16 : 4;
    for (int k = 0; k < kNumChunks; ++k)
        if (kChunks[k] <= n && kChunks[k] <= cap && kChunks[k] <= max_chunk) c = kChunks[k];
    return c;
}

void record_tuned_chunk(int func_id, int n, int precision, int chunk, bool sym) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[sym][func_id][precision][n] = chunk;
}

int tuned_mapping(int func_id, int n, int precision) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int t = g_tuned_map[precision][func_id][n];
    return t ? t : 2;
}

void record_tuned_mapping(int func_id, int n, int precision, int level) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned_map[precision][func_id][n] = level;
}

bool vector_path(int func_id) { return func_id != CHESSFAD_FLETCHER_POWELL || !g_opt_fp_mfma; }
bool fp_tile_path(int func_id, int n) {
    return func_id == CHESSFAD_FLETCHER_POWELL && n <= kFpMaxN && g_opt_fp_mfma == 3;
}

double model_flops_per_call(int func_id, int n, int C) {
    const double hadd = 2.0 * C + 2, hmul = 10.0 * C + 4, scal = 2.0 * C + 2, unary = 4.0 * C + 2, dot = 2.0 * C;
    if (func_id == CHESSFAD_ROSENBROCK) return (n - 1) * (3 * hmul + 3 * hadd + scal + 1) - hadd + dot;
    if (func_id == CHESSFAD_ACKLEY)
        return n * (hmul + hadd + scal + unary + hadd) - 2 * hadd + 4 * scal + 3 * unary + hadd + 1 + dot;
    return 2.0 * n * unary + n * (2.0 * n * scal + (2.0 * n - 1) * hadd + 1 + hmul) + (n - 1) * hadd + dot;
}

bool chunk_compiled(int c) {
    for (int k = 0; k < kNumChunks; ++k)
        if (kChunks[k] == c) return true;
    return false;
}

int option_value(int option) {
    if (option == CHESSFAD_OPT_FP_MFMA) return g_opt_fp_mfma;
    if (option == CHESSFAD_OPT_BATCH_GRAPH) return g_opt_batch_graph;
    if (option == CHESSFAD_OPT_MAPPING) return g_opt_mapping;
    if (option == CHESSFAD_OPT_FP_POINTS) return g_opt_fp_points;
    if (option == CHESSFAD_OPT_FP_BLOCKS) return g_opt_fp_blocks;
    if (option == CHESSFAD_OPT_BATCH_TUNE) return g_opt_batch_tune;
    return CHESSFAD_E_ARG;
}

}  // namespace chessfad

namespace {

// ------------------------------------------------ Fletcher-Powell parameters
struct FpSet {
    double* A = nullptr;
    double* B = nullptr;
    double* E = nullptr;
    float* A32 = nullptr;
    float* B32 = nullptr;
    int* flag = nullptr;   // device: 1 if a float32 copy is inexact
    int ab32 = 0;          // the float32 copies are exact
    int device = -1;
};

std::mutex g_fp_mu;
FpSet g_fp[CHESSFAD_MAX_N + 1];

void fp_free(FpSet& s) {
    if (s.A) (void)hipFree(s.A);
    if (s.B) (void)hipFree(s.B);
    if (s.E) (void)hipFree(s.E);
    if (s.A32) (void)hipFree(s.A32);
    if (s.B32) (void)hipFree(s.B32);
    if (s.flag) (void)hipFree(s.flag);
    s = FpSet{};
}

// The caller holds g_fp_mu until it has enqueued the work that reads the set,
// so a concurrent chessfad_fp_release (whose hipFree waits for the device)
// frees it only before the lookup or after that work.
int fp_lookup_locked(int n, FpParams& out) {
    const FpSet& s = g_fp[n];
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return CHESSFAD_E_HIP;
    if (!s.A || s.device != dev) return CHESSFAD_E_PARAMS;
    out = FpParams{s.A, s.B, s.E, s.A32, s.B32, s.ab32};
    return CHESSFAD_OK;
}

SymLaunch sym_table(int func_id, int C, bool hess, bool mixed) {
    switch (func_id) {
        case CHESSFAD_ROSENBROCK: return sym_rosenbrock(C, hess, mixed);
        case CHESSFAD_ACKLEY: return sym_ackley(C, hess, mixed);
        default: return sym_fletcher_powell(C, hess, mixed);
    }
}

template <class P>
size_t sym_lds_p(int func_id, int n, int C, int ppb, int ps, bool hess) {
    switch (func_id) {
        case CHESSFAD_ROSENBROCK: return sym_lds_bytes<P, Rosenbrock>(n, C, ppb, ps, hess);
        case CHESSFAD_ACKLEY: return sym_lds_bytes<P, Ackley>(n, C, ppb, ps, hess);
        default: return sym_lds_bytes<P, FletcherPowell>(n, C, ppb, ps, hess);
    }
}

struct SymGeometry {
    int nc, ppb, pstride;
    size_t lds;
    int64_t grid;
};

// Points per workgroup for the symmetric kernel: the count (up to 256) that
// leaves the fewest idle lanes in the last pass over the calls (the smallest
// such count when several are within half a percent), with the LDS image at
// most 32 KiB, or 64 KiB for a single point.  False when one point does not fit.
bool sym_geometry(int func_id, bool mixed, int n, int64_t npts, int C, bool hess, SymGeometry& g) {
    g.nc = (n + C - 1) / C;
    const int64_t per_point = (int64_t)C * g.nc * (g.nc + 1) / 2;
    const int max_ppb = (int)(npts < 256 ? npts : 256);
    int best = 0;
    double best_use = -1.0;
    for (int ppb = 1; ppb <= max_ppb; ++ppb) {
        const int ps = ppb | 1;
        const size_t lds = mixed ? sym_lds_p<F32C>(func_id, n, C, ppb, ps, hess)
                                 : sym_lds_p<F64>(func_id, n, C, ppb, ps, hess);
        if (lds > (ppb == 1 ? kSymMaxLds : kSymMaxLds / 2)) break;
        const int64_t total = ppb * per_point;
        const int64_t passes = (total + kSymThreads - 1) / kSymThreads;
        const double use = (double)total / (double)(passes * kSymThreads);
        if (use > best_use + 0.005) {
            best_use = use;
            best = ppb;
            g.lds = lds;
        }
    }
    if (!best) return false;
    g.ppb = best;
    g.pstride = best | 1;
    g.grid = (npts + best - 1) / best;
    return true;
}

PlainLaunch plain_table(int func_id, int C, bool hess, bool mixed) {
    switch (func_id) {
        case CHESSFAD_ROSENBROCK: return mixed ? mixed_rosenbrock(C, hess) : plain_rosenbrock(C, hess);
        case CHESSFAD_ACKLEY: return mixed ? mixed_ackley(C, hess) : plain_ackley(C, hess);
        default: return mixed ? mixed_fletcher_powell(C, hess) : plain_fletcher_powell(C, hess);
    }
}

PlainLaunch grad_table(int func_id, int C) {
    switch (func_id) {
        case CHESSFAD_ROSENBROCK: return grad_rosenbrock(C);
        case CHESSFAD_ACKLEY: return grad_ackley(C);
        default: return grad_fletcher_powell(C);
    }
}

CoarseLaunch coarse_table(int func_id, int C, int level, bool mixed) {
    switch (func_id) {
        case CHESSFAD_ROSENBROCK: return mixed ? coarse_mixed_rosenbrock(C, level) : coarse_rosenbrock(C, level);
        case CHESSFAD_ACKLEY: return mixed ? coarse_mixed_ackley(C, level) : coarse_ackley(C, level);
        default: return mixed ? coarse_mixed_fletcher_powell(C, level) : coarse_fletcher_powell(C, level);
    }
}

struct Geometry {
    int nc, rows, block, pstride;
    int64_t grid;
};

template <class F>
size_t coarse_lds(int n, int ps, bool mixed) {
    return mixed ? plain_lds_bytes<F32C, F>(n, ps, 0, false) : plain_lds_bytes<F64, F>(n, ps, 0, false);
}

size_t coarse_lds_for(int func_id, int n, int ps, bool mixed) {
    switch (func_id) {
        case CHESSFAD_ROSENBROCK: return coarse_lds<Rosenbrock>(n, ps, mixed);
        case CHESSFAD_ACKLEY: return coarse_lds<Ackley>(n, ps, mixed);
        default: return coarse_lds<FletcherPowell>(n, ps, mixed);
    }
}

// L1: 256 lanes, one per row task.  L0: one lane per point, up to 64 points
// per workgroup (fewer when their staging would pass 48 KiB of LDS).
Geometry coarse_geometry(int func_id, int n, int64_t npts, int C, int level, bool mixed, size_t& lds) {
    Geometry g;
    g.nc = (n + C - 1) / C;
    if (level == 1) {
        g.rows = 256;
        g.block = 256;
        g.pstride = (g.rows - 1) / n + 2;
    } else {
        int pts = 64;
        while (pts > 1 && coarse_lds_for(func_id, n, pts | 1, mixed) > 48 * 1024) pts /= 2;
        g.rows = pts * n;
        g.block = pts < 64 ? 64 : pts;
        g.pstride = pts | 1;
    }
    lds = coarse_lds_for(func_id, n, g.pstride, mixed);
    const int64_t nrows = npts * (int64_t)n;
    g.grid = (nrows + g.rows - 1) / g.rows;
    return g;
}

// Row tasks of nc lanes, about 256 lanes per workgroup (512 when one row
// needs more).  With n <= 512 the LDS image stays below 45 KiB.
Geometry plain_geometry(int n, int64_t npts, int C) {
    Geometry g;
    g.nc = (n + C - 1) / C;
    g.rows = g.nc >= 256 ? 1 : 256 / g.nc;
    g.block = g.rows * g.nc;
    g.pstride = (g.rows - 1) / n + 2;
    const int64_t nrows = npts * (int64_t)n;
    g.grid = (nrows + g.rows - 1) / g.rows;
    return g;
}

}  // namespace

namespace {

// Cost per point of a launch shape of the per-call FP kernel for n > 16: per
// round, 256 products per lane and tile plus about 16 instructions for each
// J entry a lane forms (pp (kbg + rb) per tile; no row slots in a round whose
// row blocks lie in its column group); the symmetric form's rounds start at
// the column group that holds the round's first row block.
double fp_round_cost(int nb, int pp, int rb, int kbg, bool sym) {
    const int kgr_n = (nb + kbg - 1) / kbg;
    double c = 0.0;
    for (int ibr = 0; ibr * rb < nb; ++ibr)
        for (int kgr = sym ? (ibr * rb) / kbg : 0; kgr < kgr_n; ++kgr) {
            const bool alias = ibr * rb >= kgr * kbg && ibr * rb + rb <= kgr * kbg + kbg;
            c += 256.0 + 16.0 * pp * (kbg + (alias ? 0 : rb));
        }
    return c / pp;
}

}  // namespace

FpDppGeometry chessfad::fp_dpp_geometry(int n, int64_t npts, int points, int blocks, bool mixed) {
    FpDppGeometry g;
    g.nb = (n + 15) / 16;
    auto bytes = [&](int pp, int rb, int kbg) {
        return mixed ? fp_dpp_lds_bytes<float>(g.nb, pp, rb, kbg) : fp_dpp_lds_bytes<double>(g.nb, pp, rb, kbg);
    };
    // column blocks per round (the option's, or every count up to 16), points
    // per workgroup (the option's, or any that leaves a column block per
    // lane row), and then as many row blocks as fill the 16 lane rows, at
    // the lowest fp_round_cost
    auto fit = [&](int pp, int kbg) { return std::max(1, std::min(g.nb, 16 / (pp * kbg))); };
    double best = -1.0;
    for (int kbg = 1; kbg <= std::min(g.nb, 16); ++kbg) {
        if (blocks && kbg != std::min(blocks, g.nb)) continue;
        const int pp_hi = std::max(1, 16 / kbg);
        const int pp_lo = points ? std::max(1, std::min(points, pp_hi)) : 1;
        for (int pp0 = pp_lo; pp0 <= (points ? pp_lo : pp_hi); ++pp0) {
            // fewer points where their LDS rows do not fit
            int pp = pp0, rb = fit(pp, kbg);
            while (pp > 1 && bytes(pp, rb, kbg) > 64 * 1024) {
                pp /= 2;
                rb = fit(pp, kbg);
            }
            const double cost = fp_round_cost(g.nb, pp, rb, kbg, false);
            if (best < 0.0 || cost < best) {
                best = cost;
                g.ppw = pp;
                g.rb = rb;
                g.kbg = kbg;
            }
        }
    }
    while (g.rb > 1 && bytes(g.ppw, g.rb, g.kbg) > 64 * 1024) --g.rb;
    const int ibr_n = (g.nb + g.rb - 1) / g.rb;   // row-block rounds per point group
    const int64_t groups = (npts + g.ppw - 1) / g.ppw;
    // split a point group's rounds over workgroups until about 2048
    // workgroups fill the GPU
    const int64_t want = (2048 + groups - 1) / groups;
    g.rsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ibr_n, want));
    g.grid = groups * g.rsplit;
    g.lds = bytes(g.ppw, g.rb, g.kbg);
    return g;
}

FpDppGeometry chessfad::fp_sym_geometry(int n, int64_t npts, int blocks, bool mixed) {
    FpDppGeometry g;
    g.nb = (n + 15) / 16;
    auto bytes = [&](int pp, int rb, int kbg) {
        return mixed ? fp_dpp_lds_bytes<float>(g.nb, pp, rb, kbg, true)
                     : fp_dpp_lds_bytes<double>(g.nb, pp, rb, kbg, true);
    };
    // fp_round_cost over the symmetric form's rounds; a point group is one
    // workgroup, so more points per workgroup only while about 1024
    // workgroups remain
    // (equal costs: the fewer LDS bytes per point, for occupancy)
    double best = -1.0, best_lds = 0.0;
    for (int kbg = 1; kbg <= std::min(g.nb, 16); ++kbg)
        for (int pp = 1; pp * kbg <= 16; ++pp) {
            if (blocks && kbg != std::min(blocks, g.nb)) break;
            if (pp > 1 && (npts + pp - 1) / pp < 1024) break;
            const int rb = std::max(1, std::min(g.nb, 16 / (pp * kbg)));
            const size_t lds = bytes(pp, rb, kbg);
            if (lds > 64 * 1024) continue;
            const double cost = fp_round_cost(g.nb, pp, rb, kbg, true);
            const double lds_pt = (double)lds / pp;
            if (best < 0.0 || cost < best * (1.0 - 1e-9) || (cost <= best * (1.0 + 1e-9) && lds_pt < best_lds)) {
                best = cost;
                best_lds = lds_pt;
                g.ppw = pp;
                g.rb = rb;
                g.kbg = kbg;
            }
        }
    if (best < 0.0) {   // not reached for n <= 512 (one point, one block pair fits)
        g.ppw = g.rb = g.kbg = 1;
    }
    g.rsplit = 1;
    g.grid = (npts + g.ppw - 1) / g.ppw;
    g.lds = bytes(g.ppw, g.rb, g.kbg);
    return g;
}

int chessfad::run_single(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, int chunk,
                         void* stream, bool hess, bool mixed, bool sym, double* grad, double* fval, int mapping) {
    if (func_id >= CHESSFAD_USER_BASE) {
        // a registered user function: float64 H.v or Hessian, full form
        if (!user_registered(func_id) || mixed || sym || grad || fval) return CHESSFAD_E_FUNC;
        if (n < 1 || n > CHESSFAD_MAX_N) return CHESSFAD_E_N;
        if (chunk == 0) chunk = n >= 4 ? 4 : n >= 2 ? 2 : 1;
        if (chunk < 0 || !chunk_compiled(chunk) || chunk > n) return CHESSFAD_E_CHUNK;
        if (npts < 0) return CHESSFAD_E_ARG;
        if (npts == 0) return CHESSFAD_OK;
        if (!x || !out || (!hess && !v)) return CHESSFAD_E_NULL;
        const size_t in_bytes = sizeof(double) * (size_t)npts * n;
        const size_t out_bytes = hess ? in_bytes * n : in_bytes;
        if (overlaps(out, out_bytes, x, in_bytes) || (!hess && overlaps(out, out_bytes, v, in_bytes)))
            return CHESSFAD_E_OVERLAP;
        return run_user(func_id, n, npts, x, v, out, chunk, static_cast<hipStream_t>(stream), hess);
    }
    int rc = check_func_n(func_id, n);
    if (rc) return rc;
    const bool auto_chunk = chunk == 0;
    if (auto_chunk && hess && !sym) {
        // full Hessians are store-bound: the widest call stores whole 16-byte
        // pairs of its row (the H.v tuning does not apply)
        chunk = 1;
        for (int k = 0; k < kNumChunks; ++k)
            if (kChunks[k] <= n) chunk = kChunks[k];
    } else if (auto_chunk) {
        chunk = resolve_chunk(func_id, n, mixed ? 1 : 0, 16, sym);
    }
    if (chunk < 0 || !chunk_compiled(chunk) || chunk > n) return CHESSFAD_E_CHUNK;
    if (npts < 0) return CHESSFAD_E_ARG;
    if (npts == 0) return CHESSFAD_OK;
    if (!x || !out || (!hess && !v)) return CHESSFAD_E_NULL;
    const size_t in_bytes = sizeof(double) * (size_t)npts * n;
    const size_t out_bytes = hess ? in_bytes * n : in_bytes;
    if (overlaps(out, out_bytes, x, in_bytes) || (!hess && overlaps(out, out_bytes, v, in_bytes)))
        return CHESSFAD_E_OVERLAP;
    const size_t f_bytes = sizeof(double) * (size_t)npts;
    if (grad && (overlaps(grad, in_bytes, x, in_bytes) || overlaps(grad, in_bytes, v, in_bytes) ||
                 overlaps(grad, in_bytes, out, out_bytes)))
        return CHESSFAD_E_OVERLAP;
    if (fval && (overlaps(fval, f_bytes, x, in_bytes) || overlaps(fval, f_bytes, v, in_bytes) ||
                 overlaps(fval, f_bytes, out, out_bytes) || (grad && overlaps(fval, f_bytes, grad, in_bytes))))
        return CHESSFAD_E_OVERLAP;
    FpParams fp{nullptr, nullptr, nullptr};
    std::unique_lock<std::mutex> fp_lock;
    if (func_id == CHESSFAD_FLETCHER_POWELL) {
        fp_lock = std::unique_lock<std::mutex>(g_fp_mu);
        rc = fp_lookup_locked(n, fp);
        if (rc) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (func_id == CHESSFAD_FLETCHER_POWELL && n <= kFpMaxN && g_opt_fp_mfma) {
        const int nk = fp_mfma_steps(n);
        FpMfmaLaunch launch = nullptr;
        if (g_opt_fp_mfma == 1 && !sym) {
            // the per-call kernel (DPP lane broadcasts)
            launch = mixed ? fp_call_entry_mixed(chunk, nk, hess, n)
                           : (grad || fval) ? fp_call_entry_grad(chunk, nk, n) : fp_call_entry(chunk, nk, hess, n);
        } else if (g_opt_fp_mfma == 3) {
            // the closed-form point tile: every call of a point is a block of
            // its J^T J tile (the chunk size and the symmetric form give the
            // same entries)
            launch = mixed ? fp_tile_entry_mixed(nk, hess) : fp_tile_entry(nk, hess);
        } else {
            // the per-call kernel with MFMA contractions (also the symmetric form)
            launch = mixed ? fp_mfma_entry_mixed(chunk, nk, hess, sym) : fp_mfma_entry(chunk, nk, hess, sym);
        }
        if (!launch) return CHESSFAD_E_CHUNK;
        const int nc = (n + chunk - 1) / chunk;
        const int64_t per_block = (int64_t)kFpWaves * kFpPointsPerWave;
        const int64_t grid = (npts + per_block - 1) / per_block;
        if (grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
        FpMfmaArgs a{x, v, out, fp, npts, n, nc, grad, fval};
        hipError_t e = launch(a, dim3((unsigned)grid), dim3(64 * kFpWaves), s);
        return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
    }
    if (sym && func_id == CHESSFAD_FLETCHER_POWELL && n > kFpMaxN && g_opt_fp_mfma == 1) {
        // the symmetric form of the per-call kernel (DPP lane broadcasts)
        FpDppLaunch launch = mixed ? fp_dpp_sym_entry_mixed(chunk, hess) : fp_dpp_sym_entry(chunk, hess);
        if (!launch) return CHESSFAD_E_CHUNK;
        const FpDppGeometry g = fp_sym_geometry(n, npts, g_opt_fp_blocks, mixed);
        if (g.grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
        FpDppArgs a{x, v, out, fp, npts, n, g.nb, g.ppw, g.rb, g.kbg, 1};
        hipError_t e = launch(a, dim3((unsigned)g.grid), dim3(kFpDppThreads), g.lds, s);
        return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
    }
    if (sym) {
        // symmetric vector kernel (all three functions; Fletcher-Powell with
        // n > 16 runs its contraction on the vector unit here)
        SymGeometry g;
        bool fits = sym_geometry(func_id, mixed, n, npts, chunk, hess, g);
        for (int k = 0; k < kNumChunks && !fits && auto_chunk; ++k)
            if (kChunks[k] > chunk && kChunks[k] <= n && sym_geometry(func_id, mixed, n, npts, kChunks[k], hess, g)) {
                chunk = kChunks[k];
                fits = true;
            }
        if (!fits) return CHESSFAD_E_CHUNK;
        if (g.grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
        SymLaunch launch = sym_table(func_id, chunk, hess, mixed);
        if (!launch) return CHESSFAD_E_CHUNK;
        SymArgs a{x, v, out, fp, npts, n, g.nc, g.ppb, g.pstride};
        hipError_t e = launch(a, dim3((unsigned)g.grid), dim3(kSymThreads), g.lds, s);
        return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
    }
    if (func_id == CHESSFAD_FLETCHER_POWELL && n > kFpMaxN && g_opt_fp_mfma == 1) {
        // the per-call kernel (DPP lane broadcasts)
        FpDppLaunch launch = mixed ? fp_dpp_entry_mixed(chunk, hess)
                                   : (grad || fval) ? fp_dpp_entry_grad(chunk) : fp_dpp_entry(chunk, hess);
        if (!launch) return CHESSFAD_E_CHUNK;
        const FpDppGeometry g = fp_dpp_geometry(n, npts, g_opt_fp_points, g_opt_fp_blocks, mixed);
        if (g.grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
        FpDppArgs a{x, v, out, fp, npts, n, g.nb, g.ppw, g.rb, g.kbg, g.rsplit, grad, fval};
        hipError_t e = launch(a, dim3((unsigned)g.grid), dim3(kFpDppThreads), g.lds, s);
        return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
    }
    if (func_id == CHESSFAD_FLETCHER_POWELL && n > kFpMaxN && g_opt_fp_mfma) {
        FpRowsLaunch launch = fp_rows_entry(chunk, hess, mixed);
        if (!launch) return CHESSFAD_E_CHUNK;
        const int nc = (n + chunk - 1) / chunk;
        const int rows = fp_rows_per_block(n, chunk);
        const int row_blocks = (n + rows - 1) / rows;
        const int64_t grid = npts * row_blocks;
        if (grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
        FpRowsArgs a{x, v, out, fp, npts, n, nc, rows, row_blocks, grad, fval};
        hipError_t e = launch(a, dim3((unsigned)grid), dim3(64 * kFpRowsWaves), s);
        return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
    }
    // the mapping of H.v: forced, asked for by the option, or the tuned one
    // for chunk = 0; with one chunk per row L2 is L1, whose kernel needs
    // fewer registers
    int want = mapping >= 0 ? mapping : g_opt_mapping;
    if (mapping < 0 && want == 2 && auto_chunk) want = tuned_mapping(func_id, n, mixed ? 1 : 0);
    const bool one_chunk = (n + chunk - 1) / chunk == 1;
    if (!hess && !grad && !fval && (want != 2 || one_chunk)) {
        const int level = want == 2 ? 1 : want;
        if (level == 1 && n == 16 && (func_id == CHESSFAD_ROSENBROCK || func_id == CHESSFAD_ACKLEY)) {
            // a point's 16 rows on one 16-lane row, its values in registers
            Row16Launch launch = func_id == CHESSFAD_ROSENBROCK
                                     ? (mixed ? row16_mixed_rosenbrock(chunk) : row16_rosenbrock(chunk))
                                     : (mixed ? row16_mixed_ackley(chunk) : row16_ackley(chunk));
            if (!launch) return CHESSFAD_E_CHUNK;
            const int64_t grid = (npts * 16 + kRow16Threads - 1) / kRow16Threads;
            if (grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
            hipError_t e = launch(Row16Args{x, v, out, npts}, dim3((unsigned)grid), s);
            return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
        }
        if (level == 1 && func_id == CHESSFAD_ROSENBROCK) {
            // Rosenbrock at other n: each lane loads its row's neighbours
            RowsLaunch launch = mixed ? rosenbrock_rows_mixed(chunk) : rosenbrock_rows(chunk);
            if (!launch) return CHESSFAD_E_CHUNK;
            const int64_t grid = (npts * n + kRow16Threads - 1) / kRow16Threads;
            if (grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
            hipError_t e = launch(Row16Args{x, v, out, npts}, n, dim3((unsigned)grid), s);
            return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
        }
        size_t lds = 0;
        const Geometry g = coarse_geometry(func_id, n, npts, chunk, level, mixed, lds);
        if (g.grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
        CoarseLaunch launch = coarse_table(func_id, chunk, level, mixed);
        if (!launch) return CHESSFAD_E_CHUNK;
        PlainArgs a{x, v, out, fp, npts, n, g.nc, g.rows, g.pstride};
        hipError_t e = launch(a, dim3((unsigned)g.grid), dim3(g.block), lds, s);
        return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
    }
    const Geometry g = plain_geometry(n, npts, chunk);
    if (g.grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
    PlainLaunch launch = grad ? grad_table(func_id, chunk) : plain_table(func_id, chunk, hess, mixed);
    if (!launch) return CHESSFAD_E_CHUNK;
    PlainArgs a{x, v, out, fp, npts, n, g.nc, g.rows, g.pstride, grad, fval};
    hipError_t e = launch(a, dim3((unsigned)g.grid), dim3(g.block), s);
    return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
}

extern "C" {

int chessfad_hvp(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, int chunk,
                 void* stream) {
    return run_single(func_id, n, npts, x, v, out, chunk, stream, false, false);
}

int chessfad_hessian(int func_id, int n, int64_t npts, const double* x, double* H, int chunk, void* stream) {
    return run_single(func_id, n, npts, x, nullptr, H, chunk, stream, true, false);
}

int chessfad_hvp_mixed(int func_id, int n, int64_t npts, const double* x, const double* v, double* out,
                       int chunk, void* stream) {
    return run_single(func_id, n, npts, x, v, out, chunk, stream, false, true);
}

int chessfad_hessian_mixed(int func_id, int n, int64_t npts, const double* x, double* H, int chunk,
                           void* stream) {
    return run_single(func_id, n, npts, x, nullptr, H, chunk, stream, true, true);
}

int chessfad_hvp_grad(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, double* grad,
                      double* fval, int chunk, void* stream) {
    if (npts > 0 && !grad) return CHESSFAD_E_NULL;
    return run_single(func_id, n, npts, x, v, out, chunk, stream, false, false, false, grad, fval);
}

int chessfad_hvp_sym(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, int chunk,
                     int precision, void* stream) {
    if (precision != 0 && precision != 1) return CHESSFAD_E_ARG;
    return run_single(func_id, n, npts, x, v, out, chunk, stream, false, precision == 1, true);
}

int chessfad_hessian_sym(int func_id, int n, int64_t npts, const double* x, double* H, int chunk, int precision,
                         void* stream) {
    if (precision != 0 && precision != 1) return CHESSFAD_E_ARG;
    return run_single(func_id, n, npts, x, nullptr, H, chunk, stream, true, precision == 1, true);
}

int chessfad_fp_set_params(int n, const double* A, const double* B, const double* alpha, void* stream) {
    if (n < 1 || n > CHESSFAD_MAX_N) return CHESSFAD_E_N;
    if (!A || !B || !alpha) return CHESSFAD_E_NULL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_fp_mu);
    FpSet& set = g_fp[n];
    fp_free(set);
    const size_t mat = sizeof(double) * (size_t)n * n;
    hipError_t e = hipGetDevice(&set.device);
    if (e == hipSuccess) e = hipMalloc(&set.A, mat);
    if (e == hipSuccess) e = hipMalloc(&set.B, mat);
    if (e == hipSuccess) e = hipMalloc(&set.E, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&set.A32, sizeof(float) * (size_t)n * n);
    if (e == hipSuccess) e = hipMalloc(&set.B32, sizeof(float) * (size_t)n * n);
    if (e == hipSuccess) e = hipMalloc(&set.flag, sizeof(int));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fp_clear_flag_kernel, dim3(1), dim3(1), 0, s, set.flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(set.A, A, mat, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(set.B, B, mat, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fp_offsets_kernel, dim3((n + 63) / 64), dim3(64), 0, s, n, set.A, set.B, alpha, set.E);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        const int count = n * n;
        hipLaunchKernelGGL(fp_to_f32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, count, set.A, set.B,
                           set.A32, set.B32, set.flag);
        e = hipGetLastError();
    }
    // the set is complete on the device before any stream can read it
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int inexact = 1;
    if (e == hipSuccess) e = hipMemcpy(&inexact, set.flag, sizeof(int), hipMemcpyDeviceToHost);
    set.ab32 = inexact == 0;
    if (e != hipSuccess) {
        fp_free(set);
        return hip_fail(e);
    }
    return CHESSFAD_OK;
}

int chessfad_fp_release(int n) {
    if (n < 1 || n > CHESSFAD_MAX_N) return CHESSFAD_E_N;
    std::lock_guard<std::mutex> lk(g_fp_mu);
    fp_free(g_fp[n]);
    return CHESSFAD_OK;
}

const char* chessfad_strerror(int code) {
    switch (code) {
        case CHESSFAD_OK: return "ok";
        case CHESSFAD_E_FUNC: return "unknown func_id";
        case CHESSFAD_E_N: return "n out of range for this function";
        case CHESSFAD_E_CHUNK: return "chunk size not compiled or larger than n";
        case CHESSFAD_E_NULL: return "NULL array pointer";
        case CHESSFAD_E_PARAMS: return "Fletcher-Powell parameters not set for this n on this device";
        case CHESSFAD_E_OVERLAP: return "output overlaps an input";
        case CHESSFAD_E_HIP: return g_hip_error.empty() ? "HIP error" : g_hip_error.c_str();
        case CHESSFAD_E_ARG: return "invalid argument";
        case CHESSFAD_E_COMPILE: {
            const char* log = user_compile_log();
            return log && *log ? log : "user function failed to compile";
        }
        default: return "unknown status";
    }
}

int chessfad_set_option(int option, int value) {
    int* slot = option == CHESSFAD_OPT_FP_MFMA ? &g_opt_fp_mfma
              : option == CHESSFAD_OPT_BATCH_GRAPH ? &g_opt_batch_graph
              : option == CHESSFAD_OPT_MAPPING ? &g_opt_mapping
              : option == CHESSFAD_OPT_FP_POINTS ? &g_opt_fp_points
              : option == CHESSFAD_OPT_FP_BLOCKS ? &g_opt_fp_blocks
              : option == CHESSFAD_OPT_BATCH_TUNE ? &g_opt_batch_tune : nullptr;
    if (!slot) return CHESSFAD_E_ARG;
    if (option == CHESSFAD_OPT_FP_POINTS) {
        if (value != 0 && value != 1 && value != 4 && value != 16) return CHESSFAD_E_ARG;
    } else if (option == CHESSFAD_OPT_FP_BLOCKS) {
        if (value < 0 || value > 16) return CHESSFAD_E_ARG;
    } else {
        const int maxv = option == CHESSFAD_OPT_FP_MFMA ? 3 : option == CHESSFAD_OPT_MAPPING ? 2 : 1;
        if (value < 0 || value > maxv) return CHESSFAD_E_ARG;
    }
    const int prev = *slot;
    *slot = value;
    return prev;
}

int chessfad_default_chunk(int func_id, int n) {
    int rc = check_func_n(func_id, n);
    return rc ? rc : resolve_chunk(func_id, n, 0, 16);
}

int chessfad_fp_launch_shape(int n, int64_t npts, int precision, int sym, chessfad_fp_shape* out) {
    if (n <= kFpMaxN || n > CHESSFAD_MAX_N) return CHESSFAD_E_N;
    if (npts < 1 || (precision != 0 && precision != 1)) return CHESSFAD_E_ARG;
    if (!out) return CHESSFAD_E_NULL;
    const FpDppGeometry g = sym ? fp_sym_geometry(n, npts, g_opt_fp_blocks, precision == 1)
                                : fp_dpp_geometry(n, npts, g_opt_fp_points, g_opt_fp_blocks, precision == 1);
    out->points = g.ppw;
    out->row_blocks = g.rb;
    out->column_blocks = g.kbg;
    out->split = g.rsplit;
    out->grid = g.grid;
    out->lds_bytes = g.lds;
    return CHESSFAD_OK;
}

int chessfad_default_mapping(int func_id, int n, int precision) {
    int rc = check_func_n(func_id, n);
    if (rc) return rc;
    if (precision != 0 && precision != 1) return CHESSFAD_E_ARG;
    if (g_opt_mapping != 2) return g_opt_mapping;
    const int c = resolve_chunk(func_id, n, precision, 16);
    return (n + c - 1) / c == 1 ? 1 : tuned_mapping(func_id, n, precision);
}

}  // extern "C"
