// Host-side services shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chessfad {

// Records the HIP error text for chessfad_strerror and returns CHESSFAD_E_HIP.
int hip_fail(hipError_t e);

// Checks (func_id, n) against the compiled limits.
int check_func_n(int func_id, int n);

// Chunk used when the caller passes 0: the autotuned choice for
// (form, func_id, n, precision) if there is one, else the built-in default
// (full form: the largest compiled chunk <= 4; symmetric form: the compiled
// chunk that minimises the multiplication count of Sec. V).
int resolve_chunk(int func_id, int n, int precision, int max_chunk, bool sym = false);
void record_tuned_chunk(int func_id, int n, int precision, int chunk, bool sym = false);

// Single-instance launch shared by chessfad_hvp / _hessian / _mixed / _sym.
// With chunk == 0 and sym, a chunk whose symmetric workgroup would not fit
// in LDS is replaced by the next larger one that fits.
// grad / fval (H.v, float64, full form only) receive the gradient and f.
// mapping: -1 decides from CHESSFAD_OPT_MAPPING and the tuned table; 1 or 2
// forces L1 or L2 for float64 H.v on the vector path.
int run_single(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, int chunk,
               void* stream, bool hess, bool mixed, bool sym = false, double* grad = nullptr,
               double* fval = nullptr, int mapping = -1);

// User functions (user.hip): registered?, the last compile log of this
// thread, and the H.v / Hessian launch (arguments already checked).
bool user_registered(int func_id);
const char* user_compile_log();
int run_user(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, int chunk,
             hipStream_t stream, bool hess);

// Float64 H.v of func_id runs its f on the vector ALUs (not on MFMA).
bool vector_path(int func_id);
// Fletcher-Powell at n <= 16 on the point tile: every chunk gives the same launch
bool fp_tile_path(int func_id, int n);

// GPU mapping (1 = L1, 2 = L2) chosen by the autotuner for float64 H.v of
// (func_id, n) with chunk = 0; 2 when none was recorded.
int tuned_mapping(int func_id, int n, int precision);
void record_tuned_mapping(int func_id, int n, int precision, int level);

// Paper-model flops of one f call (Sec. V operation counts, chunk dot included).
double model_flops_per_call(int func_id, int n, int C);

bool chunk_compiled(int c);

// Launch shape of the per-call Fletcher-Powell kernel for n > 16: blocks of
// 16 variables, points per workgroup and column blocks per round (`points`
// and `blocks`, or chosen by a cost model where 0), row blocks per round
// (as many as fill the 16 lane rows), the split of a point group's rounds
// over workgroups, grid and LDS bytes.
struct FpDppGeometry {
    int nb = 0, ppw = 0, rb = 1, kbg = 1, rsplit = 1;
    int64_t grid = 0;
    size_t lds = 0;
};
FpDppGeometry fp_dpp_geometry(int n, int64_t npts, int points, int blocks, bool mixed);
// Launch shape of its symmetric form: the same cost model over the rounds
// of the block pairs kb >= ib (column blocks per round: `blocks`, or the
// model's where 0), one workgroup per point group.
FpDppGeometry fp_sym_geometry(int n, int64_t npts, int blocks, bool mixed);

// Current value of a chessfad_option.
int option_value(int option);

inline bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

}  // namespace chessfad
