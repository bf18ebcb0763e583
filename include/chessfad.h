/*
 * chessfad.h - C ABI of the MI355X (gfx950) chunked forward-mode Hessian library.
 *
 * The library computes, at many independent points, full Hessians and
 * Hessian-vector products of three test functions (Rosenbrock, Ackley,
 * Fletcher-Powell; Sec. VII) by the chunked forward-mode method of
 * Sec. III.B: every value is an hDual carrying the value, the derivative
 * with respect to the row variable x_i, a chunk of csize first derivatives
 * and the matching chunk of row i of the Hessian (Sec. IV), and f is
 * evaluated once per (point, row i, chunk) with CHUNK-INIT seeds.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer (hipMalloc'd memory or a
 *     torch CUDA tensor) owned by the caller; the library never frees it.
 *   - Arrays are dense, row-major and point-major: point p occupies
 *     x[p*n .. p*n+n), v[p*n .. p*n+n), out[p*n .. p*n+n) and, for Hessians,
 *     H[p*n*n .. p*n*n+n*n) with H[p][i][j] at p*n*n + i*n + j.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Compute calls
 *     only enqueue work and return without synchronising.
 *   - Return value: CHESSFAD_OK (0) or a negative chessfad_status.  All
 *     argument checks happen on the host before anything is enqueued; a
 *     failed check leaves every output untouched.  CHESSFAD_E_HIP reports a
 *     HIP launch/runtime error (text via chessfad_strerror).
 *   - npts == 0 is a no-op returning CHESSFAD_OK.
 *   - chunk is the chunk size csize; 0 picks the library default for
 *     (func_id, n).  Compiled sizes: 1, 2, 4, 8, 16.  chunk may not exceed
 *     n; when n is not a multiple of chunk the last chunk of every row is
 *     ragged (it seeds only the columns < n; Sec. III.B assumes csize | n).
 *   - x, v and the Fletcher-Powell parameters must be finite, and so must f
 *     and its derivatives at x: the kernels are built assuming finite values
 *     (non-finite inputs give unspecified results, not an error), and a
 *     zero result may come out as -0.0 or +0.0.
 *   - Calls on different streams are independent.  A Fletcher-Powell
 *     parameter set is complete on the device when chessfad_fp_set_params
 *     returns; replacing or releasing it waits for the work already enqueued
 *     on the device (hipFree), and compute calls made while it is replaced
 *     or released see the old set, the new one or CHESSFAD_E_PARAMS.
 */
#ifndef CHESSFAD_H
#define CHESSFAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum chessfad_func {
    CHESSFAD_ROSENBROCK = 0,      /* sum_{k<n-1} 100 (x_{k+1} - x_k^2)^2 + (1 - x_k)^2, n >= 2 */
    CHESSFAD_ACKLEY = 1,          /* -20 exp(-0.2 sqrt(sum x^2 / n)) - exp(sum cos(2 pi x) / n) + 20 + e */
    CHESSFAD_FLETCHER_POWELL = 2  /* sum_m (E_m - sum_j A_mj sin x_j + B_mj cos x_j)^2 */
};

enum chessfad_status {
    CHESSFAD_OK = 0,
    CHESSFAD_E_FUNC = -1,     /* func_id is neither a chessfad_func nor a registered user function,
                                 or the entry point does not take user functions */
    CHESSFAD_E_N = -2,        /* n < 1, n > CHESSFAD_MAX_N, or n < 2 for Rosenbrock */
    CHESSFAD_E_CHUNK = -3,    /* chunk not compiled, negative, or larger than n */
    CHESSFAD_E_NULL = -4,     /* a required pointer is NULL while npts > 0 */
    CHESSFAD_E_PARAMS = -5,   /* Fletcher-Powell parameters not set for this n */
    CHESSFAD_E_OVERLAP = -6,  /* an output array overlaps an input array */
    CHESSFAD_E_HIP = -7,      /* HIP error while allocating or launching */
    CHESSFAD_E_ARG = -8,      /* npts < 0 or another malformed argument */
    CHESSFAD_E_COMPILE = -9   /* a user function did not compile (chessfad_strerror gives the log) */
};

#define CHESSFAD_MAX_N 512

/* func_ids of registered user functions: CHESSFAD_USER_BASE + 0 .. CHESSFAD_MAX_USER - 1 */
#define CHESSFAD_USER_BASE 16
#define CHESSFAD_MAX_USER 64

/*
 * Hessian-vector products, plain float64 (CHESS-VEC, Sec. VI; Sec. III.C).
 *   x   [npts][n]  points at which H(x) is taken (read only)
 *   v   [npts][n]  vectors to multiply (read only)
 *   out [npts][n]  out[p] = H(x[p]) v[p]; must not overlap x or v
 * Row i of the Hessian is produced chunk by chunk, each chunk dotted with
 * the matching entries of v and summed (H is never stored).
 */
int chessfad_hvp(int func_id, int n, int64_t npts, const double* x, const double* v,
                 double* out, int chunk, void* stream);

/*
 * H.v together with the gradient and f (float64).  The calls that form H.v
 * also carry f's value and first derivatives (Sec. III.B: the second and
 * first hDual components), so the row's first call hands them out at no
 * extra evaluation:
 *   out  [npts][n]  H.v as chessfad_hvp computes it (the vector-ALU
 *                   functions run a separate instantiation of the kernel, so
 *                   the last bits may differ)
 *   grad [npts][n]  grad[p][i] = df/dx_i at x[p]  (required)
 *   fval [npts]     f(x[p])  (may be NULL)
 * grad and fval must not overlap x, v, out or each other (CHESSFAD_E_OVERLAP).
 * Always the L2 mapping; otherwise as chessfad_hvp.
 */
int chessfad_hvp_grad(int func_id, int n, int64_t npts, const double* x, const double* v,
                      double* out, double* grad, double* fval, int chunk, void* stream);

/*
 * Full Hessians, plain float64 (CHUNK-HESS, Sec. III.B).
 *   x [npts][n]     points (read only)
 *   H [npts][n][n]  H[p][i][j] = d2f/dx_i dx_j at x[p]; every entry is
 *                   computed by its own row's call (no symmetry is used),
 *                   so the output is symmetric only up to rounding.
 * chunk = 0: the largest compiled chunk <= n (at most 16), whatever the H.v
 * autotuner recorded: Hessians are bound by their stores, and a wide call
 * writes whole 16-byte pairs of its row (at n = 16 over 2^19 points: 0.41
 * against 0.82 ms at chunk 1 for Fletcher-Powell).
 */
int chessfad_hessian(int func_id, int n, int64_t npts, const double* x, double* H,
                     int chunk, void* stream);

/*
 * Mixed precision: the same H.v and Hessian with float32 hDual arithmetic
 * (same arguments, layouts and checks as chessfad_hvp / chessfad_hessian;
 * inputs and outputs stay float64).
 *   - every hDual component is carried in float32 (coordinates, v and the
 *     per-coordinate sin/cos tables are rounded to float32 where used);
 *   - the Hessian-chunk components of the Fletcher-Powell sum of squared
 *     residuals: for n <= 16 one float32 MFMA block over the residuals; for
 *     n > 16 plain float32 blocks of sixteen residuals entering a two-sum
 *     compensated running sum; Rosenbrock's and Ackley's sums, where each
 *     component has at most two nonzero terms and compensation cannot
 *     change the rounded result, are plain;
 *   - the chunk dot with v and the row sum over chunks are float64 (a
 *     float32 x float32 product is exact in float64);
 *   - per-point float64 islands: Ackley's two outer functions with their
 *     first two derivatives, and the Fletcher-Powell residual values
 *     E_m - sum_j (A_mj sin x_j + B_mj cos x_j), which cancel.
 * The error is bounded by float32 rounding of the inputs and of the hDual
 * arithmetic: normwise relative errors of a few 1e-7 on the test inputs.
 */
int chessfad_hvp_mixed(int func_id, int n, int64_t npts, const double* x, const double* v,
                       double* out, int chunk, void* stream);
int chessfad_hessian_mixed(int func_id, int n, int64_t npts, const double* x, double* H,
                           int chunk, void* stream);

/*
 * Symmetric forms (SCHUNK-HESS, Sec. III.B; SC-HESS-VEC, Sec. VI; count in
 * Sec. V).  Row i evaluates f only for its own chunk i / chunk and the
 * chunks after it: n (n / chunk + 1) / 2 calls per point when chunk divides
 * n, instead of n * ceil(n / chunk).  An entry H(i, s) of a later chunk
 * stands in for H(s, i):
 *   chessfad_hessian_sym  stores it at both places, so H is exactly
 *                         symmetric outside the diagonal blocks;
 *   chessfad_hvp_sym      adds H(i, s) v[s] to out[i] and H(i, s) v[i] to
 *                         out[s] (the mirror terms are summed in float64).
 * Arguments, layouts, ownership and checks as chessfad_hvp /
 * chessfad_hessian, plus
 *   precision  0: float64 hDuals; 1: the mixed-precision arithmetic of
 *              chessfad_hvp_mixed.  Anything else: CHESSFAD_E_ARG.
 *   chunk      0 picks the chessfad_autotune_sym choice if there is one,
 *              else the compiled chunk that minimises Sec. V's
 *              multiplication count (near sqrt(n / 2)).
 * The vector-ALU kernels hold a whole point's partial sums in LDS
 * (n * ceil(n / chunk) doubles for H.v): a chunk for which that does not
 * fit returns CHESSFAD_E_CHUNK (with chunk = 0 the next larger chunk that
 * fits is used).  Fletcher-Powell with n <= 16 runs on MFMA as in the full
 * form and has no such limit.
 */
int chessfad_hvp_sym(int func_id, int n, int64_t npts, const double* x, const double* v,
                     double* out, int chunk, int precision, void* stream);
int chessfad_hessian_sym(int func_id, int n, int64_t npts, const double* x, double* H,
                         int chunk, int precision, void* stream);

/*
 * User functions (the paper's library surface: "include the header; write f
 * templated on the data type", Sec. I, Sec. IV).  `source` is HIP C++ that
 * defines
 *     template <class V, class Y> __device__ V chessfad_user_f(const Y& y, int n);
 * over the hDual type and operators of chessfad_device.h (y[k], k < n, is
 * the k-th variable as an hDual; return f).  The library compiles it with
 * hipRTC for gfx950 together with that header (the call takes a second or
 * so), keeps the code object, and returns a func_id in *func_id.
 * chessfad_hvp and chessfad_hessian then accept that func_id for any n in
 * 1..CHESSFAD_MAX_N and chunk in {0 (= min(4, n) rounded down to a
 * compiled chunk), 1, 2, 4, 8, 16}; they run it in float64 on the paper's
 * L1 mapping (one lane per (point, row), walking the row's chunks).  The
 * other entry points return CHESSFAD_E_FUNC for user func_ids.
 * Errors: CHESSFAD_E_NULL for NULL arguments; CHESSFAD_E_COMPILE when the
 * source does not compile, with the compiler log available from
 * chessfad_strerror(CHESSFAD_E_COMPILE) on the same thread;
 * CHESSFAD_E_ARG when all CHESSFAD_MAX_USER slots are taken.
 * chessfad_release_function frees the slot and its code (the caller ensures
 * no enqueued work still runs it); CHESSFAD_E_FUNC for an unknown func_id.
 */
int chessfad_register_function(const char* source, int* func_id);
int chessfad_release_function(int func_id);

/*
 * Fletcher-Powell parameters for problem size n.  The function needs two
 * n x n integer-valued matrices A, B and a base point alpha; the method's
 * signatures have no slot for them, so they are registered per n.
 *   A, B   [n][n] device arrays (row-major), alpha [n] device array.
 * The library copies them into memory it owns, computes
 * E_m = sum_j A_mj sin(alpha_j) + B_mj cos(alpha_j) in float64 on `stream`,
 * synchronises `stream` (so compute calls on any stream may read the set
 * once this returns), and keeps the set until chessfad_fp_release(n) or a
 * new set for n.
 * Returns CHESSFAD_E_N for a bad n, CHESSFAD_E_NULL for a NULL array,
 * CHESSFAD_E_HIP if allocation or the copy fails.
 */
int chessfad_fp_set_params(int n, const double* A, const double* B, const double* alpha,
                           void* stream);

/* Frees the Fletcher-Powell parameter set of size n (no-op if none).  The
 * free waits for the work enqueued on the device (hipFree synchronises), and
 * it is serialised against the lookup and enqueue of compute calls. */
int chessfad_fp_release(int n);

/* Static description of a status code (for CHESSFAD_E_HIP, the text of the
 * last HIP error seen by the calling thread). */
const char* chessfad_strerror(int code);

/*
 * Process-wide options (not thread-safe against concurrent compute calls).
 * Returns the previous value, or CHESSFAD_E_ARG for an unknown option or value.
 *   CHESSFAD_OPT_FP_MFMA  the Fletcher-Powell engine for n <= 16:
 *                         1 (default): the per-call kernel: the dense value
 *                         contraction [A B] . [sin x; cos x] of every point on
 *                         MFMA, then per (point, row, chunk) call the
 *                         residuals' chunk components and the product rule
 *                         of their squares on the vector ALUs, each lane of a
 *                         point's 16-lane row holding one variable's column
 *                         and the call's chunk columns read from the other
 *                         lanes by DPP broadcasts (float32 products in the
 *                         mixed path); the symmetric form runs on engine 2;
 *                         2: the per-call kernel whose contractions of every
 *                         hDual component run on MFMA, the rest of each call
 *                         on the vector ALUs (full and symmetric form);
 *                         3: the closed form, not the chunked method: the
 *                         second-order components of all calls of a point as
 *                         one 16 x 16 MFMA tile 2 (J^T J + diag(D^T r)) whose
 *                         blocks the calls are (float32 MFMA in the mixed
 *                         path); for comparison;
 *                         0: every step of f on the vector ALUs.
 *                         All give the same derivative components; only the
 *                         order of the final sum over residuals differs.
 *                         Fletcher-Powell with n > 16: 1 runs the per-call
 *                         kernel for n > 16 (each lane row of 16 lanes holds
 *                         16 rows of one point; per call and residual the
 *                         lanes form their J entries elementwise and the
 *                         chunk's products read the chunk columns from the
 *                         other lanes by DPP broadcasts); 2 and 3 run the
 *                         row-block kernel that contracts the hDual columns
 *                         as 16 x 16 MFMA tiles; 0 the vector ALUs.
 *   CHESSFAD_OPT_FP_POINTS  points per workgroup of the per-call kernel for
 *                         Fletcher-Powell with n > 16: 16, 4 or 1, at most
 *                         16 / ceil(n / 16) (each point's rows then take
 *                         fewer row blocks per round); 0 (default): as many
 *                         as fill the workgroup's 16 lane rows with whole
 *                         rounds of row and column blocks.
 *   CHESSFAD_OPT_FP_BLOCKS  column blocks of 16 variables per round of the
 *                         same kernel (full and symmetric form): 1 .. 16 (at
 *                         most ceil(n / 16)); 0 (default): with the points
 *                         per workgroup, the count that a cost model of a
 *                         round (products per lane, J entries formed per
 *                         lane) finds cheapest.
 *   CHESSFAD_OPT_BATCH_TUNE  1 (default): chessfad_batch_create tunes the
 *                         body configuration of the instances with chunk 0
 *                         on the instances themselves (see below); 0: they
 *                         take the defaults.
 *   CHESSFAD_OPT_BATCH_GRAPH  1 (default): chessfad_batch_run replays the
 *                         plan's captured hipGraph; 0: it launches the same
 *                         kernels directly on the stream.
 *   CHESSFAD_OPT_MAPPING  the GPU mapping of chessfad_hvp and
 *                         chessfad_hvp_mixed (Sec. VI) where
 *                         f runs on the vector ALUs (Rosenbrock, Ackley;
 *                         Fletcher-Powell with CHESSFAD_OPT_FP_MFMA = 0):
 *                         2 (default): L2, one lane per (point, row, chunk)
 *                            (a row with a single chunk runs on the L1
 *                            kernel, the same mapping then; with chunk = 0
 *                            the mapping chessfad_autotune chose, if any);
 *                         1: L1, one lane per (point, row), walking its chunks;
 *                         0: L0, one lane per point, walking rows and chunks.
 *                         Every mapping computes the same sums in the same
 *                         order (the compiler may contract multiply-adds
 *                         differently in each kernel, so results can differ
 *                         in the last bits).  Other entry points always use
 *                         their own mapping.
 */
enum chessfad_option {
    CHESSFAD_OPT_FP_MFMA = 1,
    CHESSFAD_OPT_BATCH_GRAPH = 2,
    CHESSFAD_OPT_MAPPING = 3,
    CHESSFAD_OPT_FP_POINTS = 4,
    CHESSFAD_OPT_BATCH_TUNE = 5,
    CHESSFAD_OPT_FP_BLOCKS = 6
};
int chessfad_set_option(int option, int value);

/*
 * Batched H.v over many instances of mixed functions and sizes in one
 * persistent launch.
 *
 * An instance is one function with its own n, points, vectors, output,
 * chunk, precision, input/output type and (Fletcher-Powell) parameters.
 * chessfad_batch_create validates every instance (on failure *bad_index
 * names it), prepares the Fletcher-Powell offsets and float32 copies, and
 * splits every instance into work items of the single-instance kernels'
 * workgroup bodies (Rosenbrock and Ackley: the vector-ALU hDual evaluation
 * in the L1 mapping, one lane per (point, row), or the L2 mapping, one lane
 * per (point, row, chunk); Fletcher-Powell: the per-call kernel with DPP
 * lane broadcasts, one item per point group and share of its row blocks).
 * The items are sorted by their operation-count cost, largest first, and a
 * persistent kernel per (precision, body kind) - sized to fill the GPU -
 * takes them from an atomic counter until none is left.  The plan captures
 * a counter reset kernel and the persistent kernels in one hipGraph;
 * chessfad_batch_run replays it on `stream` (asynchronous; replays on one
 * stream are ordered, replays of one plan on different streams race on its
 * counters).
 *
 * chunk == 0 leaves the body configuration to the library.  With
 * CHESSFAD_OPT_BATCH_TUNE set (the default), chessfad_batch_create groups
 * those instances by (function, octave of n, precision) and times every
 * candidate configuration on each group's own instances - Rosenbrock and
 * Ackley: each compiled chunk up to the group's smallest n in the L1
 * mapping, and up to 8 in the L2 mapping; Fletcher-Powell: 16, 4 or 1
 * points per workgroup - keeping the fastest (the tuning runs write the
 * instances' outputs; chessfad_batch_choices lists the choices).  Otherwise
 * they take the autotuned chunk for (func_id, n, precision) if
 * chessfad_autotune has recorded one, else the default.  A given chunk must
 * be compiled (1, 2, 4, 8, 16) and at most n; Rosenbrock and Ackley run
 * chunks above 8, and rows of a single chunk, in the L1 mapping.
 * All arrays are device pointers that must stay valid while the plan is
 * used; outputs must not overlap their inputs.  With io_fp32 = 1, x, v and
 * out are float32 (the parameters A, B, alpha stay float64): the inputs are
 * widened on load and the float64 results rounded on store.
 * The plan owns its device memory (descriptors, work list, counters,
 * Fletcher-Powell offsets and float32 copies); chessfad_batch_destroy frees it.
 * Results are the same as chessfad_hvp / chessfad_hvp_mixed on each instance
 * in the same body configuration, up to the order of the sum over residuals
 * (Fletcher-Powell) and multiply-add contraction.
 */
typedef struct chessfad_instance {
    int func_id;          /* chessfad_func */
    int n;                /* variables, 1..CHESSFAD_MAX_N */
    int chunk;            /* 0 or a compiled chunk <= n */
    int precision;        /* 0: float64 hDuals; 1: mixed, as chessfad_hvp_mixed */
    int io_fp32;          /* 0: x, v, out are float64; 1: float32 */
    int64_t npts;         /* points of this instance, >= 0 */
    const void* x;        /* [npts][n] */
    const void* v;        /* [npts][n] */
    void* out;            /* [npts][n] */
    const double* A;      /* Fletcher-Powell only: [n][n] */
    const double* B;      /* Fletcher-Powell only: [n][n] */
    const double* alpha;  /* Fletcher-Powell only: [n] */
} chessfad_instance;

/* One plan-time tuning decision: the instances of func_id with n in
 * [n_lo, n_hi] (one octave) at `precision` run `chunk` with `mapping`
 * (Rosenbrock, Ackley: 1 = L1, 2 = L2) or `points` per workgroup and
 * `blocks` column blocks per round (Fletcher-Powell; 0 = the default, as
 * CHESSFAD_OPT_FP_POINTS / _FP_BLOCKS); ms is its time on those instances,
 * `candidates` the number of configurations timed. */
typedef struct chessfad_batch_choice {
    int func_id, n_lo, n_hi, precision, instances;
    int chunk, mapping, points, blocks, candidates;
    float ms;
} chessfad_batch_choice;

typedef struct chessfad_batch chessfad_batch;

int chessfad_batch_create(const chessfad_instance* inst, int ninst, void* stream, chessfad_batch** plan,
                          int* bad_index);
int chessfad_batch_run(chessfad_batch* plan, void* stream);
int chessfad_batch_destroy(chessfad_batch* plan);
/* Work items, persistent workgroups launched, and paper-model flops of one run. */
int chessfad_batch_info(const chessfad_batch* plan, int64_t* items, int* workgroups, double* model_flops);
/* The plan-time tuner's choices: up to `cap` into out[], their number in *count. */
int chessfad_batch_choices(const chessfad_batch* plan, chessfad_batch_choice* out, int cap, int* count);

/*
 * Allocation-free batched H.v, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Validates and plans the instances exactly as
 * chessfad_batch_create does with CHESSFAD_OPT_BATCH_TUNE = 0 (same work
 * items, same kernels, so the same results as such a plan of the same
 * instances; it does not tune), but places the plan - its
 * descriptors, work lists, counters and Fletcher-Powell offsets and float32
 * copies - in a fixed library-owned device array of
 * CHESSFAD_NOALLOC_SCRATCH_BYTES bytes instead of allocating, launches the
 * persistent kernels directly on `stream` (no graph), and waits for
 * `stream` before returning.  No device memory is allocated or freed (the
 * planning itself uses host memory).
 * Each GPU the library runs on holds one such array from its first use
 * until the process ends; every call on that GPU uses it, so calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.
 * Errors: as chessfad_batch_create (on a failed check *bad_index names the
 * instance; nothing is enqueued); CHESSFAD_E_ARG when the plan needs more
 * than CHESSFAD_NOALLOC_SCRATCH_BYTES bytes (8 bytes per work item and
 * about 100 per instance, plus per Fletcher-Powell instance 8n bytes of
 * offsets and, in mixed precision, 8n^2 bytes of float32 copies, each
 * rounded up to 256 bytes); CHESSFAD_E_HIP for a HIP error.
 */
#define CHESSFAD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int chessfad_batch_run_noalloc(const chessfad_instance* inst, int ninst, void* stream, int* bad_index);

/*
 * Launch shape of the per-call Fletcher-Powell kernel for 16 < n <= 512
 * (host only, no device work): what chessfad_hvp / _mixed (sym = 0) or
 * chessfad_hvp_sym (sym = 1) would launch for npts points at precision 0
 * or 1 under the current CHESSFAD_OPT_FP_POINTS / CHESSFAD_OPT_FP_BLOCKS.
 * Each of `points` points per workgroup takes, per round, row_blocks x
 * column_blocks (block of 16 rows, block of 16 columns) pairs on that many
 * 16-lane rows, a point group's rounds split over `split` workgroups; the
 * symmetric form takes only the pairs with column block >= row block, one
 * workgroup per point group (split = 1).  CHESSFAD_E_N for n outside 17 .. 512,
 * CHESSFAD_E_ARG for npts < 1 or another precision, CHESSFAD_E_NULL for
 * out == NULL.
 */
typedef struct {
    int points, row_blocks, column_blocks, split;
    int64_t grid;        /* workgroups */
    size_t lds_bytes;    /* per workgroup */
} chessfad_fp_shape;
int chessfad_fp_launch_shape(int n, int64_t npts, int precision, int sym, chessfad_fp_shape* out);

/*
 * Autotuner: times chessfad_hvp (precision 0) or chessfad_hvp_mixed (1) for
 * every compiled chunk <= n on npts device-generated points and records the
 * fastest for (func_id, n, precision) (a larger chunk within 2% of the
 * fastest time wins the tie: it makes fewer f calls); chunk == 0 then uses it (single calls
 * and batched plans; plans take recorded chunks <= 8, or <= 16 for
 * Fletcher-Powell).  Fletcher-Powell
 * needs its parameters registered for n.  Allocates and frees temporary
 * device memory and synchronises `stream`.  Returns the chosen chunk in
 * *best_chunk and its time per launch in *best_ms (either may be NULL).
 * For H.v whose f runs on the vector ALUs it times the L1 mapping beside
 * L2 at every chunk and records the faster one too, per precision:
 * chessfad_hvp (precision 0) or chessfad_hvp_mixed (1) with chunk = 0 then
 * runs that mapping (unless CHESSFAD_OPT_MAPPING is set to 0 or 1).
 */
int chessfad_autotune(int func_id, int n, int precision, int64_t npts, void* stream, int* best_chunk,
                      float* best_ms);

/* The same search for the symmetric H.v (chessfad_hvp_sym); the choice is
 * recorded for chunk = 0 in chessfad_hvp_sym / chessfad_hessian_sym.
 * Chunks whose symmetric workgroup does not fit in LDS are skipped;
 * CHESSFAD_E_CHUNK if none fits. */
int chessfad_autotune_sym(int func_id, int n, int precision, int64_t npts, void* stream,
                          int* best_chunk, float* best_ms);

/* Default chunk size the library uses for (func_id, n) when chunk == 0,
 * or a negative status for invalid arguments. */
int chessfad_default_chunk(int func_id, int n);

/* The GPU mapping chessfad_hvp (precision 0) or chessfad_hvp_mixed (1) uses
 * for (func_id, n) with chunk = 0 when f runs on the vector ALUs: 0 (L0),
 * 1 (L1) or 2 (L2); the option if set, else 1 when the chunk chunk = 0
 * resolves to leaves one chunk per row, else the tuned mapping, else 2.
 * Host only; a negative status for a bad func_id, n or precision. */
int chessfad_default_mapping(int func_id, int n, int precision);

#ifdef __cplusplus
}
#endif

#endif /* CHESSFAD_H */
