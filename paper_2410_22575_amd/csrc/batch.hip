// Batched plans (persistent kernel + hipGraph) and the chunk autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "dispatch.hpp"
#include "chessfad.h"
#include "fp_params.hpp"
#include "runtime.hpp"

using namespace chessfad;

struct chessfad_batch {
    int device = -1;
    char* dmem = nullptr;            // descriptors, work lists, counters, FP workspace
    unsigned* counters = nullptr;    // one per list
    // lists: index 2 * precision + kind (kind 0: vector rows, 1: FP MFMA rows)
    BatchArgs args[4] = {};
    int grid[4] = {0, 0, 0, 0};
    size_t lds[4] = {0, 0, 0, 0};
    int64_t items = 0;
    double flops = 0.0;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<chessfad_batch_choice> choices;   // the plan-time tuner's choices
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// An instance's body configuration: chunk, mapping of the vector bodies (1 =
// L1, 2 = L2), points per workgroup and column blocks per round of the
// Fletcher-Powell body; 0 = the default.
struct InstCfg {
    int C = 0, mapping = 0, points = 0, blocks = 0;
};

struct PlanEntry {
    BatchDesc d;
    int src;   // instance index
    int prec;
    int64_t blocks;
    double cost_per_block;  // paper-model flops of a full block
    size_t lds;             // LDS bytes of its body
};

template <class P>
size_t vector_lds(int func, int n, int pstride, int block) {
    return func == CHESSFAD_ROSENBROCK ? plain_lds_bytes<P, Rosenbrock>(n, pstride, block, false)
                                       : plain_lds_bytes<P, Ackley>(n, pstride, block, false);
}

using BatchKernel = void (*)(BatchArgs);

BatchKernel batch_kernel_for(int list) {
    switch (list) {
        case 0: return batch_kernel<F64, 0>;
        case 1: return batch_kernel<F64, 1>;
        case 2: return batch_kernel<F32C, 0>;
        default: return batch_kernel<F32C, 1>;
    }
}


void destroy(chessfad_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
}

// deterministic points in a function's domain for timing (splitmix64 hash)
__global__ void tune_fill_kernel(double* x, double* v, int64_t count, double lo, double hi) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    uint64_t z = (uint64_t)k * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    x[k] = lo + (hi - lo) * u;
    v[k] = u - 0.5;
}

}  // namespace

namespace {

// ------------------------------------------------------------ planning
// Everything a plan needs that does not depend on where its device memory
// lives: the validated instances, the sorted work lists, the byte layout of
// the plan's device memory, and the persistent grids.
struct PlanLayout {
    std::vector<PlanEntry> entries;
    std::vector<size_t> ws_off;  // per instance: offset of its Fletcher-Powell workspace
    std::vector<BatchDesc> descs[4];
    std::vector<BatchItem> flat[4];
    size_t off_desc[4] = {}, off_items[4] = {}, lds[4] = {};
    size_t off_counters = 0, off_ws = 0, total = 0;
    int grid[4] = {0, 0, 0, 0};
    int64_t items = 0;
    double flops = 0.0;
};

// Validates the instances and builds the work lists (host only; nothing is
// enqueued).  cfg (optional, one per instance) overrides the chunk, mapping
// and points per workgroup of instances.  On failure *bad_index names the
// instance.
int plan_instances(const chessfad_instance* inst, int ninst, int* bad_index, PlanLayout& L,
                   const InstCfg* cfg = nullptr) {
    if (bad_index) *bad_index = -1;
    if ((ninst > 0 && !inst) || ninst < 0) return CHESSFAD_E_ARG;
    L.entries.reserve(ninst);
    L.ws_off.assign(ninst, 0);
    size_t ws_bytes = 0;  // Fletcher-Powell workspace
    for (int k = 0; k < ninst; ++k) {
        const chessfad_instance& c = inst[k];
        auto bad = [&](int rc) {
            if (bad_index) *bad_index = k;
            return rc;
        };
        int rc = check_func_n(c.func_id, c.n);
        if (rc) return bad(rc);
        if (c.precision != 0 && c.precision != 1) return bad(CHESSFAD_E_ARG);
        if (c.io_fp32 != 0 && c.io_fp32 != 1) return bad(CHESSFAD_E_ARG);
        if (c.npts < 0) return bad(CHESSFAD_E_ARG);
        const bool fp = c.func_id == CHESSFAD_FLETCHER_POWELL;
        const InstCfg o = cfg ? cfg[k] : InstCfg{};
        const int C = o.C ? o.C : c.chunk ? c.chunk : resolve_chunk(c.func_id, c.n, c.precision, 16);
        if (C < 0 || !chunk_compiled(C) || C > c.n) return bad(CHESSFAD_E_CHUNK);
        const int nc = (c.n + C - 1) / C;
        // vector bodies: L1 for one chunk per row or C = 16 (L2 is compiled
        // for chunks up to 8), else the given or tuned mapping
        int mapping = 0;
        if (!fp) {
            mapping = o.mapping ? o.mapping : (nc == 1 || C > 8) ? 1 : tuned_mapping(c.func_id, c.n, c.precision);
            if (mapping != 1 && mapping != 2) return bad(CHESSFAD_E_ARG);
            if (mapping == 2 && (C > 8 || nc > kBatchThreads)) return bad(CHESSFAD_E_CHUNK);
        }
        if (c.npts == 0) continue;
        if (!c.x || !c.v || !c.out) return bad(CHESSFAD_E_NULL);
        if (fp && (!c.A || !c.B || !c.alpha)) return bad(CHESSFAD_E_PARAMS);
        const size_t bytes = (c.io_fp32 ? sizeof(float) : sizeof(double)) * (size_t)c.npts * c.n;
        if (overlaps(c.out, bytes, c.x, bytes) || overlaps(c.out, bytes, c.v, bytes)) return bad(CHESSFAD_E_OVERLAP);

        PlanEntry e{};
        e.src = k;
        e.prec = c.precision;
        e.d.func = c.func_id;
        e.d.C = C;
        e.d.n = c.n;
        e.d.nc = nc;
        e.d.io32 = c.io_fp32;
        e.d.npts = c.npts;
        e.d.x = static_cast<const double*>(c.x);
        e.d.v = static_cast<const double*>(c.v);
        e.d.out = static_cast<double*>(c.out);
        e.d.fp = FpParams{c.A, c.B, nullptr, nullptr, nullptr};
        const double per_call = model_flops_per_call(c.func_id, c.n, C);
        if (fp) {
            const FpDppGeometry g = fp_dpp_geometry(c.n, c.npts, o.points, o.blocks, c.precision == 1);
            e.d.kind = 1;
            e.d.nb = g.nb;
            e.d.ppw = g.ppw;
            e.d.rb = g.rb;
            e.d.kbg = g.kbg;
            e.d.rsplit = g.rsplit;
            e.blocks = g.grid;
            e.lds = g.lds;
            e.cost_per_block = per_call * (double)c.n * nc * g.ppw / g.rsplit;
            L.ws_off[k] = ws_bytes;
            ws_bytes += align_up(sizeof(double) * c.n, 256);
            if (c.precision == 1) ws_bytes += 2 * align_up(sizeof(float) * (size_t)c.n * c.n, 256);
        } else {
            e.d.kind = 0;
            e.d.mapping = mapping;
            e.d.rows = mapping == 1 ? kBatchThreads : kBatchThreads / nc;
            e.d.pstride = (e.d.rows - 1) / c.n + 2;
            e.blocks = (c.npts * c.n + e.d.rows - 1) / e.d.rows;
            const int block = mapping == 1 ? 0 : e.d.rows * nc;
            e.lds = c.precision ? vector_lds<F32C>(c.func_id, c.n, e.d.pstride, block)
                                : vector_lds<F64>(c.func_id, c.n, e.d.pstride, block);
            e.cost_per_block = per_call * e.d.rows * nc;
        }
        if (e.blocks > 0x7fffffffLL) return bad(CHESSFAD_E_ARG);
        L.entries.push_back(e);
    }

    // the byte layout: descriptors, items, counters, Fletcher-Powell workspace
    size_t nitems[4] = {0, 0, 0, 0}, ndesc[4] = {0, 0, 0, 0};
    for (const PlanEntry& e : L.entries) {
        nitems[2 * e.prec + e.d.kind] += (size_t)e.blocks;
        ndesc[2 * e.prec + e.d.kind] += 1;
    }
    size_t total = 0;
    for (int l = 0; l < 4; ++l) {
        L.off_desc[l] = total;
        total = align_up(total + sizeof(BatchDesc) * ndesc[l], 256);
        L.off_items[l] = total;
        total = align_up(total + sizeof(BatchItem) * nitems[l], 256);
    }
    L.off_counters = total;
    total = align_up(total + 4 * sizeof(unsigned), 256);
    L.off_ws = total;
    L.total = total + ws_bytes;

    // work lists per (precision, kind), largest model cost first; a
    // descriptor's index in its list is its position among the list's entries
    std::vector<std::pair<double, BatchItem>> items[4];
    int ndescs[4] = {0, 0, 0, 0};
    for (const PlanEntry& e : L.entries) {
        const int list = 2 * e.prec + e.d.kind;
        const int di = ndescs[list]++;
        for (int64_t blk = 0; blk < e.blocks; ++blk) {
            double cost = e.cost_per_block;
            if (e.d.kind == 0) {
                const int64_t q0 = blk * e.d.rows, rows = std::min<int64_t>(e.d.rows, e.d.npts * e.d.n - q0);
                cost = cost * (double)rows / e.d.rows;
            }
            items[list].push_back({cost, BatchItem{di, (int)blk}});
            L.flops += cost;
        }
    }
    for (int l = 0; l < 4; ++l) {
        std::stable_sort(items[l].begin(), items[l].end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        L.flat[l].reserve(items[l].size());
        for (const auto& it : items[l]) L.flat[l].push_back(it.second);
        L.items += (int64_t)L.flat[l].size();
        for (const PlanEntry& e : L.entries)
            if (2 * e.prec + e.d.kind == l) L.lds[l] = std::max(L.lds[l], e.lds);
    }
    return CHESSFAD_OK;
}

// Sizes the persistent grids for `device` (occupancy x compute units, at
// most one workgroup per item).
hipError_t size_grids(PlanLayout& L, int device) {
    int cus = 0;
    hipError_t err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    for (int l = 0; l < 4 && err == hipSuccess; ++l) {
        L.grid[l] = 0;
        if (L.flat[l].empty()) continue;
        int per_cu = 0;
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel_for(l), kBatchThreads, L.lds[l]);
        L.grid[l] = (int)std::min<int64_t>((int64_t)std::max(per_cu, 1) * cus, (int64_t)L.flat[l].size());
    }
    return err;
}

// Places the plan in the device memory at `base` (L.total bytes): enqueues
// the Fletcher-Powell offsets and float32 copies and the uploads of the
// descriptors and work lists on `s`, and fills args.  The host arrays are
// read by the copies, so the caller keeps L alive until `s` has passed them.
hipError_t materialize(PlanLayout& L, const chessfad_instance* inst, char* base, hipStream_t s, BatchArgs args[4],
                       unsigned*& counters) {
    hipError_t err = hipSuccess;
    counters = reinterpret_cast<unsigned*>(base + L.off_counters);
    for (int l = 0; l < 4; ++l) L.descs[l].clear();
    for (PlanEntry& e : L.entries) {
        if (e.d.kind == 1 && err == hipSuccess) {
            const chessfad_instance& c = inst[e.src];
            char* w = base + L.off_ws + L.ws_off[e.src];
            double* E = reinterpret_cast<double*>(w);
            float* A32 = reinterpret_cast<float*>(w + align_up(sizeof(double) * c.n, 256));
            float* B32 = reinterpret_cast<float*>(reinterpret_cast<char*>(A32) +
                                                  align_up(sizeof(float) * (size_t)c.n * c.n, 256));
            hipLaunchKernelGGL(fp_offsets_kernel, dim3((c.n + 63) / 64), dim3(64), 0, s, c.n, c.A, c.B, c.alpha, E);
            err = hipGetLastError();
            if (c.precision == 1 && err == hipSuccess) {
                const int count = c.n * c.n;
                hipLaunchKernelGGL(fp_to_f32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, count, c.A, c.B,
                                   A32, B32, nullptr);
                err = hipGetLastError();
            }
            e.d.fp = c.precision == 1 ? FpParams{c.A, c.B, E, A32, B32} : FpParams{c.A, c.B, E, nullptr, nullptr};
        }
        L.descs[2 * e.prec + e.d.kind].push_back(e.d);
    }
    for (int l = 0; l < 4 && err == hipSuccess; ++l) {
        BatchDesc* dd = reinterpret_cast<BatchDesc*>(base + L.off_desc[l]);
        BatchItem* di = reinterpret_cast<BatchItem*>(base + L.off_items[l]);
        if (!L.descs[l].empty())
            err = hipMemcpyAsync(dd, L.descs[l].data(), sizeof(BatchDesc) * L.descs[l].size(), hipMemcpyHostToDevice, s);
        if (err == hipSuccess && !L.flat[l].empty())
            err = hipMemcpyAsync(di, L.flat[l].data(), sizeof(BatchItem) * L.flat[l].size(), hipMemcpyHostToDevice, s);
        args[l] = BatchArgs{dd, di, (int)L.flat[l].size(), counters + l};
    }
    return err;
}

hipError_t launch_lists(const BatchArgs args[4], const int grid[4], const size_t lds[4], unsigned* counters,
                        hipStream_t s) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, counters, 4);
    hipError_t e = hipGetLastError();
    for (int l = 0; l < 4 && e == hipSuccess; ++l) {
        if (!args[l].nitems) continue;
        hipLaunchKernelGGL(batch_kernel_for(l), dim3(grid[l]), dim3(kBatchThreads), lds[l], s, args[l]);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_all(chessfad_batch* b, hipStream_t s) { return launch_lists(b->args, b->grid, b->lds, b->counters, s); }

// ------------------------------------------------------ plan-time tuning
// For the instances that leave the chunk to the library, grouped by
// (function, octave of n, precision): each candidate body configuration is
// timed on the group's own instances (a plan of just those, one warm-up and
// two timed runs of its persistent kernels; the runs write the instances'
// outputs) and the fastest is kept; a larger chunk within 2% of the fastest
// wins (fewer f calls).  Candidates: Rosenbrock and Ackley, every compiled
// chunk up to the group's smallest n in the L1 mapping and, up to 8 with
// several chunks per row, in the L2 mapping; Fletcher-Powell, the largest
// chunk up to 16 at 16, 4 and 1 points per workgroup and the default, each
// with the default column blocks per round and with as many as the
// variables have (up to 16).
int tune_plan(const chessfad_instance* inst, int ninst, hipStream_t s, std::vector<InstCfg>& cfg,
              std::vector<chessfad_batch_choice>& choices) {
    struct Group {
        int func, prec, nmin = 1 << 30, nmax = 0;
        std::vector<int> members;
    };
    std::map<std::tuple<int, int, int>, Group> groups;
    for (int k = 0; k < ninst; ++k) {
        const chessfad_instance& c = inst[k];
        if (c.chunk != 0 || c.npts <= 0 || check_func_n(c.func_id, c.n) != CHESSFAD_OK) continue;
        int oct = 0;
        while ((2 << oct) <= c.n) ++oct;
        Group& g = groups[std::make_tuple(c.func_id, oct, c.precision)];
        g.func = c.func_id;
        g.prec = c.precision;
        g.nmin = std::min(g.nmin, c.n);
        g.nmax = std::max(g.nmax, c.n);
        g.members.push_back(k);
    }
    if (groups.empty()) return CHESSFAD_OK;
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    for (auto& kv : groups) {
        if (err != hipSuccess) break;
        Group& g = kv.second;
        std::vector<InstCfg> cands;
        if (g.func == CHESSFAD_FLETCHER_POWELL) {
            int C = 1;
            for (int k = 0; k < kNumChunks; ++k)
                if (kChunks[k] <= std::min(16, g.nmin)) C = kChunks[k];
            for (int blocks : {0, 16})
                for (int pts : {0, 16, 4, 1}) cands.push_back(InstCfg{C, 0, pts, blocks});
        } else {
            for (int k = 0; k < kNumChunks; ++k) {
                const int C = kChunks[k];
                if (C > g.nmin) break;
                cands.push_back(InstCfg{C, 1, 0});
                if (C <= 8 && C < g.nmax) cands.push_back(InstCfg{C, 2, 0});
            }
        }
        std::vector<chessfad_instance> sub;
        for (int k : g.members) sub.push_back(inst[k]);
        const int m = (int)sub.size();
        float best_ms = -1.0f, fastest = -1.0f;
        std::vector<float> times(cands.size(), -1.0f);
        for (size_t ci = 0; ci < cands.size() && err == hipSuccess; ++ci) {
            std::vector<InstCfg> cc(m, cands[ci]);
            PlanLayout L;
            if (plan_instances(sub.data(), m, nullptr, L, cc.data()) != CHESSFAD_OK) continue;
            char* mem = nullptr;
            err = hipMalloc(&mem, std::max<size_t>(L.total, 256));
            if (err == hipSuccess) err = size_grids(L, device);
            BatchArgs args[4];
            unsigned* counters = nullptr;
            if (err == hipSuccess) err = materialize(L, sub.data(), mem, s, args, counters);
            if (err == hipSuccess) err = launch_lists(args, L.grid, L.lds, counters, s);
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            for (int r = 0; r < 2 && err == hipSuccess; ++r) err = launch_lists(args, L.grid, L.lds, counters, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (mem) (void)hipFree(mem);
            if (err != hipSuccess) break;
            times[ci] = ms / 2.0f;
            if (fastest < 0.0f || times[ci] < fastest) fastest = times[ci];
        }
        if (err != hipSuccess || fastest < 0.0f) continue;
        int pick = -1;
        for (size_t ci = 0; ci < cands.size(); ++ci)
            if (times[ci] >= 0.0f && times[ci] <= 1.02f * fastest &&
                (pick < 0 || cands[ci].C > cands[pick].C || (cands[ci].C == cands[pick].C && times[ci] < best_ms))) {
                pick = (int)ci;
                best_ms = times[ci];
            }
        for (int k : g.members) cfg[k] = cands[pick];
        chessfad_batch_choice ch{};
        ch.func_id = g.func;
        ch.n_lo = g.nmin;
        ch.n_hi = g.nmax;
        ch.precision = g.prec;
        ch.instances = m;
        ch.chunk = cands[pick].C;
        ch.mapping = cands[pick].mapping;
        ch.points = cands[pick].points;
        ch.blocks = cands[pick].blocks;
        ch.ms = best_ms;
        ch.candidates = (int)cands.size();
        choices.push_back(ch);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return err == hipSuccess ? CHESSFAD_OK : hip_fail(err);
}


// ------------------------------------------------ allocation-free batches
// The device memory of chessfad_batch_run_noalloc: one fixed array per GPU
// (each device holds its own copy of this module's globals), kept until the
// process ends.  Host code never passes `scratch` itself to the device: its
// address on a device comes from hipGetSymbolAddress, taken once per device
// with that device current.
constexpr size_t kScratchBytes = CHESSFAD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[64] = {};

hipError_t scratch_base(int device, char** base) {
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<char*>(ptr);
    }
    *base = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" {

int chessfad_batch_create(const chessfad_instance* inst, int ninst, void* stream, chessfad_batch** plan,
                          int* bad_index) {
    if (bad_index) *bad_index = -1;
    if (!plan) return CHESSFAD_E_ARG;
    *plan = nullptr;
    PlanLayout L;
    int rc = plan_instances(inst, ninst, bad_index, L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<chessfad_batch_choice> choices;
    if (option_value(CHESSFAD_OPT_BATCH_TUNE)) {
        // the instances were valid as given; re-plan them with the tuned bodies
        std::vector<InstCfg> cfg(ninst);
        rc = tune_plan(inst, ninst, s, cfg, choices);
        if (rc) return rc;
        L = PlanLayout{};
        rc = plan_instances(inst, ninst, bad_index, L, cfg.data());
        if (rc) return rc;
    }
    chessfad_batch* b = new chessfad_batch;
    b->choices = std::move(choices);
    hipError_t err = hipGetDevice(&b->device);
    if (err == hipSuccess) err = hipMalloc(&b->dmem, std::max<size_t>(L.total, 256));
    if (err == hipSuccess) err = size_grids(L, b->device);
    if (err == hipSuccess) err = materialize(L, inst, b->dmem, s, b->args, b->counters);
    // the uploads read L's host arrays
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
        destroy(b);
        return hip_fail(err);
    }
    for (int l = 0; l < 4; ++l) {
        b->grid[l] = L.grid[l];
        b->lds[l] = L.lds[l];
    }
    b->items = L.items;
    b->flops = L.flops;
    // capture reset + persistent kernels in one graph
    err = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
        hipError_t le = launch_all(b, b->capture);
        err = hipStreamEndCapture(b->capture, &b->graph);
        if (err == hipSuccess) err = le;
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        destroy(b);
        return hip_fail(err);
    }
    *plan = b;
    return CHESSFAD_OK;
}

int chessfad_batch_run_noalloc(const chessfad_instance* inst, int ninst, void* stream, int* bad_index) {
    if (bad_index) *bad_index = -1;
    PlanLayout L;
    const int rc = plan_instances(inst, ninst, bad_index, L);
    if (rc) return rc;
    if (L.total > kScratchBytes) return CHESSFAD_E_ARG;
    if (L.items == 0) return CHESSFAD_OK;
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    char* base = nullptr;
    if (err == hipSuccess) err = scratch_base(device, &base);
    if (err == hipSuccess) err = size_grids(L, device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchArgs args[4];
    unsigned* counters = nullptr;
    if (err == hipSuccess) err = materialize(L, inst, base, s, args, counters);
    if (err == hipSuccess) err = launch_lists(args, L.grid, L.lds, counters, s);
    // the uploads read L's host arrays, and the next call on this GPU reuses
    // the array: wait for this call's work
    const hipError_t serr = hipStreamSynchronize(s);
    if (err == hipSuccess) err = serr;
    return err == hipSuccess ? CHESSFAD_OK : hip_fail(err);
}

int chessfad_batch_run(chessfad_batch* plan, void* stream) {
    if (!plan) return CHESSFAD_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = option_value(CHESSFAD_OPT_BATCH_GRAPH) ? hipGraphLaunch(plan->exec, s) : launch_all(plan, s);
    return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
}

int chessfad_batch_destroy(chessfad_batch* plan) {
    if (!plan) return CHESSFAD_E_ARG;
    destroy(plan);
    return CHESSFAD_OK;
}

int chessfad_batch_choices(const chessfad_batch* plan, chessfad_batch_choice* out, int cap, int* count) {
    if (!plan || cap < 0 || (cap > 0 && !out)) return CHESSFAD_E_ARG;
    const int total = (int)plan->choices.size();
    for (int k = 0; k < total && k < cap; ++k) out[k] = plan->choices[k];
    if (count) *count = total;
    return CHESSFAD_OK;
}

int chessfad_batch_info(const chessfad_batch* plan, int64_t* items, int* workgroups, double* model_flops) {
    if (!plan) return CHESSFAD_E_ARG;
    if (items) *items = plan->items;
    if (workgroups) *workgroups = plan->grid[0] + plan->grid[1] + plan->grid[2] + plan->grid[3];
    if (model_flops) *model_flops = plan->flops;
    return CHESSFAD_OK;
}

}  // extern "C"

namespace {

// Times H.v (full or symmetric form) at every compiled chunk <= n and records
// the choice for chunk = 0.  A symmetric chunk whose workgroup does not fit
// in LDS is skipped.
int autotune(int func_id, int n, int precision, int64_t npts, void* stream, int* best_chunk, float* best_ms,
             bool sym) {
    int rc = check_func_n(func_id, n);
    if (rc) return rc;
    if ((precision != 0 && precision != 1) || npts <= 0) return CHESSFAD_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t count = (size_t)npts * n;
    double *x = nullptr, *v = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipMalloc(&x, count * sizeof(double));
    if (err == hipSuccess) err = hipMalloc(&v, count * sizeof(double));
    if (err == hipSuccess) err = hipMalloc(&out, count * sizeof(double));
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    const double lo = func_id == CHESSFAD_ROSENBROCK ? -2.0 : func_id == CHESSFAD_ACKLEY ? -5.0 : -3.141592653589793;
    if (err == hipSuccess) {
        hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x, v,
                           (int64_t)count, lo, -lo);
        err = hipGetLastError();
    }
    // H.v on the vector path: the L1 mapping is timed beside L2
    const bool two_maps = !sym && vector_path(func_id);
    float times[kNumChunks];
    int maps[kNumChunks];
    int tried = 0;
    // the point tile runs the same launch for every chunk: time the largest only
    const bool tile = fp_tile_path(func_id, n);
    for (int k = 0; k < kNumChunks && err == hipSuccess && rc == CHESSFAD_OK; ++k) {
        const int C = kChunks[k];
        if (C > n) break;
        times[k] = -1.0f;
        maps[k] = 2;
        tried = k + 1;
        if (tile && k + 1 < kNumChunks && kChunks[k + 1] <= n) continue;
        const bool both = two_maps && (n + C - 1) / C > 1;
        for (int level = 2; level >= (both ? 1 : 2) && err == hipSuccess && rc == CHESSFAD_OK; --level) {
            const int map = sym ? -1 : level;
            rc = run_single(func_id, n, npts, x, v, out, C, stream, false, precision == 1, sym, nullptr, nullptr,
                            map);  // warm-up
            if (sym && rc == CHESSFAD_E_CHUNK) {
                rc = CHESSFAD_OK;
                break;
            }
            if (rc) break;
            err = hipEventRecord(e0, s);
            for (int r = 0; r < 3 && rc == CHESSFAD_OK; ++r)
                rc = run_single(func_id, n, npts, x, v, out, C, stream, false, precision == 1, sym, nullptr, nullptr,
                                map);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            ms /= 3.0f;
            if (times[k] < 0.0f || ms < times[k]) {
                times[k] = ms;
                maps[k] = level;
            }
        }
    }
    // the largest chunk within 2% (timing noise) of the fastest: fewer f calls
    // for the same Hessian entries
    int best = 0, best_map = 2;
    float best_t = 0.0f;
    if (err == hipSuccess && rc == CHESSFAD_OK && tried > 0) {
        float fastest = -1.0f;
        for (int k = 0; k < tried; ++k)
            if (times[k] >= 0.0f && (fastest < 0.0f || times[k] < fastest)) fastest = times[k];
        for (int k = 0; k < tried; ++k)
            if (times[k] >= 0.0f && times[k] <= 1.02f * fastest) {
                best = kChunks[k];
                best_t = times[k];
                best_map = maps[k];
            }
    }
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (x) (void)hipFree(x);
    if (v) (void)hipFree(v);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (err != hipSuccess) return hip_fail(err);
    if (!best) return CHESSFAD_E_CHUNK;
    record_tuned_chunk(func_id, n, precision, best, sym);
    if (two_maps) record_tuned_mapping(func_id, n, precision, best_map);
    if (best_chunk) *best_chunk = best;
    if (best_ms) *best_ms = best_t;
    return CHESSFAD_OK;
}

}  // namespace

extern "C" {

int chessfad_autotune(int func_id, int n, int precision, int64_t npts, void* stream, int* best_chunk,
                      float* best_ms) {
    return autotune(func_id, n, precision, npts, stream, best_chunk, best_ms, false);
}

int chessfad_autotune_sym(int func_id, int n, int precision, int64_t npts, void* stream, int* best_chunk,
                          float* best_ms) {
    return autotune(func_id, n, precision, npts, stream, best_chunk, best_ms, true);
}

}  // extern "C"
