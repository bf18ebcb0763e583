// Persistent batched H.v over many instances of mixed functions and sizes.
//
// A plan turns a list of instances (function, n, points, chunk, precision,
// float32 or float64 I/O) into work items (instance, workgroup block) of the
// workgroup bodies the single-instance kernels use: for Rosenbrock and Ackley
// the vector-ALU hDual evaluation in the L1 mapping (coarse_block) or the L2
// mapping (plain_block), for Fletcher-Powell the per-call kernel with DPP lane
// broadcasts (fp_dpp_block).  Items are sorted by their paper-model cost,
// largest first, and a persistent kernel - one per precision and body kind,
// sized to fill the chip - takes them from an atomic counter until its list
// is exhausted (longest-processing-time-first list scheduling).  Every
// workgroup leaves the loop when the counter passes the end of the list.  The
// two body kinds get separate persistent kernels and lists, so each is
// compiled with the registers its own bodies need.
#pragma once

#include <stdint.h>

#include "kernel_fp_dpp.hpp"
#include "kernel_plain.hpp"

namespace chessfad {

constexpr int kBatchThreads = 256;

struct BatchDesc {
    int kind;        // 0: vector bodies (Rosenbrock, Ackley), 1: the Fletcher-Powell per-call body
    int func;
    int C;
    int n, nc;
    int mapping;     // kind 0: 1 = L1 (coarse_block), 2 = L2 (plain_block)
    int rows;        // kind 0: row tasks per item
    int pstride;     // kind 0: LDS rows per staged array
    int nb, ppw, rb, kbg, rsplit;   // kind 1: the per-call kernel's geometry
    int io32;        // x, v, out are float32
    int64_t npts;
    const double* x;
    const double* v;
    double* out;
    FpParams fp;
};

struct BatchItem {
    int inst;
    int blk;
};

struct BatchArgs {
    const BatchDesc* desc;
    const BatchItem* items;
    int nitems;
    unsigned* counter;
};

template <class P, class F>
__device__ __forceinline__ void batch_plain(const PlainArgs& pa, int C, int64_t blk, double* lds) {
    switch (C) {
        case 1: plain_block<P, F, 1, false>(pa, blk, lds); break;
        case 2: plain_block<P, F, 2, false>(pa, blk, lds); break;
        case 4: plain_block<P, F, 4, false>(pa, blk, lds); break;
        default: plain_block<P, F, 8, false>(pa, blk, lds); break;
    }
}

template <class P, class F>
__device__ __forceinline__ void batch_coarse(const PlainArgs& pa, int C, int64_t blk, double* lds) {
    switch (C) {
        case 1: coarse_block<P, F, 1, 1>(pa, blk, lds); break;
        case 2: coarse_block<P, F, 2, 1>(pa, blk, lds); break;
        case 4: coarse_block<P, F, 4, 1>(pa, blk, lds); break;
        case 8: coarse_block<P, F, 8, 1>(pa, blk, lds); break;
        default: coarse_block<P, F, 16, 1>(pa, blk, lds); break;
    }
}

template <class P, int kKind>
__global__ __launch_bounds__(kBatchThreads) void batch_kernel(BatchArgs b) {
    extern __shared__ double lds[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(b.counter, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= b.nitems) break;
        const BatchItem item = b.items[it];
        const BatchDesc d = b.desc[item.inst];
        if constexpr (kKind == 1) {
            FpDppArgs fa{d.x, d.v, d.out, d.fp, d.npts, d.n, d.nb, d.ppw, d.rb, d.kbg, d.rsplit, nullptr, nullptr,
                         d.io32};
            const int64_t pg = item.blk / d.rsplit;
            int ibr0, ibr1;
            fp_dpp_rounds(d.nb, d.rb, d.rsplit, (int)(item.blk - pg * d.rsplit), ibr0, ibr1);
            switch (d.C) {
                case 1: fp_dpp_block<P, 1, false, false>(fa, pg, ibr0, ibr1, lds); break;
                case 2: fp_dpp_block<P, 2, false, false>(fa, pg, ibr0, ibr1, lds); break;
                case 4: fp_dpp_block<P, 4, false, false>(fa, pg, ibr0, ibr1, lds); break;
                case 8: fp_dpp_block<P, 8, false, false>(fa, pg, ibr0, ibr1, lds); break;
                default: fp_dpp_block<P, 16, false, false>(fa, pg, ibr0, ibr1, lds); break;
            }
        } else {
            PlainArgs pa{d.x, d.v, d.out, d.fp, d.npts, d.n, d.nc, d.rows, d.pstride, nullptr, nullptr, d.io32};
            if (d.mapping == 1) {
                if (d.func == 0)
                    batch_coarse<P, Rosenbrock>(pa, d.C, item.blk, lds);
                else
                    batch_coarse<P, Ackley>(pa, d.C, item.blk, lds);
            } else {
                if (d.func == 0)
                    batch_plain<P, Rosenbrock>(pa, d.C, item.blk, lds);
                else
                    batch_plain<P, Ackley>(pa, d.C, item.blk, lds);
            }
        }
    }
}

// counters[0..k) = 0 (a kernel rather than a memset node, so the graph can
// be replayed safely)
__global__ void batch_reset_kernel(unsigned* counters, int k) {
    if ((int)threadIdx.x < k) counters[threadIdx.x] = 0u;
}

}  // namespace chessfad
