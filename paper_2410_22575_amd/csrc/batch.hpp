// Persistent batched H.v over many instances of mixed functions and sizes.
//
// A plan turns a list of instances (function, n, points, chunk, precision)
// into work items (instance, workgroup block) of the same two block bodies
// the single-instance kernels use: plain_block (Rosenbrock, Ackley; the
// vector-ALU hDual evaluation) and fp_rows_block (Fletcher-Powell on MFMA,
// calls as matrix columns).  Items are sorted by their paper-model cost,
// largest first, and a persistent kernel - one per precision and body kind,
// sized to fill the chip - takes them from an atomic counter until its list is exhausted
// (longest-processing-time-first list scheduling).  Every workgroup leaves
// the loop when the counter passes the end of the list.  The two body kinds
// get separate persistent kernels and lists, so each is compiled with the
// registers its own bodies need.
#pragma once

#include <stdint.h>

#include "kernel_fp_rows.hpp"
#include "kernel_plain.hpp"

namespace chessfad {

constexpr int kBatchThreads = 256;

struct BatchDesc {
    int kind;        // 0: plain_block, 1: fp_rows_block
    int func;
    int C;
    int n, nc;
    int rows;        // rows per item
    int pstride;     // plain_block LDS stride
    int row_blocks;  // fp_rows_block items per point
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
            FpRowsArgs fa{d.x, d.v, d.out, d.fp, d.npts, d.n, d.nc, d.rows, d.row_blocks};
            FpRowsShared<typename P::T>& sh = *reinterpret_cast<FpRowsShared<typename P::T>*>(lds);
            switch (d.C) {
                case 1: fp_rows_block<P, 1, false>(fa, item.blk, sh); break;
                case 2: fp_rows_block<P, 2, false>(fa, item.blk, sh); break;
                case 4: fp_rows_block<P, 4, false>(fa, item.blk, sh); break;
                case 8: fp_rows_block<P, 8, false>(fa, item.blk, sh); break;
                default: fp_rows_block<P, 16, false>(fa, item.blk, sh); break;
            }
        } else {
            PlainArgs pa{d.x, d.v, d.out, d.fp, d.npts, d.n, d.nc, d.rows, d.pstride};
            if (d.func == 0)
                batch_plain<P, Rosenbrock>(pa, d.C, item.blk, lds);
            else
                batch_plain<P, Ackley>(pa, d.C, item.blk, lds);
        }
    }
}

// counters[0..k) = 0 (a kernel rather than a memset node, so the graph can
// be replayed safely)
__global__ void batch_reset_kernel(unsigned* counters, int k) {
    if ((int)threadIdx.x < k) counters[threadIdx.x] = 0u;
}

}  // namespace chessfad
