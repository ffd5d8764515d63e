// Device side of the batched launch (many Algorithm 3 solves of uneven size
// in one persistent launch, Sec. 4 per instance): the kernel template,
// instantiated per operator kind in batch_stencil.hip and batch_csr.hip so
// that the large kernels compile in parallel.  Host side: batch.hip.
#pragma once

#include "solve_body.h"

namespace phc {

// Variant of an instance inside the batched kernel: R (1..4) and the row
// layout (1, 2 or 4 rows per thread with E in registers, or E in memory).
constexpr int kLayouts = 4;
constexpr int kLayoutEmem = 3;

template <int KIND, int R, bool MIX>
__device__ __forceinline__ void run_layout(int layout, const SolveArgs &P, SolveShared &sh,
                                           unsigned G, unsigned bid) {
    switch (layout) {
    case 0: solve_body<KIND, R, 1, false, MIX>(P, sh, G, bid, (int)bid); break;
    case 1: solve_body<KIND, R, 2, false, MIX>(P, sh, G, bid, (int)bid); break;
    case 2: solve_body<KIND, R, 4, false, MIX>(P, sh, G, bid, (int)bid); break;
    default: solve_body<KIND, R, 1, true, MIX>(P, sh, G, bid, (int)bid); break;
    }
}

// wg_group[b]: group of workgroup b; gfirst/gsize: first workgroup and size of
// each group; glist[goff[g] .. goff[g+1]): the instances group g runs, in order.
// ts[it][0..1]: device wall clock at the start and end of instance it (for
// the cost model's calibration).
template <int KIND, bool MIX>
__global__ __launch_bounds__(kNT) void solve_batch_kernel(const SolveArgs *__restrict__ args,
                                                          const int *__restrict__ variant,
                                                          const int *__restrict__ wg_group,
                                                          const int *__restrict__ gfirst,
                                                          const int *__restrict__ gsize,
                                                          const int *__restrict__ goff,
                                                          const int *__restrict__ glist,
                                                          long long *__restrict__ ts) {
    __shared__ SolveShared sh;
    const int g = wg_group[blockIdx.x];
    const unsigned G = (unsigned)gsize[g];
    const unsigned bid = blockIdx.x - (unsigned)gfirst[g];
    for (int q = goff[g]; q < goff[g + 1]; ++q) {
        const int it = glist[q];
        const SolveArgs &P = args[it];
        const int v = variant[it];
        const int layout = v % kLayouts;
        if (bid == 0 && threadIdx.x == 0)
            ts[2 * it] = wall_clock64();
        switch (v / kLayouts) {
        case 0: run_layout<KIND, 1, MIX>(layout, P, sh, G, bid); break;
        case 1: run_layout<KIND, 2, MIX>(layout, P, sh, G, bid); break;
        case 2: run_layout<KIND, 3, MIX>(layout, P, sh, G, bid); break;
        default: run_layout<KIND, 4, MIX>(layout, P, sh, G, bid); break;
        }
        if (bid == 0 && threadIdx.x == 0)
            ts[2 * it + 1] = wall_clock64();
        __syncthreads();   // the next instance reuses the shared state
    }
}

using BatchKernel = void (*)(const SolveArgs *, const int *, const int *, const int *,
                             const int *, const int *, const int *, long long *);

// Kernel of the batched launch for one operator kind (stencil or CSR).
BatchKernel batch_kernel_stencil(bool mix);
BatchKernel batch_kernel_csr(bool mix);

}  // namespace phc
