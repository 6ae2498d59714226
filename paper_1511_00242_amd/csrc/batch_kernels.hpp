// batch_kernels.hpp -- gfx950 device code of the batched form: many independent
// cases of uneven size, relaxation time, time step and boundary kinds advanced by one
// launch per time step (or per two), with the step kernels' per-wave marches.
#pragma once
#include "kernels.hpp"

namespace lbfv {

// Work item of the batched form: case id, strip x0, rows [j0, j1).
struct BatchItem {
    int32_t c, x0, j0, j1;
};

// Batched form: every wave walks the flat work list over all cases with a grid stride
// (a grid of one wave per item takes one item per wave); each case carries its own
// mesh, tau, dt, boundaries and buffers.
template <typename T, typename S, int SCHEME, bool BND>
__global__ __launch_bounds__(256) void batch_kernel(const StepParams<T> *__restrict__ cases,
                                                    const BatchItem *__restrict__ items, int nitems,
                                                    int parity) {
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    int w = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (int)(threadIdx.x >> 6));
    for (; w < nitems; w += nw) {
        const BatchItem it = items[w];
        // a reference into the case table: a local copy would be indexed dynamically
        // (sides, buffers) and live in scratch memory
        const StepParams<T> &P = cases[it.c];
        const S *src = (const S *)P.buf[parity];
        S *dst = (S *)P.buf[parity ^ 1];
        March<T, S, SCHEME, BND, 1, false> m(P, src, dst, it.x0);
        m.run(it.j0, it.j1);
    }
}

// Two time steps per launch of the batched form (every case in the 60-column strip
// layout): a wave whose row block needs no ghost rows takes the rotating march (x-side
// ghost lanes refilled where the strip has them), the others the march with level-1 ghost
// rows, as in the single-case two-step kernel.
template <typename T, typename S, int SCHEME, bool BND>
__global__ __launch_bounds__(256) void batch2_kernel(const StepParams<T> *__restrict__ cases,
                                                     const BatchItem *__restrict__ items, int nitems,
                                                     int parity) {
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    int w = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (int)(threadIdx.x >> 6));
    for (; w < nitems; w += nw) {
        const BatchItem it = items[w];
        const StepParams<T> &P = cases[it.c];
        const S *src = (const S *)P.buf[parity];
        S *dst = (S *)P.buf[parity ^ 1];
        March<T, S, SCHEME, BND, 2, false> m(P, src, dst, it.x0);
        if constexpr (BND) {
            const bool inner_y = m.per_y || (it.j0 >= 2 && it.j1 <= P.ny - 2);
            if (inner_y) m.run2(it.j0, it.j1);
            else m.run2b(it.j0, it.j1);
        } else {
            m.run2(it.j0, it.j1);
        }
    }
}

// Two time steps per launch of the batched form split over a pair of waves per work item
// (a workgroup of two waves; as step2p_kernel / step2bp_kernel): the workgroup walks the
// work list with a grid stride, both waves taking the same items, so both pass the same
// barriers.  The same bits as batch2_kernel.
template <typename T, typename S, int SCHEME, bool BND>
__global__ __launch_bounds__(128) void batch2p_kernel(const StepParams<T> *__restrict__ cases,
                                                      const BatchItem *__restrict__ items, int nitems,
                                                      int parity) {
    __shared__ T ring[2 * 9 * 64];
    const bool producer = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) == 0;
    for (int w = xcd_block(); w < nitems; w += gridDim.x) {
        const BatchItem it = items[w];
        const StepParams<T> &P = cases[it.c];
        const S *src = (const S *)P.buf[parity];
        S *dst = (S *)P.buf[parity ^ 1];
        March<T, S, SCHEME, BND, 2, false> m(P, src, dst, it.x0);
        bool inner = true;
        if constexpr (BND) inner = m.per_y || (it.j0 >= 2 && it.j1 <= P.ny - 2);
        if (inner) {
            if (producer) m.produce(it.j0, it.j1, ring);
            else m.consume(it.j0, it.j1, ring);
        } else {
            if (producer) m.produce_b(it.j0, it.j1, ring);
            else m.consume_b(it.j0, it.j1, ring);
        }
    }
}

}  // namespace lbfv
