// batch_kernels.hpp -- gfx950 device code of the batched form: many independent
// cases of uneven size, relaxation time, time step and boundary kinds advanced by one
// persistent launch per time step, with the step kernel's per-wave march.
#pragma once
#include "kernels.hpp"

namespace lbfv {

// Work item of the batched form: case id, strip x0, rows [j0, j1).
struct BatchItem {
    int32_t c, x0, j0, j1;
};

// Batched persistent form: every wave walks the flat work list over all cases with a
// grid stride; each case carries its own mesh, tau, dt, boundaries and buffers.
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
        March<T, S, SCHEME, BND> m(P, src, dst, it.x0);
        m.run(it.j0, it.j1);
    }
}

}  // namespace lbfv
