// Copy kernel of the device batch assembly: each block handles up to
// kSegChunk elements of one segment (assemble.hpp): plain copies, index
// shifts and fills of the member images into the batch's tables.
#include <hip/hip_runtime.h>

#include "assemble.hpp"

namespace bddmma {

namespace {

__global__ __launch_bounds__(256) void k_assemble(const Seg *__restrict__ segs, const int64_t *__restrict__ items)
{
    const int64_t si = items[2 * blockIdx.x], begin = items[2 * blockIdx.x + 1];
    const Seg g = segs[si];
    const int64_t end = begin + kSegChunk < g.n ? begin + kSegChunk : g.n;
    for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
        if (g.elem == 1) {
            uint8_t *d = reinterpret_cast<uint8_t *>(g.dst);
            d[i] = g.op == SEG_FILL ? (uint8_t)g.a : reinterpret_cast<const uint8_t *>(g.src)[i];
        } else if (g.elem == 2) {
            uint16_t *d = reinterpret_cast<uint16_t *>(g.dst);
            d[i] = g.op == SEG_FILL ? (uint16_t)g.a : reinterpret_cast<const uint16_t *>(g.src)[i];
        } else if (g.elem == 4) {
            int32_t v = g.op == SEG_FILL ? (int32_t)g.a : reinterpret_cast<const int32_t *>(g.src)[i];
            if (g.op == SEG_ADD) v += (int32_t)g.a;
            else if (g.op == SEG_PADVAR) v = v == (int32_t)g.b ? (int32_t)g.c : v + (int32_t)g.a;
            reinterpret_cast<int32_t *>(g.dst)[i] = v;
        } else {
            int64_t v = g.op == SEG_FILL ? g.a : reinterpret_cast<const int64_t *>(g.src)[i];
            if (g.op == SEG_ADD) v += g.a;
            reinterpret_cast<int64_t *>(g.dst)[i] = v;
        }
    }
}

}  // namespace

// items: n_items pairs (segment index, first element), device memory
void launch_assemble(const Seg *segs, const int64_t *items, int64_t n_items, hipStream_t st)
{
    if (n_items > 0) hipLaunchKernelGGL(k_assemble, dim3((unsigned)n_items), dim3(256), 0, st, segs, items);
}

}  // namespace bddmma
