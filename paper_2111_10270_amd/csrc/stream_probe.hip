// bddmma_stream_probe: the in-place stream that bounds an updating sweep.
//
// An updating sweep reads the multipliers and differences of every slot of a
// tile and writes both back in place (Alg. 1); everything else it touches is
// small and cache-resident.  This kernel moves exactly those bytes in the
// same shape and nothing else, so its rate at a given array size is the
// bandwidth an updating sweep over arrays of that size can reach on the
// device, including the effect of the last-level cache when both arrays fit.
#include <hip/hip_runtime.h>

#include <string>

#include "bddmma.h"
#include "device_common.hpp"
#include "solver_internal.hpp"

namespace {

constexpr int kProbeRows = 9;      // rows of 64 elements per wave (the 9-layer register class)
constexpr int kProbeWaves = 4;     // waves per block

// wave w owns rows w*kProbeRows .. +kProbeRows-1 of both arrays: all loads
// first, then the stores (a + 1, b * 2)
template <typename T, bool FULL>
__device__ __forceinline__ void stream_rows(T *__restrict__ a, T *__restrict__ b, int64_t base, int64_t n)
{
    T x[kProbeRows], y[kProbeRows];
#pragma unroll
    for (int h = 0; h < kProbeRows; ++h) {
        const int64_t i = base + (int64_t)h * 64;
        x[h] = FULL || i < n ? a[i] : T(0);
        y[h] = FULL || i < n ? b[i] : T(0);
    }
#pragma unroll
    for (int h = 0; h < kProbeRows; ++h) {
        const int64_t i = base + (int64_t)h * 64;
        if (FULL || i < n) {
            a[i] = x[h] + T(1);
            b[i] = y[h] * T(2);
        }
    }
}

// blocks map to rows as the sweeps' blocks map to tiles (xcd_block: a run of
// consecutive blocks per XCD; the grid is a multiple of 8, blocks past the
// end have no rows)
template <typename T>
__global__ __launch_bounds__(64 * kProbeWaves) void k_stream_probe(T *__restrict__ a, T *__restrict__ b, int64_t n)
{
    const int64_t first = (bddmma::xcd_block() * kProbeWaves + (threadIdx.x >> 6)) * (kProbeRows * 64);
    const int64_t base = first + (threadIdx.x & 63);
    // whole rows without per-lane checks, so that all loads are in flight
    // before the first value is used (as in the sweep, whose tiles are whole)
    if (first + kProbeRows * 64 <= n)
        stream_rows<T, true>(a, b, base, n);
    else
        stream_rows<T, false>(a, b, base, n);
}

}  // namespace

extern "C" int bddmma_stream_probe(void *a, void *b, int64_t n, int32_t elem_bytes, void *hip_stream)
{
    using bddmma::set_error;
    if (n < 0) return set_error(BDDMMA_ERR_INVALID_ARG, "bddmma_stream_probe: n < 0");
    if (elem_bytes != 4 && elem_bytes != 8)
        return set_error(BDDMMA_ERR_INVALID_ARG, "bddmma_stream_probe: elem_bytes must be 4 or 8");
    if (n == 0) return BDDMMA_OK;
    if (!a || !b) return set_error(BDDMMA_ERR_INVALID_ARG, "bddmma_stream_probe: NULL array");
    const int64_t per_block = (int64_t)kProbeRows * 64 * kProbeWaves;
    const int64_t blocks = ((n + per_block - 1) / per_block + 7) & ~int64_t(7);
    if (blocks > 0x7FFFFFF8) return set_error(BDDMMA_ERR_INVALID_ARG, "bddmma_stream_probe: n too large");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_stream_probe<float>, dim3((unsigned)blocks), dim3(64 * kProbeWaves), 0, st,
                           static_cast<float *>(a), static_cast<float *>(b), n);
    else
        hipLaunchKernelGGL(k_stream_probe<double>, dim3((unsigned)blocks), dim3(64 * kProbeWaves), 0, st,
                           static_cast<double *>(a), static_cast<double *>(b), n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(BDDMMA_ERR_HIP, std::string("bddmma_stream_probe: ") + hipGetErrorString(e));
    return BDDMMA_OK;
}
