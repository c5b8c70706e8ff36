// Device helpers shared by the solver's HIP translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "layout.hpp"

namespace bddmma {
namespace {

constexpr int kWavesPerBlock = 2;
constexpr int kThreads = kWavesPerBlock * kLanes;
constexpr int kRedThreads = 256;
constexpr int kPrefetch = 8;
constexpr int kRegWaves = 4;

template <typename T>
__device__ __forceinline__ T inf_of();
template <>
__device__ __forceinline__ float inf_of<float>() { return __builtin_huge_valf(); }
template <>
__device__ __forceinline__ double inf_of<double>() { return __builtin_huge_val(); }

__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// Blocks are handed to the 8 XCDs round robin; remap so that consecutive
// logical blocks (and hence neighbouring tiles, which share variables) run on
// the same XCD and share its L2.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t b = blockIdx.x, per = gridDim.x >> 3;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int64_t grid_round8(int64_t blocks) { return (blocks + 7) & ~int64_t(7); }

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return b < a ? b : a; }

struct TileView {
    uint32_t pb, nb, lb, cb, fb, K, NN;
    bool shared;
};

__device__ __forceinline__ TileView load_tile(const TileDesc *td)
{
    TileView v;
    v.pb = uni(td->pair_base);
    v.nb = uni(td->node_base);
    v.lb = uni(td->layer_base);
    v.cb = uni(td->code_base);
    v.fb = uni(td->fast_base);
    v.K = uni(td->K);
    v.NN = uni(td->nodes);
    v.shared = (uni(td->flags) & TILE_SHARED) != 0;
    return v;
}

__device__ __forceinline__ uint32_t node_word(const uint32_t *__restrict__ child, const TileView &tv, uint32_t node,
                                              int lane)
{
    return tv.shared ? child[tv.nb + node] : child[tv.nb + (size_t)node * kLanes + lane];
}

// value of an arc's head in the distance-to-accept array (layer offset noffn)
template <typename T>
__device__ __forceinline__ T head_val(uint32_t c, const T *Bk, uint32_t noffn)
{
    return c == kTop ? T(0) : (c == kBot ? inf_of<T>() : Bk[(size_t)(noffn + c) * kLanes]);
}

template <typename T>
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanes);
    return v;
}


// averaged term of slot s from its code (layout.hpp); mo = mm[s] on entry to
// the sweep, which for slots averaged by the averaging kernel is the term itself
template <typename T>
__device__ __forceinline__ T averaged_term(const T *mm, uint32_t pb, uint32_t code, T mo, Omega<T> w)
{
    if (code == kCodeGlobal) return mo;
    if (code == kCodeSelf) return w.w1 * mo;
    return w.w2 * (mo + mm[pb + code]);
}

}  // namespace
}  // namespace bddmma
