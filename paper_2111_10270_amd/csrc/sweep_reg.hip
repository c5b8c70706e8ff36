// Register-resident sweep kernels of the fast path.  This file is compiled
// once per (precision, direction) pair, selected by BDDMMA_REG_T and
// BDDMMA_REG_DIR, so the heavily unrolled instantiations build in parallel.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

#ifndef BDDMMA_REG_T
#define BDDMMA_REG_T float
#endif
#ifndef BDDMMA_REG_DIR
#define BDDMMA_REG_DIR 0
#endif

namespace bddmma {

namespace {

// ---------------------------------------------------------------------------
// Register-resident sweep for tiles of the fast path (fixed layer stride W,
// at most KMAX layers).  The layer loop is unrolled to KMAX with a uniform
// guard h < K, so every per-lane array below lives in VGPRs: the multipliers
// and averaged terms of all layers, the node words, and the opposite
// direction's distances.  All loads are issued before the first use.  The
// arithmetic is the same as in k_sweep (same operations, same order).
// ---------------------------------------------------------------------------
// v[c] for c < W, as a tree of selects on the bits of c (no indexed access,
// so the arrays stay in registers)
template <int W, typename T>
__device__ __forceinline__ T pick(const T (&v)[W], uint32_t c)
{
    static_assert(W == 2 || W == 4, "fast path widths are 2 and 4");
    if constexpr (W == 2) {
        return (c == 1u) ? v[1] : v[0];
    } else {
        const T lo = (c & 1u) ? v[1] : v[0];
        const T hi = (c & 1u) ? v[3] : v[2];
        return (c & 2u) ? hi : lo;
    }
}

template <int W, typename T>
__device__ __forceinline__ T head(uint32_t c, const T (&next)[W])
{
    return c == kTop ? T(0) : (c == kBot ? inf_of<T>() : pick<W>(next, c));
}

template <int W, typename T>
__device__ __forceinline__ void push_min(T (&dst)[W], uint32_t c, T v)
{
    if constexpr (W == 2) {
#pragma unroll
        for (int q = 0; q < W; ++q)
            if (c == (uint32_t)q) dst[q] = tmin(dst[q], v);
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const T m = tmin(dst[q], v);
            dst[q] = (c == (uint32_t)q) ? m : dst[q];
        }
    }
}

// mm is read (previous M, in-tile averaging) before it is overwritten, so it
// is deliberately not __restrict__: the partner loads must stay ahead of the
// stores of this sweep.
template <typename T, int DIR, int W, int KMAX>
__global__ __launch_bounds__(kRegWaves * kLanes) void k_sweep_reg(DevProblem P, T *__restrict__ lam, T *mm,
                                                                   const T *__restrict__ abar,
                                                                   double *__restrict__ tile_lb, Omega<T> w,
                                                                   const int32_t *__restrict__ list,
                                                                   int64_t tile_count)
{
    const T omega = w.w1;
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t lt = xcd_block() * kRegWaves + uni(threadIdx.x >> 6);
    if (lt >= tile_count) return;
    const int64_t tile = (int64_t)uni((uint32_t)list[lt]);
    const TileView tv = load_tile(P.tiles + tile);
    const int K = (int)tv.K;
    const T INF = inf_of<T>();

    T l[KMAX], a[KMAX], mo[KMAX];
    uint32_t cd[KMAX];
    uint32_t wd[KMAX][W];
#pragma unroll
    for (int h = 0; h < KMAX; ++h) {
        l[h] = T(0);
        a[h] = T(0);
        mo[h] = T(0);
        cd[h] = kCodeSelf;
#pragma unroll
        for (int q = 0; q < W; ++q) wd[h][q] = kBot | (kBot << 16);
    }
#pragma unroll
    for (int h = 0; h < KMAX; ++h) {
        if (h < K) {
            const uint32_t s = tv.pb + (uint32_t)h * kLanes + lane;
            l[h] = lam[s];
            mo[h] = mm[s];
            cd[h] = P.code[s];
#pragma unroll
            for (int q = 0; q < W; ++q) wd[h][q] = node_word(P.child, tv, (uint32_t)(h * W + q), lane);
        }
    }
#pragma unroll
    for (int h = 0; h < KMAX; ++h)
        if (h < K) a[h] = averaged_term(mm, abar, tv.pb, tv.pb + (uint32_t)h * kLanes + lane, cd[h], mo[h], w);

    double lbacc = 0.0;
    T energy;
    if (DIR == 0) {
        // SP(v, top) of every layer under the current multipliers
        T bk[KMAX + 1][W];
#pragma unroll
        for (int h = 0; h <= KMAX; ++h)
#pragma unroll
            for (int q = 0; q < W; ++q) bk[h][q] = INF;
#pragma unroll
        for (int h = KMAX - 1; h >= 0; --h) {
            if (h < K) {
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t c = wd[h][q];
                    const T b0 = head<W>(c & 0xFFFFu, bk[h + 1]);
                    const T b1 = head<W>(c >> 16, bk[h + 1]) + l[h];
                    bk[h][q] = tmin(b0, b1);
                }
            }
        }
        // forward sweep with updates
        T f[W];
#pragma unroll
        for (int q = 0; q < W; ++q) f[q] = q == 0 ? T(0) : INF;
        T top = INF;
#pragma unroll
        for (int h = 0; h < KMAX; ++h) {
            if (h < K) {
                T m0 = INF, m1 = INF;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    if (lo != kBot) m0 = tmin(m0, f[q] + head<W>(lo, bk[h + 1]));
                    if (hi != kBot) m1 = tmin(m1, (f[q] + l[h]) + head<W>(hi, bk[h + 1]));
                }
                const T M = m1 - m0;
                const T lu = (l[h] - omega * M) + a[h];
                const uint32_t s = tv.pb + (uint32_t)h * kLanes + lane;
                mm[s] = M;
                lam[s] = lu;
                lbacc += (double)(M < T(0) ? M : T(0));
                T fn[W];
#pragma unroll
                for (int q = 0; q < W; ++q) fn[q] = INF;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    if (lo != kBot) {
                        if (lo == kTop) top = tmin(top, f[q]);
                        else push_min<W>(fn, lo, f[q]);
                    }
                    if (hi != kBot) {
                        const T v = f[q] + lu;
                        if (hi == kTop) top = tmin(top, v);
                        else push_min<W>(fn, hi, v);
                    }
                }
#pragma unroll
                for (int q = 0; q < W; ++q) f[q] = fn[q];
            }
        }
        energy = top;
    } else {
        // SP(root, v) of every layer under the current multipliers
        T fw[KMAX][W];
#pragma unroll
        for (int h = 0; h < KMAX; ++h)
#pragma unroll
            for (int q = 0; q < W; ++q) fw[h][q] = (h == 0 && q == 0) ? T(0) : INF;
#pragma unroll
        for (int h = 0; h + 1 < KMAX; ++h) {
            if (h + 1 < K) {
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    if (lo < kTop) push_min<W>(fw[h + 1], lo, fw[h][q]);
                    if (hi < kTop) push_min<W>(fw[h + 1], hi, fw[h][q] + l[h]);
                }
            }
        }
        // backward sweep with updates
        T bn[W];
#pragma unroll
        for (int q = 0; q < W; ++q) bn[q] = INF;
#pragma unroll
        for (int h = KMAX - 1; h >= 0; --h) {
            if (h < K) {
                T m0 = INF, m1 = INF;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    if (lo != kBot) m0 = tmin(m0, fw[h][q] + head<W>(lo, bn));
                    if (hi != kBot) m1 = tmin(m1, (fw[h][q] + l[h]) + head<W>(hi, bn));
                }
                const T M = m1 - m0;
                const T lu = (l[h] - omega * M) + a[h];
                const uint32_t s = tv.pb + (uint32_t)h * kLanes + lane;
                mm[s] = M;
                lam[s] = lu;
                lbacc += (double)(M < T(0) ? M : T(0));
                T bc[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t c = wd[h][q];
                    const T b0 = head<W>(c & 0xFFFFu, bn);
                    const T b1 = head<W>(c >> 16, bn) + lu;
                    bc[q] = tmin(b0, b1);
                }
#pragma unroll
                for (int q = 0; q < W; ++q) bn[q] = bc[q];
            }
        }
        energy = bn[0];
    }
    if (tile_lb) {
        const double e = wave_sum<T>((double)energy + (double)omega * lbacc);
        if (lane == 0) tile_lb[tile] = e;
    }
}

inline unsigned grid8(int64_t tiles, int per_block)
{
    return (unsigned)((((tiles + per_block - 1) / per_block) + 7) & ~int64_t(7));
}

}  // namespace

template <typename T, int DIR, int W>
void launch_reg(const DevProblem &p, int wi, T *lam, T *mm, const T *abar, double *tile_lb, Omega<T> w,
                hipStream_t st)
{
#define BDDMMA_REG(KI, KM)                                                                                         \
    {                                                                                                              \
        const int l = fast_list(wi, KI);                                                                           \
        const int64_t n = p.list_off[l + 1] - p.list_off[l];                                                       \
        if (n > 0)                                                                                                 \
            hipLaunchKernelGGL((k_sweep_reg<T, DIR, W, KM>), dim3(grid8(n, kRegWaves)), dim3(kRegWaves * kLanes), \
                               0, st, p, lam, mm, abar, tile_lb, w, p.lists + p.list_off[l], n);                   \
    }
    BDDMMA_REG(0, 4)
    BDDMMA_REG(1, 8)
    BDDMMA_REG(2, 12)
    BDDMMA_REG(3, 16)
    BDDMMA_REG(4, 24)
    BDDMMA_REG(5, 32)
#undef BDDMMA_REG
}

template void launch_reg<BDDMMA_REG_T, BDDMMA_REG_DIR, 2>(const DevProblem &, int, BDDMMA_REG_T *, BDDMMA_REG_T *,
                                                           const BDDMMA_REG_T *, double *, Omega<BDDMMA_REG_T>,
                                                           hipStream_t);
template void launch_reg<BDDMMA_REG_T, BDDMMA_REG_DIR, 4>(const DevProblem &, int, BDDMMA_REG_T *, BDDMMA_REG_T *,
                                                           const BDDMMA_REG_T *, double *, Omega<BDDMMA_REG_T>,
                                                           hipStream_t);

}  // namespace bddmma
