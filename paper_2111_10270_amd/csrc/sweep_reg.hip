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
// Register-resident sweep for tiles of the fast path (64 BDDs of one topology,
// fixed layer stride W, at most KMAX layers).  The node words are uniform
// across the wave, so every arc test is a scalar branch.  The layer loop is unrolled to KMAX with a uniform
// guard h < K, so every per-lane array below lives in VGPRs: the multipliers
// and averaged terms of all layers, the node words, and the opposite
// direction's distances.  All loads are issued before the first use.  The
// arithmetic is the same as in k_sweep (same operations, same order).
// ---------------------------------------------------------------------------
// v[c] for c < W, as a tree of selects on the bits of c (no indexed access,
// so the arrays stay in registers)
// Uniform arc penalty: 0 when the arc's head is `target`, +inf otherwise.
// Adding it to a value and taking a min routes the value along the arc with
// one v_add and one v_min, without branches or per-lane selects.
template <typename T>
__device__ __forceinline__ T pen(uint32_t head, uint32_t target);

// the selection happens on the scalar unit; the result is an SGPR operand
template <>
__device__ __forceinline__ float pen<float>(uint32_t head, uint32_t target)
{
    return __uint_as_float(uni(head == target ? 0u : 0x7F800000u));
}

template <>
__device__ __forceinline__ double pen<double>(uint32_t head, uint32_t target)
{
    const uint32_t hi = uni(head == target ? 0u : 0x7FF00000u);
    return __hiloint2double((int)hi, 0);
}

// min over next-layer nodes t of nx[t] + pen(head, t): the value at the arc's
// head for an arc that stays inside the BDD (heads of layers before the last)
template <int W, typename T>
__device__ __forceinline__ T head_inner(uint32_t head, const T (&nx)[W])
{
    T r = nx[0] + pen<T>(head, 0);
#pragma unroll
    for (int t = 1; t < W; ++t) r = fmin(r, nx[t] + pen<T>(head, (uint32_t)t));
    return r;
}

// value at the head of an arc of the last layer: 0 at the accepting terminal
template <typename T>
__device__ __forceinline__ T head_last(uint32_t head)
{
    return pen<T>(head, kTop);
}

// update == false: min-marginal differences at fixed multipliers (Alg. 2),
// written to mm, which is then output only.
template <typename T, int DIR, int W, int KMAX>
__global__ __launch_bounds__(kRegWaves * kLanes) void k_sweep_reg(DevProblem P, T *__restrict__ lam, T *mm,
                                                                   const T *__restrict__ abar,
                                                                   double *__restrict__ tile_lb, Omega<T> w,
                                                                   const int32_t *__restrict__ list,
                                                                   int64_t tile_count, int update)
{
    const T omega = w.w1;
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t lt = xcd_block() * kRegWaves + uni(threadIdx.x >> 6);
    if (lt >= tile_count) return;
    const int64_t tile = (int64_t)uni((uint32_t)list[lt]);
    const TileView tv = load_tile(P.tiles + tile);
    const int K = (int)tv.K;
    const T INF = inf_of<T>();

    // prologue: every load is issued before the first use
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
            if (update) {
                mo[h] = mm[s];
                cd[h] = P.code[tv.cb + (uint32_t)h * kLanes + lane];
            }
#pragma unroll
            for (int q = 0; q < W; ++q) wd[h][q] = uni(P.child[tv.nb + (uint32_t)(h * W + q)]);
        }
    }
    if (update) {
#pragma unroll
        for (int h = 0; h < KMAX; ++h)
            if (h < K) a[h] = averaged_term(mm, abar, tv.pb, tv.pb + (uint32_t)h * kLanes + lane, cd[h], mo[h], w);
    }

    double lbacc = 0.0;
    T energy;
    if (DIR == 0) {
        // SP(v, top) of every layer under the current multipliers; keep the
        // values at the heads of every arc for the update pass
        T hd0[KMAX][W], hd1[KMAX][W];
        T nx[W];
#pragma unroll
        for (int q = 0; q < W; ++q) nx[q] = INF;
#pragma unroll
        for (int h = KMAX - 1; h >= 0; --h) {
#pragma unroll
            for (int q = 0; q < W; ++q) {
                hd0[h][q] = INF;
                hd1[h][q] = INF;
            }
            if (h < K) {
                T b[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    const T v0 = (h == K - 1) ? head_last<T>(lo) : head_inner<W>(lo, nx);
                    const T v1 = (h == K - 1) ? head_last<T>(hi) : head_inner<W>(hi, nx);
                    hd0[h][q] = v0;
                    hd1[h][q] = v1;
                    b[q] = fmin(v0, v1 + l[h]);
                }
#pragma unroll
                for (int q = 0; q < W; ++q) nx[q] = b[q];
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
                T m0 = f[0] + hd0[h][0];
                T m1 = (f[0] + l[h]) + hd1[h][0];
#pragma unroll
                for (int q = 1; q < W; ++q) {
                    m0 = fmin(m0, f[q] + hd0[h][q]);
                    m1 = fmin(m1, (f[q] + l[h]) + hd1[h][q]);
                }
                const T M = m1 - m0;
                const T lu = update ? (l[h] - omega * M) + a[h] : l[h];
                const uint32_t s = tv.pb + (uint32_t)h * kLanes + lane;
                mm[s] = M;
                if (update) lam[s] = lu;
                lbacc += (double)fmin(M, T(0));
                if (h == K - 1) {
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                        top = fmin(top, fmin(f[q] + head_last<T>(lo), (f[q] + lu) + head_last<T>(hi)));
                    }
                } else {
                    T fn[W];
#pragma unroll
                    for (int t = 0; t < W; ++t) fn[t] = INF;
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                        const T v1 = f[q] + lu;
#pragma unroll
                        for (int t = 0; t < W; ++t)
                            fn[t] = fmin(fn[t], fmin(f[q] + pen<T>(lo, (uint32_t)t), v1 + pen<T>(hi, (uint32_t)t)));
                    }
#pragma unroll
                    for (int t = 0; t < W; ++t) f[t] = fn[t];
                }
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
                    const T v0 = fw[h][q], v1 = fw[h][q] + l[h];
#pragma unroll
                    for (int t = 0; t < W; ++t)
                        fw[h + 1][t] =
                            fmin(fw[h + 1][t], fmin(v0 + pen<T>(lo, (uint32_t)t), v1 + pen<T>(hi, (uint32_t)t)));
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
                T v0[W], v1[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    v0[q] = (h == K - 1) ? head_last<T>(lo) : head_inner<W>(lo, bn);
                    v1[q] = (h == K - 1) ? head_last<T>(hi) : head_inner<W>(hi, bn);
                }
                T m0 = fw[h][0] + v0[0];
                T m1 = (fw[h][0] + l[h]) + v1[0];
#pragma unroll
                for (int q = 1; q < W; ++q) {
                    m0 = fmin(m0, fw[h][q] + v0[q]);
                    m1 = fmin(m1, (fw[h][q] + l[h]) + v1[q]);
                }
                const T M = m1 - m0;
                const T lu = update ? (l[h] - omega * M) + a[h] : l[h];
                const uint32_t s = tv.pb + (uint32_t)h * kLanes + lane;
                mm[s] = M;
                if (update) lam[s] = lu;
                lbacc += (double)fmin(M, T(0));
#pragma unroll
                for (int q = 0; q < W; ++q) bn[q] = fmin(v0[q], v1[q] + lu);
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
                int update, hipStream_t st)
{
#define BDDMMA_REG(KI, KM)                                                                                         \
    {                                                                                                              \
        const int l = fast_list(wi, KI);                                                                           \
        const int64_t n = p.list_off[l + 1] - p.list_off[l];                                                       \
        if (n > 0)                                                                                                 \
            hipLaunchKernelGGL((k_sweep_reg<T, DIR, W, KM>), dim3(grid8(n, kRegWaves)), dim3(kRegWaves * kLanes), \
                               0, st, p, lam, mm, abar, tile_lb, w, p.lists + p.list_off[l], n, update);           \
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
                                                           const BDDMMA_REG_T *, double *, Omega<BDDMMA_REG_T>, int,
                                                           hipStream_t);
template void launch_reg<BDDMMA_REG_T, BDDMMA_REG_DIR, 4>(const DevProblem &, int, BDDMMA_REG_T *, BDDMMA_REG_T *,
                                                           const BDDMMA_REG_T *, double *, Omega<BDDMMA_REG_T>, int,
                                                           hipStream_t);

}  // namespace bddmma
