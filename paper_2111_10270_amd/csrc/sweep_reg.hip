// Register-resident sweep kernels of the fast path.  This file is compiled
// once per (precision, direction, update) triple, selected by BDDMMA_REG_T,
// BDDMMA_REG_DIR and BDDMMA_REG_UPD, so the heavily unrolled instantiations
// build in parallel.
#include <hip/hip_runtime.h>

#include <utility>

#include "device_common.hpp"
#include "kernels.hpp"
#include "sweep_tile.hpp"

#ifndef BDDMMA_REG_T
#define BDDMMA_REG_T float
#endif
#ifndef BDDMMA_REG_DIR
#define BDDMMA_REG_DIR 0
#endif
#ifndef BDDMMA_REG_UPD
#define BDDMMA_REG_UPD true
#endif

namespace bddmma {

namespace {

// One wave per tile of `list` (tiles first, first + 1, ... when first >= 0);
// the sweep of the tile is sweep_tile.
template <typename T, int DIR, int W, int KMAX, bool UPD, bool SH, bool GAT>
__global__ __launch_bounds__(kRegWaves * kLanes) void k_sweep_reg(DevProblem P, T *__restrict__ lam,
                                                                   T *__restrict__ mm, double *__restrict__ tile_lb,
                                                                   Omega<T> w, const int32_t *__restrict__ list,
                                                                   int64_t tile_count, int32_t first)
{
    extern __shared__ __align__(16) unsigned char lds_bytes[];
    const int64_t lt = xcd_block() * (int64_t)(blockDim.x >> 6) + uni(threadIdx.x >> 6);
    if (lt >= tile_count) return;
    const int64_t tile = first >= 0 ? first + lt : (int64_t)uni((uint32_t)list[lt]);
    T *sh = reinterpret_cast<T *>(lds_bytes) + (size_t)uni(threadIdx.x >> 6) * KMAX * kLanes;
    sweep_tile<T, DIR, W, KMAX, UPD, SH, GAT>(P, lam, mm, tile_lb, w, tile, sh);
}

// ---------------------------------------------------------------------------
// Long width-2 tiles (more layers than the register classes): the arithmetic
// of k_sweep_reg (same operations, same order) over layer chunks of kChunk
// held in registers.  The first pass runs in the opposite direction without
// updates and stores, per layer, the two distances the update pass needs
// (DIR 1: SP(root, v) of the layer; DIR 0: SP(v, top) of the next layer) and,
// with UPD, the averaged term, computed before any M of the tile is
// overwritten.  The update pass reads them back chunk by chunk.
// ---------------------------------------------------------------------------
constexpr int kChunk = 8;

// per-chunk register state; loads for chunk c+1 are issued before chunk c is
// computed, so a wave overlaps its memory latency with its own arithmetic
template <typename T, int W>
struct LongChunk {
    T l[kChunk];              // multipliers
    uint32_t wd[kChunk][W];   // node words
    T d[kChunk][W];           // stored distances (update pass)
    T a[kChunk];              // averaged terms (update pass)
    T mo[kChunk];             // previous M (first pass, UPD)
    uint32_t cd[kChunk];      // averaging codes (first pass, UPD)
};

template <typename T, int DIR, bool UPD, bool SH>
__global__ __launch_bounds__(kRegWaves * kLanes) void k_sweep_long(DevProblem P, T *__restrict__ lam,
                                                                    T *__restrict__ mm, double *__restrict__ tile_lb,
                                                                    Omega<T> w, const int32_t *__restrict__ list,
                                                                    int64_t tile_count)
{
    constexpr int W = 2;
    const T omega = w.w1;
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t lt = xcd_block() * (int64_t)(blockDim.x >> 6) + uni(threadIdx.x >> 6);
    if (lt >= tile_count) return;
    const int64_t tile = (int64_t)uni((uint32_t)list[lt]);
    const TileView tv = load_tile(P.tiles + tile);
    const int K = (int)tv.K;
    const T INF = inf_of<T>();
    T *const lrow = lam + tv.pb + lane;
    T *const mtile = mm + tv.pb;
    T *const mrow = mtile + lane;
    const uint16_t *const crow = P.code + tv.cb + lane;
    const uint32_t *const wrow = P.child + tv.fb + (SH ? 0 : lane);
    T *const sp = reinterpret_cast<T *>(P.scratch) + (size_t)uni(P.tiles[tile].scratch_base) + lane;
    T *const sa = sp + (size_t)2 * K * kLanes;   // averaged terms
    const int nchunk = (K + kChunk - 1) / kChunk;
    using Chunk = LongChunk<T, W>;

    // first pass loads: multipliers, node words, and with UPD the previous M
    // and the codes (no store of this sweep has touched M yet)
    auto load_first = [&](int c, Chunk &k) {
        const int c0 = c * kChunk;
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int h = c0 + u;
            k.l[u] = T(0);
            k.mo[u] = T(0);
            k.cd[u] = kCodeSelf;
#pragma unroll
            for (int q = 0; q < W; ++q) k.wd[u][q] = kBot | (kBot << 16);
            if (h < K) {
                k.l[u] = lrow[(size_t)h * kLanes];
#pragma unroll
                for (int q = 0; q < W; ++q)
                    k.wd[u][q] = SH ? uni(wrow[h * W + q]) : wrow[(size_t)(h * W + q) * kLanes];
                if (UPD) {
                    k.mo[u] = mrow[(size_t)h * kLanes];
                    k.cd[u] = crow[(size_t)h * kLanes];
                }
            }
        }
    };
    // update pass loads: multipliers, node words, stored distances and terms
    auto load_second = [&](int c, Chunk &k) {
        const int c0 = c * kChunk;
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int h = c0 + u;
            k.l[u] = T(0);
            k.a[u] = T(0);
#pragma unroll
            for (int q = 0; q < W; ++q) {
                k.wd[u][q] = kBot | (kBot << 16);
                k.d[u][q] = INF;
            }
            if (h < K) {
                k.l[u] = lrow[(size_t)h * kLanes];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    k.wd[u][q] = SH ? uni(wrow[h * W + q]) : wrow[(size_t)(h * W + q) * kLanes];
                    k.d[u][q] = sp[(size_t)(2 * h + q) * kLanes];
                }
                if (UPD) k.a[u] = sa[(size_t)h * kLanes];
            }
        }
    };
    // averaged terms of a chunk (same formula as k_sweep_reg): issue the
    // partner loads, return them for the store after the chunk's arithmetic
    auto partner_loads = [&](int c, const Chunk &k, T (&x)[kChunk]) {
        const int c0 = c * kChunk;
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int h = c0 + u;
            x[u] = T(0);
            if (h < K) x[u] = mtile[k.cd[u] < kCodeSelf ? k.cd[u] : (uint32_t)(h * kLanes + lane)];
        }
    };
    auto store_terms = [&](int c, const Chunk &k, const T (&x)[kChunk]) {
        const int c0 = c * kChunk;
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int h = c0 + u;
            if (h < K) {
                const T cf = k.cd[u] == kCodeGlobal ? T(0.5) : w.w2;
                sa[(size_t)h * kLanes] = cf * (k.mo[u] + x[u]);
            }
        }
    };

    double lbacc = 0.0;
    T energy;
    if (DIR == 0) {
        // first pass, descending: store the next layer's distances to top
        T nx[W];
#pragma unroll
        for (int q = 0; q < W; ++q) nx[q] = q == 0 ? T(0) : INF;   // terminal layer
        Chunk cur, nxt;
        load_first(nchunk - 1, cur);
        for (int c = nchunk - 1; c >= 0; --c) {
            if (c > 0) load_first(c - 1, nxt);
            T x[kChunk];
            if (UPD) partner_loads(c, cur, x);
            const int c0 = c * kChunk;
#pragma unroll
            for (int u = kChunk - 1; u >= 0; --u) {
                const int h = c0 + u;
                if (h < K) {
#pragma unroll
                    for (int q = 0; q < W; ++q) sp[(size_t)(2 * h + q) * kLanes] = nx[q];
                    T b[W];
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t lo = cur.wd[u][q] & 0xFFFFu, hi = cur.wd[u][q] >> 16;
                        b[q] = fmin(head_at<SH, W>(lo, nx), head_at<SH, W>(hi, nx) + cur.l[u]);
                    }
#pragma unroll
                    for (int q = 0; q < W; ++q) nx[q] = b[q];
                }
            }
            if (UPD) store_terms(c, cur, x);
            cur = nxt;
        }
        // update pass, ascending
        T f[W];
#pragma unroll
        for (int q = 0; q < W; ++q) f[q] = q == 0 ? T(0) : INF;
        load_second(0, cur);
        for (int c = 0; c < nchunk; ++c) {
            if (c + 1 < nchunk) load_second(c + 1, nxt);
            const int c0 = c * kChunk;
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int h = c0 + u;
                if (h < K) {
                    T hd0[W], hd1[W];
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t lo = cur.wd[u][q] & 0xFFFFu, hi = cur.wd[u][q] >> 16;
                        hd0[q] = head_at<SH, W>(lo, cur.d[u]);
                        hd1[q] = head_at<SH, W>(hi, cur.d[u]);
                    }
                    T m0 = f[0] + hd0[0];
                    T m1 = (f[0] + cur.l[u]) + hd1[0];
#pragma unroll
                    for (int q = 1; q < W; ++q) {
                        m0 = fmin(m0, f[q] + hd0[q]);
                        m1 = fmin(m1, (f[q] + cur.l[u]) + hd1[q]);
                    }
                    const T M = m1 - m0;
                    const T lu = UPD ? (cur.l[u] - omega * M) + cur.a[u] : cur.l[u];
                    mrow[(size_t)h * kLanes] = M;
                    if (UPD) {
                        lrow[(size_t)h * kLanes] = lu;
                        lbacc += (double)fmin(M, T(0));
                    }
                    T fn[W];
#pragma unroll
                    for (int t = 0; t < W; ++t) fn[t] = INF;
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t lo = cur.wd[u][q] & 0xFFFFu, hi = cur.wd[u][q] >> 16;
                        const T v1 = f[q] + lu;
#pragma unroll
                        for (int t = 0; t < W; ++t) fn[t] = fmin(fn[t], arc_to<SH>(lo, hi, (uint32_t)t, f[q], v1));
                    }
#pragma unroll
                    for (int t = 0; t < W; ++t) f[t] = fn[t];
                }
            }
            cur = nxt;
        }
        energy = f[0];
    } else {
        // first pass, ascending: store SP(root, v) of every layer
        T f[W];
#pragma unroll
        for (int q = 0; q < W; ++q) f[q] = q == 0 ? T(0) : INF;
        Chunk cur, nxt;
        load_first(0, cur);
        for (int c = 0; c < nchunk; ++c) {
            if (c + 1 < nchunk) load_first(c + 1, nxt);
            T x[kChunk];
            if (UPD) partner_loads(c, cur, x);
            const int c0 = c * kChunk;
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int h = c0 + u;
                if (h < K) {
#pragma unroll
                    for (int q = 0; q < W; ++q) sp[(size_t)(2 * h + q) * kLanes] = f[q];
                    if (h + 1 < K) {
                        T fn[W];
#pragma unroll
                        for (int t = 0; t < W; ++t) fn[t] = INF;
#pragma unroll
                        for (int q = 0; q < W; ++q) {
                            const uint32_t lo = cur.wd[u][q] & 0xFFFFu, hi = cur.wd[u][q] >> 16;
                            const T v0 = f[q], v1 = f[q] + cur.l[u];
#pragma unroll
                            for (int t = 0; t < W; ++t) fn[t] = fmin(fn[t], arc_to<SH>(lo, hi, (uint32_t)t, v0, v1));
                        }
#pragma unroll
                        for (int t = 0; t < W; ++t) f[t] = fn[t];
                    }
                }
            }
            if (UPD) store_terms(c, cur, x);
            cur = nxt;
        }
        // update pass, descending
        T bn[W];
#pragma unroll
        for (int q = 0; q < W; ++q) bn[q] = q == 0 ? T(0) : INF;   // terminal layer
        load_second(nchunk - 1, cur);
        for (int c = nchunk - 1; c >= 0; --c) {
            if (c > 0) load_second(c - 1, nxt);
            const int c0 = c * kChunk;
#pragma unroll
            for (int u = kChunk - 1; u >= 0; --u) {
                const int h = c0 + u;
                if (h < K) {
                    T v0[W], v1[W];
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t lo = cur.wd[u][q] & 0xFFFFu, hi = cur.wd[u][q] >> 16;
                        v0[q] = head_at<SH, W>(lo, bn);
                        v1[q] = head_at<SH, W>(hi, bn);
                    }
                    T m0 = cur.d[u][0] + v0[0];
                    T m1 = (cur.d[u][0] + cur.l[u]) + v1[0];
#pragma unroll
                    for (int q = 1; q < W; ++q) {
                        m0 = fmin(m0, cur.d[u][q] + v0[q]);
                        m1 = fmin(m1, (cur.d[u][q] + cur.l[u]) + v1[q]);
                    }
                    const T M = m1 - m0;
                    const T lu = UPD ? (cur.l[u] - omega * M) + cur.a[u] : cur.l[u];
                    mrow[(size_t)h * kLanes] = M;
                    if (UPD) {
                        lrow[(size_t)h * kLanes] = lu;
                        lbacc += (double)fmin(M, T(0));
                    }
#pragma unroll
                    for (int q = 0; q < W; ++q) bn[q] = fmin(v0[q], v1[q] + lu);
                }
            }
            cur = nxt;
        }
        energy = bn[0];
    }
    if (UPD && tile_lb) {
        const double e = wave_sum<T>((double)energy + (double)omega * lbacc);
        if (lane == 0) tile_lb[tile] = e;
    }
}

inline unsigned grid8(int64_t tiles, int per_block)
{
    return (unsigned)((((tiles + per_block - 1) / per_block) + 7) & ~int64_t(7));
}

// waves per block of a register-kernel launch: small launches (a few tiles per
// compute unit, latency-bound) spread one wave per block over more compute
// units; large ones keep kRegWaves
inline int reg_waves(int64_t tiles) { return tiles <= 4096 ? 1 : kRegWaves; }

template <typename T, int DIR, int W, bool UPD, int KI>
void launch_class(const DevProblem &p, int wi, T *lam, T *mm, double *tile_lb, Omega<T> w, hipStream_t st)
{
    if constexpr (fast_class_ok(W == 2 ? 0 : 1, KI)) {
        const int l = fast_list(wi, KI);
        const int64_t n = p.list_off[l + 1] - p.list_off[l];
        if (n > 0)
            hipLaunchKernelGGL((k_sweep_reg<T, DIR, W, kKClass[KI], UPD, true, false>), dim3(grid8(n, reg_waves(n))),
                               dim3(reg_waves(n) * kLanes), (UPD ? reg_waves(n) * sweep_lds_bytes<T, kKClass[KI]>() : 0),
                               st, p, lam, mm, tile_lb, w, p.lists + p.list_off[l], n, p.list_first[l]);
    }
    if constexpr (W == 2 && mix_class_ok(KI)) {
        const int l = mix_list(KI);
        const int64_t n = p.list_off[l + 1] - p.list_off[l];
        if (n > 0) {
            const size_t lds = UPD ? reg_waves(n) * sweep_lds_bytes<T, kKClass[KI]>() : 0;
            constexpr bool can_fuse = UPD && fuse_class_ok(sizeof(T), kKClass[KI]);
            if (can_fuse && p.gmeta)
                hipLaunchKernelGGL((k_sweep_reg<T, DIR, W, kKClass[KI], UPD, false, can_fuse>),
                                   dim3(grid8(n, reg_waves(n))), dim3(reg_waves(n) * kLanes), lds, st, p, lam, mm,
                                   tile_lb, w, p.lists + p.list_off[l], n, p.list_first[l]);
            else
                hipLaunchKernelGGL((k_sweep_reg<T, DIR, W, kKClass[KI], UPD, false, false>),
                                   dim3(grid8(n, reg_waves(n))), dim3(reg_waves(n) * kLanes), lds, st, p, lam, mm,
                                   tile_lb, w, p.lists + p.list_off[l], n, p.list_first[l]);
        }
    }
}

template <typename T, int DIR, int W, bool UPD, int... KI>
void launch_classes(const DevProblem &p, int wi, T *lam, T *mm, double *tile_lb, Omega<T> w, hipStream_t st,
                    std::integer_sequence<int, KI...>)
{
    (launch_class<T, DIR, W, UPD, KI>(p, wi, lam, mm, tile_lb, w, st), ...);
}

}  // namespace

template <typename T, int DIR, int W, bool UPD>
void launch_reg(const DevProblem &p, int wi, T *lam, T *mm, double *tile_lb, Omega<T> w, hipStream_t st)
{
    launch_classes<T, DIR, W, UPD>(p, wi, lam, mm, tile_lb, w, st, std::make_integer_sequence<int, kNumKClasses>{});
    if constexpr (W == 2) {
        for (int l : {(int)LIST_LONG_SH, (int)LIST_LONG_MIX}) {
            const int64_t n = p.list_off[l + 1] - p.list_off[l];
            if (n == 0) continue;
            if (l == LIST_LONG_SH)
                hipLaunchKernelGGL((k_sweep_long<T, DIR, UPD, true>), dim3(grid8(n, reg_waves(n))),
                                   dim3(reg_waves(n) * kLanes), 0, st, p, lam, mm, tile_lb, w, p.lists + p.list_off[l], n);
            else
                hipLaunchKernelGGL((k_sweep_long<T, DIR, UPD, false>), dim3(grid8(n, reg_waves(n))),
                                   dim3(reg_waves(n) * kLanes), 0, st, p, lam, mm, tile_lb, w, p.lists + p.list_off[l], n);
        }
    }
}

template void launch_reg<BDDMMA_REG_T, BDDMMA_REG_DIR, 2, BDDMMA_REG_UPD>(const DevProblem &, int, BDDMMA_REG_T *,
                                                                          BDDMMA_REG_T *, double *,
                                                                          Omega<BDDMMA_REG_T>, hipStream_t);
template void launch_reg<BDDMMA_REG_T, BDDMMA_REG_DIR, 4, BDDMMA_REG_UPD>(const DevProblem &, int, BDDMMA_REG_T *,
                                                                          BDDMMA_REG_T *, double *,
                                                                          Omega<BDDMMA_REG_T>, hipStream_t);

}  // namespace bddmma
