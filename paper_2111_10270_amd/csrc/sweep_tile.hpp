// Register-resident sweep of one tile of the fast path (shared by the
// per-sweep kernels of sweep_reg.hip and the persistent kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace bddmma {

namespace {

// ---------------------------------------------------------------------------
// Register-resident sweep for tiles of the fast path (64 BDDs of one topology
// if SH, else of any topologies; fixed layer stride W, exactly KMAX layers).  The layer loops are unrolled,
// so every per-lane array below lives in VGPRs: the multipliers and averaged terms of all layers and the opposite
// direction's distances.  With SH the node words are uniform across the wave
// and live in SGPRs, and each arc test becomes a scalar penalty (see pen);
// otherwise each lane holds its own words in VGPRs and selects per lane.  All loads are
// issued before the first use.  The arithmetic is the same as in k_sweep
// (same operations, same order).
// ---------------------------------------------------------------------------
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
// head (after the last layer, nx is the terminal layer {0, inf, ...})
template <int W, typename T>
__device__ __forceinline__ T head_inner(uint32_t head, const T (&nx)[W])
{
    T r = nx[0] + pen<T>(head, 0);
#pragma unroll
    for (int t = 1; t < W; ++t) r = fmin(r, nx[t] + pen<T>(head, (uint32_t)t));
    return r;
}

// Per-lane topologies (mixed tiles): the value at the arc's head is selected
// per lane; the same values as the penalty form up to the sign of a zero.
template <int W, typename T>
__device__ __forceinline__ T head_lane(uint32_t head, const T (&nx)[W])
{
    T r = inf_of<T>();
#pragma unroll
    for (int t = 0; t < W; ++t) r = head == (uint32_t)t ? nx[t] : r;
    return r;
}

// value an arc pair of one node contributes to next-layer node t: v0 along
// the 0-arc lo, v1 along the 1-arc hi
template <bool SH, typename T>
__device__ __forceinline__ T arc_to(uint32_t lo, uint32_t hi, uint32_t t, T v0, T v1)
{
    if constexpr (SH) return fmin(v0 + pen<T>(lo, t), v1 + pen<T>(hi, t));
    else {
        const T INF = inf_of<T>();
        return fmin(lo == t ? v0 : INF, hi == t ? v1 : INF);
    }
}

template <bool SH, int W, typename T>
__device__ __forceinline__ T head_at(uint32_t head, const T (&nx)[W])
{
    if constexpr (SH) return head_inner<W>(head, nx);
    else return head_lane<W>(head, nx);
}

// The update pass derives its arc tests anew in deep classes.  Kept from
// the first pass, the tests of every layer do not fit in SGPRs and spill to
// VGPR lanes, whose v_writelane / v_readlane pairs and wait states cost more
// than the tests: in mixed tiles the per-lane compare masks from 6 layers
// on, in tiles of one topology the 2 W^2 scalar penalties per layer (of
// sizeof(T) / 4 SGPRs each) once they reach about 96 SGPRs.  Shallower
// classes keep them.  The empty asm only makes the node words opaque to
// the compiler; it emits no instruction.
template <typename T, bool SH, int KMAX, int W>
__device__ __forceinline__ void fresh_arcs(uint32_t (&wd)[KMAX][W])
{
    if constexpr (SH ? KMAX * 2 * W * W * (int)sizeof(T) / 4 >= 96 : KMAX >= 6) {
#pragma unroll
        for (int h = 0; h < KMAX; ++h)
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if constexpr (SH) asm volatile("" : "+s"(wd[h][q]));
                else asm volatile("" : "+v"(wd[h][q]));
            }
    }
}

// UPD = false: min-marginal differences at fixed multipliers (Alg. 2),
// written to mm, which is then output only.  With UPD the slots averaged by
// the averaging kernel hold their averaged term in mm on entry (stored there
// just before this sweep); every other slot holds its previous M.  With fused
// averaging (mixed tiles flagged TILE_GATHER) the slots of such variables
// instead sum their variable's previous differences from the per-variable
// copy (layout.hpp) and write their new one into the other copy.
// LDS of one wave of an updating register sweep: its tile's previous
// differences, K x 64 values
template <typename T, int KMAX>
constexpr size_t sweep_lds_bytes() { return (size_t)KMAX * kLanes * sizeof(T); }

// LDS written by the lanes of one wave, then read by other lanes of it
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sh: this wave's LDS (sweep_lds_bytes), used with UPD only.  GAT: compiled
// with the fused averaging (updating sweeps of mixed tiles of the classes
// fuse_class_ok admits); the tiles flagged TILE_GATHER then use it.
template <typename T, int DIR, int W, int KMAX, bool UPD, bool SH, bool GAT = false>
__device__ __forceinline__ void sweep_tile(const DevProblem &P, T *__restrict__ lam, T *__restrict__ mm,
                                           double *__restrict__ tile_lb, const Omega<T> &w, int64_t tile,
                                           T *__restrict__ sh)
{
    const T omega = w.w1;
    const int lane = threadIdx.x & (kLanes - 1);
    const TileView tv = load_tile(P.tiles + tile);
    static_assert(!GAT || (UPD && !SH && fuse_class_ok(sizeof(T), KMAX)), "fused averaging: mixed updating sweeps");
    constexpr int K = KMAX;   // fast tiles have exactly their class's layer count
    const T INF = inf_of<T>();
    // 64-bit bases: every per-layer access below is base + constant offset
    T *const lrow = lam + tv.pb + lane;
    T *const mrow = mm + tv.pb + lane;
    const uint16_t *const crow = P.code + tv.cb + lane;
    // node words: one copy per tile (SH) or one per lane at stride 64
    const uint32_t *const wrow = P.child + tv.fb + (SH ? 0 : lane);
    // fused averaging: per-variable copies read (this direction) and written
    // (the next one); wave-uniform
    bool gat = false;
    const uint32_t *grow = nullptr;
    const T *gcur = nullptr;
    T *gnxt = nullptr;
    if constexpr (GAT) {
        gat = P.gmeta != nullptr && (uni(P.tiles[tile].flags) & TILE_GATHER) != 0;
        grow = P.gmeta + tv.pb + lane;
        gcur = static_cast<const T *>(P.gbuf) + (DIR == 0 ? 0 : P.n_g);
        gnxt = static_cast<T *>(P.gbuf) + (DIR == 0 ? P.n_g : 0);
    }

    // prologue: every load is issued before the first use
    T l[KMAX], a[KMAX], mo[KMAX];
    uint32_t cd[KMAX], gm[KMAX];
    uint32_t wd[KMAX][W];
#pragma unroll
    for (int h = 0; h < KMAX; ++h) {
        l[h] = T(0);
        a[h] = T(0);
        mo[h] = T(0);
        cd[h] = kCodeSelf;
        gm[h] = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) wd[h][q] = kBot | (kBot << 16);
    }
#pragma unroll
    for (int h = 0; h < KMAX; ++h) {
        if (h < K) {
            l[h] = lrow[h * kLanes];
            if (UPD) {
                mo[h] = mrow[h * kLanes];
                cd[h] = crow[h * kLanes];
            }
            if constexpr (GAT)
                if (gat) gm[h] = grow[h * kLanes];
#pragma unroll
            for (int q = 0; q < W; ++q)
                wd[h][q] = SH ? uni(wrow[h * W + q]) : wrow[(h * W + q) * kLanes];
        }
    }
    if (UPD) {
        // a = c * (M + x) without a branch: an in-tile partner gives c = w2,
        // x = M_partner; a variable of this BDD only gives c = w2, x = M
        // (w2 * 2M = w1 * M exactly, w2 = w1 / 2); a slot averaged by the
        // averaging kernel holds its term t in mm and gives c = 1/2, x = t (t
        // exactly).  The partners' M come from the tile's copy in LDS, not
        // from a second, dependent trip to memory.
#pragma unroll
        for (int h = 0; h < KMAX; ++h)
            if (h < K) sh[h * kLanes + lane] = mo[h];
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < KMAX; ++h) {
            if (h < K) {
                const T x = cd[h] < kCodeSelf ? sh[cd[h]] : mo[h];
                const T c = cd[h] == kCodeGlobal ? T(0.5) : w.w2;
                a[h] = c * (mo[h] + x);
            }
        }
        if constexpr (GAT) {
            if (gat) {
                // a = (omega/|J_i|) * (sum over the variable's slots, ascending
                // rows), the operations of the averaging kernel.  The slot's
                // own entry equals its M-bar (mo); the at most kGatherOthers
                // other entries of its variable's block are loaded for all
                // layers at once, so they share one trip to memory (lanes that
                // need no entry read entry 0, which all share).  Entries past
                // a block add +0, which leaves a sum that cannot be -0
                // unchanged.
                constexpr int LC = sizeof(T) == 8 && KMAX > 16 ? 8 : KMAX;
#pragma unroll
                for (int h0 = 0; h0 < KMAX; h0 += LC) {
                    T v[LC][kGatherOthers];
#pragma unroll
                    for (int u = 0; u < LC; ++u) {
                        const int h = h0 + u;
                        const uint32_t g = h < KMAX ? gm[h] : 0u;
                        const uint32_t deg = (g >> 28) + 1u, rank = (g >> 24) & 0xFu;
                        const uint32_t base = (g & 0xFFFFFFu) - rank;
                        const bool glob = h < K && cd[h] == kCodeGlobal;
#pragma unroll
                        for (uint32_t j = 0; j < kGatherOthers; ++j) {
                            const uint32_t k = j + (j >= rank ? 1u : 0u);   // j-th entry other than its own
                            v[u][j] = gcur[glob && k < deg ? base + k : 0u];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < LC; ++u) {
                        const int h = h0 + u;
                        if (h < K && cd[h] == kCodeGlobal) {
                            const uint32_t deg = (gm[h] >> 28) + 1u, rank = (gm[h] >> 24) & 0xFu;
                            T sum = T(0);
#pragma unroll
                            for (int k = 0; k <= kGatherOthers; ++k) {
                                // entry k: its own value, or the other entry j = k (below
                                // the own rank) or j = k - 1 (above it)
                                const T lo = k < kGatherOthers ? v[u][k < kGatherOthers ? k : 0] : T(0);
                                const T hi = k >= 1 ? v[u][k >= 1 ? k - 1 : 0] : T(0);
                                const uint32_t ku = (uint32_t)k;
                                sum += ku == rank ? mo[h] : ku >= deg ? T(0) : ku < rank ? lo : hi;
                            }
                            a[h] = (T)(w.w64 / (double)deg) * sum;
                        }
                    }
                }
            }
        }
    }

    double lbacc = 0.0;
    T energy;
    if (DIR == 0) {
        // SP(v, top) of every layer under the current multipliers; keep the
        // values at the heads of every arc for the update pass
        T hd0[KMAX][W], hd1[KMAX][W];
        T nx[W];
#pragma unroll
        for (int q = 0; q < W; ++q) nx[q] = q == 0 ? T(0) : INF;   // terminal layer
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
                    const T v0 = head_at<SH, W>(lo, nx);
                    const T v1 = head_at<SH, W>(hi, nx);
                    hd0[h][q] = v0;
                    hd1[h][q] = v1;
                    b[q] = fmin(v0, v1 + l[h]);
                }
#pragma unroll
                for (int q = 0; q < W; ++q) nx[q] = b[q];
            }
        }
        // forward sweep with updates
        fresh_arcs<T, SH>(wd);
        T f[W];
#pragma unroll
        for (int q = 0; q < W; ++q) f[q] = q == 0 ? T(0) : INF;
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
                const T lu = UPD ? (l[h] - omega * M) + a[h] : l[h];
                mrow[h * kLanes] = M;
                if (UPD) {
                    lrow[h * kLanes] = lu;
                    lbacc += (double)fmin(M, T(0));
                }
                if constexpr (GAT)
                    if (gat && cd[h] == kCodeGlobal) gnxt[gm[h] & 0xFFFFFFu] = M;
                T fn[W];
#pragma unroll
                for (int t = 0; t < W; ++t) fn[t] = INF;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    const T v1 = f[q] + lu;
#pragma unroll
                    for (int t = 0; t < W; ++t) fn[t] = fmin(fn[t], arc_to<SH>(lo, hi, (uint32_t)t, f[q], v1));
                }
#pragma unroll
                for (int t = 0; t < W; ++t) f[t] = fn[t];
            }
        }
        energy = f[0];   // node 0 of the terminal layer: accept
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
                    for (int t = 0; t < W; ++t) fw[h + 1][t] = fmin(fw[h + 1][t], arc_to<SH>(lo, hi, (uint32_t)t, v0, v1));
                }
            }
        }
        // backward sweep with updates
        fresh_arcs<T, SH>(wd);
        T bn[W];
#pragma unroll
        for (int q = 0; q < W; ++q) bn[q] = q == 0 ? T(0) : INF;   // terminal layer
#pragma unroll
        for (int h = KMAX - 1; h >= 0; --h) {
            if (h < K) {
                T v0[W], v1[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t lo = wd[h][q] & 0xFFFFu, hi = wd[h][q] >> 16;
                    v0[q] = head_at<SH, W>(lo, bn);
                    v1[q] = head_at<SH, W>(hi, bn);
                }
                T m0 = fw[h][0] + v0[0];
                T m1 = (fw[h][0] + l[h]) + v1[0];
#pragma unroll
                for (int q = 1; q < W; ++q) {
                    m0 = fmin(m0, fw[h][q] + v0[q]);
                    m1 = fmin(m1, (fw[h][q] + l[h]) + v1[q]);
                }
                const T M = m1 - m0;
                const T lu = UPD ? (l[h] - omega * M) + a[h] : l[h];
                mrow[h * kLanes] = M;
                if (UPD) {
                    lrow[h * kLanes] = lu;
                    lbacc += (double)fmin(M, T(0));
                }
                if constexpr (GAT)
                    if (gat && cd[h] == kCodeGlobal) gnxt[gm[h] & 0xFFFFFFu] = M;
#pragma unroll
                for (int q = 0; q < W; ++q) bn[q] = fmin(v0[q], v1[q] + lu);
            }
        }
        energy = bn[0];
    }
    if (UPD && tile_lb) {
        const double e = wave_sum<T>((double)energy + (double)omega * lbacc);
        if (lane == 0) tile_lb[tile] = e;
    }
}

}  // namespace

}  // namespace bddmma
