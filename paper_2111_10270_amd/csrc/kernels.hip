// HIP kernels of the solver, written for CDNA4 (gfx950, 64-wide wavefronts).
//
// Hot path (Alg. 1): every wavefront owns one tile of 64 whole BDDs, one BDD
// per lane, and runs the whole layer loop of a sweep inside the kernel.  The
// shortest-path distances the min-marginal formula needs (Sec. 5, min-marginal
// via shortest paths: SP(r, v) and SP(s(v), top)) are recomputed at the start
// of each sweep from the current multipliers and kept in LDS (lane-minor, so
// every LDS access is bank-conflict free); they never travel through HBM.  HBM
// traffic per sweep is one coalesced read of the multipliers and the pair ->
// variable map, one gather of the averaged term, and coalesced writes of the
// updated multipliers and min-marginal differences.  No MFMA: the work is
// min-plus arithmetic on sparse, data-dependent graphs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace bddmma {

namespace {

// ---------------------------------------------------------------------------
// The sweep.  DIR 0: ascending variables (Alg. 3), DIR 1: descending (Alg. 4).
// MODE_UPDATE: at every layer compute M = m^1 - m^0 and apply the deferred
// parallel update  lambda <- (lambda - omega M) + a_i  before the distances of
// the next layer are propagated with the new multiplier (Alg. 1).
// MODE_FIXED: same min-marginals at fixed multipliers.
// ---------------------------------------------------------------------------
template <typename T, int DIR, int MODE, bool LDS>
__global__ __launch_bounds__(kThreads) void k_sweep(DevProblem P, T *__restrict__ lam, T *mm,
                                                     double *__restrict__ tile_lb, Omega<T> w,
                                                     const int32_t *__restrict__ list, int64_t tile_count)
{
    const T omega = w.w1;
    T *const mm_out = mm;   // read for the in-tile averaging before this sweep overwrites it
    extern __shared__ unsigned char smem_raw[];
    const int lane = threadIdx.x & (kLanes - 1);
    const uint32_t wave = uni(threadIdx.x >> 6);
    const int64_t lt = xcd_block() * kWavesPerBlock + wave;
    if (lt >= tile_count) return;
    const int64_t tile = (int64_t)uni((uint32_t)list[lt]);
    const TileView tv = load_tile(P.tiles + tile);
    const uint32_t *__restrict__ child = P.child;
    const uint32_t *__restrict__ layers = P.layers + tv.lb;

    T *base;
    if (LDS)
        base = reinterpret_cast<T *>(smem_raw) + (size_t)wave * kLanes * P.lds_lane_elems + lane;
    else
        base = reinterpret_cast<T *>(P.scratch) + (size_t)P.tiles[tile].scratch_base + lane;
    T *lamS = base;                               // [K]  multipliers of this lane's BDD
    T *avS = lamS + (size_t)tv.K * kLanes;         // [K]  averaged terms a_i
    T *F = avS + (size_t)tv.K * kLanes;            // [NN] SP(root, v)
    T *Bk = F + (size_t)tv.NN * kLanes;            // [NN] SP(v, top)
    const T INF = inf_of<T>();

    // stage multipliers (and averaged terms) of all layers: all loads of a
    // chunk are issued before the first one is used
    for (uint32_t h0 = 0; h0 < tv.K; h0 += kPrefetch) {
        T lv[kPrefetch], mv[kPrefetch];
        uint32_t cv[kPrefetch];
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u) {
            const uint32_t h = h0 + u;
            if (h < tv.K) {
                const uint32_t s = tv.pb + h * kLanes + lane;
                lv[u] = lam[s];
                if (MODE == MODE_UPDATE) {
                    mv[u] = mm[s];
                    cv[u] = P.code[tv.cb + h * kLanes + lane];
                }
            }
        }
        if (MODE == MODE_UPDATE) {
            T av[kPrefetch];
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u)
                if (h0 + u < tv.K)
                    av[u] = averaged_term(mm, tv.pb, cv[u], mv[u], w);
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u)
                if (h0 + u < tv.K) avS[(size_t)(h0 + u) * kLanes] = av[u];
        }
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u)
            if (h0 + u < tv.K) lamS[(size_t)(h0 + u) * kLanes] = lv[u];
    }

    double lbacc = 0.0;   // sum over layers of min(M, 0)
    T energy;

    if (DIR == 0) {
        // SP(v, top) under the current multipliers (Alg. 4 without updates)
        for (int h = (int)tv.K - 1; h >= 0; --h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            const T l = lamS[(size_t)h * kLanes];
            for (uint32_t q = 0; q < W; ++q) {
                const uint32_t c = node_word(child, tv, noff + q, lane);
                const T b0 = head_val(c & 0xFFFFu, Bk, noffn);
                const T b1 = head_val(c >> 16, Bk, noffn) + l;
                Bk[(size_t)(noff + q) * kLanes] = tmin(b0, b1);
            }
        }
        // forward sweep with updates (Alg. 3 + the update of Alg. 1)
        F[0] = T(0);
        T top = INF;
        for (uint32_t h = 0; h < tv.K; ++h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            const uint32_t Wn = (h + 1 < tv.K) ? (uni(layers[h + 1]) >> 16) : 0u;
            const T l = lamS[(size_t)h * kLanes];
            T m0 = INF, m1 = INF;
            for (uint32_t q = 0; q < W; ++q) {
                const T f = F[(size_t)(noff + q) * kLanes];
                const uint32_t c = node_word(child, tv, noff + q, lane);
                const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                if (lo != kBot) m0 = tmin(m0, f + head_val(lo, Bk, noffn));
                if (hi != kBot) m1 = tmin(m1, (f + l) + head_val(hi, Bk, noffn));
            }
            const T M = m1 - m0;
            const uint32_t s = tv.pb + h * kLanes + lane;
            mm_out[s] = M;
            T lu = l;
            if (MODE == MODE_UPDATE) {
                lu = (l - omega * M) + avS[(size_t)h * kLanes];
                lam[s] = lu;
                lbacc += (double)(M < T(0) ? M : T(0));
            }
            for (uint32_t q = 0; q < Wn; ++q) F[(size_t)(noffn + q) * kLanes] = INF;
            for (uint32_t q = 0; q < W; ++q) {
                const T f = F[(size_t)(noff + q) * kLanes];
                const uint32_t c = node_word(child, tv, noff + q, lane);
                const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                if (lo != kBot) {
                    if (lo == kTop) top = tmin(top, f);
                    else {
                        T &d = F[(size_t)(noffn + lo) * kLanes];
                        d = tmin(d, f);
                    }
                }
                if (hi != kBot) {
                    const T v = f + lu;
                    if (hi == kTop) top = tmin(top, v);
                    else {
                        T &d = F[(size_t)(noffn + hi) * kLanes];
                        d = tmin(d, v);
                    }
                }
            }
        }
        energy = top;
    } else {
        // SP(root, v) under the current multipliers (Alg. 3 without updates)
        F[0] = T(0);
        for (uint32_t h = 0; h + 1 < tv.K; ++h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            const uint32_t Wn = uni(layers[h + 1]) >> 16;
            const T l = lamS[(size_t)h * kLanes];
            for (uint32_t q = 0; q < Wn; ++q) F[(size_t)(noffn + q) * kLanes] = INF;
            for (uint32_t q = 0; q < W; ++q) {
                const T f = F[(size_t)(noff + q) * kLanes];
                const uint32_t c = node_word(child, tv, noff + q, lane);
                const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                if (lo < kTop) {
                    T &d = F[(size_t)(noffn + lo) * kLanes];
                    d = tmin(d, f);
                }
                if (hi < kTop) {
                    T &d = F[(size_t)(noffn + hi) * kLanes];
                    d = tmin(d, f + l);
                }
            }
        }
        // backward sweep with updates (Alg. 4 + the update of Alg. 1)
        for (int h = (int)tv.K - 1; h >= 0; --h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            const T l = lamS[(size_t)h * kLanes];
            T m0 = INF, m1 = INF;
            for (uint32_t q = 0; q < W; ++q) {
                const T f = F[(size_t)(noff + q) * kLanes];
                const uint32_t c = node_word(child, tv, noff + q, lane);
                const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                if (lo != kBot) m0 = tmin(m0, f + head_val(lo, Bk, noffn));
                if (hi != kBot) m1 = tmin(m1, (f + l) + head_val(hi, Bk, noffn));
            }
            const T M = m1 - m0;
            const uint32_t s = tv.pb + (uint32_t)h * kLanes + lane;
            mm_out[s] = M;
            T lu = l;
            if (MODE == MODE_UPDATE) {
                lu = (l - omega * M) + avS[(size_t)h * kLanes];
                lam[s] = lu;
                lbacc += (double)(M < T(0) ? M : T(0));
            }
            for (uint32_t q = 0; q < W; ++q) {
                const uint32_t c = node_word(child, tv, noff + q, lane);
                const T b0 = head_val(c & 0xFFFFu, Bk, noffn);
                const T b1 = head_val(c >> 16, Bk, noffn) + lu;
                Bk[(size_t)(noff + q) * kLanes] = tmin(b0, b1);
            }
        }
        energy = Bk[0];
    }
    if (tile_lb) {
        const double e = wave_sum<T>((double)energy + (double)omega * lbacc);
        if (lane == 0) tile_lb[tile] = e;
    }
}


// ---------------------------------------------------------------------------
// Wide tiles: one BDD per single-wave block, the lanes spread over the nodes
// of a layer (the paper's node-parallel scheme, inside one wave).  Same
// arithmetic as k_sweep: distances to top by a gather over each node's two
// arcs, distances from the root by a scatter with an LDS minimum (min is
// order free, so the result does not depend on the order of the updates),
// min-marginals as wave minima over the layer's nodes.  Multipliers and
// averaged terms of the BDD are staged in LDS first; only lane 0 writes the
// BDD's lambda and M.  The BDDs of one tile run in different blocks, so the
// packer gives wide tiles no in-tile averaging partners (only the BDD's own
// slot or the averaging kernel's term are read).  Blocks of dummy lanes (padding BDDs) return at once:
// a padding BDD keeps lambda = 0 and M = 0.
// ---------------------------------------------------------------------------
// *p = min(*p, v) in LDS with the native float / double min (ds_min_f32,
// ds_min_f64): exact, so the result does not depend on the order of the lanes
template <typename T>
__device__ __forceinline__ void lds_min(T *p, T v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// min over the LPB lanes of a group (aligned groups of LPB lanes of one wave)
template <int LPB, typename T>
__device__ __forceinline__ T group_min(T v)
{
    for (int off = LPB / 2; off > 0; off >>= 1) v = tmin(v, (T)__shfl_xor(v, off, kLanes));
    return v;
}

// One BDD per group of LPB lanes; a single-wave block holds G = 64 / LPB BDDs
// of one tile, which share the tile's layer structure, so every group runs
// the same loops and the block's barriers stay uniform.  Each group has its
// own LDS region of region_bytes.  Padding BDDs take part in the barriers
// only.
template <typename T, int DIR, bool UPD, int LPB>
__global__ __launch_bounds__(kLanes) void k_sweep_wide(DevProblem P, T *__restrict__ lam, T *mm,
                                                        Omega<T> w, const int32_t *__restrict__ list,
                                                        int64_t count, uint32_t region_bytes)
{
    constexpr int G = kLanes / LPB;
    extern __shared__ unsigned char smem_raw[];
    const int t = (int)threadIdx.x % LPB;                // lane in the group
    const int g = (int)threadIdx.x / LPB;                // group = BDD of the block
    const int64_t wt = (int64_t)blockIdx.x / LPB;        // index in the wide list (LPB blocks per tile)
    const int j = (int)(blockIdx.x % LPB) * G + g;       // lane (BDD) of the tile
    if (wt >= count) return;                             // uniform over the block
    const int64_t tile = (int64_t)uni((uint32_t)list[wt]);
    const TileView tv = load_tile(P.tiles + tile);
    double *const part = P.wide_part + wt * kLanes + j;
    const bool live = P.pair_var[tv.pb + j] < P.n_vars;  // false: padding BDD
    const T omega = w.w1;
    const int K = (int)tv.K, NN = (int)tv.NN;
    const T INF = inf_of<T>();
    const uint32_t *__restrict__ layers = P.layers + tv.lb;
    const uint32_t *__restrict__ words = tv.shared ? P.child + tv.nb : P.child + tv.fb + (size_t)j * NN;
    unsigned char *const region = smem_raw + (size_t)g * region_bytes;
    T *const F = reinterpret_cast<T *>(region);         // [NN] SP(root, v)
    T *const Bk = F + NN;                                // [NN] SP(v, top)
    T *const lamS = Bk + NN;                             // [K]
    T *const avS = lamS + K;                             // [K]
    uint32_t *const Wd = reinterpret_cast<uint32_t *>(avS + K);   // [NN] node words
    auto head = [&](uint32_t c, uint32_t noffn) -> T {
        return c == kTop ? T(0) : (c == kBot ? INF : Bk[noffn + c]);
    };

    // the BDD's node words are staged in LDS once, so no layer waits on a
    // global load
    if (live) {
        for (int n = t; n < NN; n += LPB) Wd[n] = words[n];
        for (int h = t; h < K; h += LPB) {
            const uint32_t s = tv.pb + (uint32_t)h * kLanes + j;
            lamS[h] = lam[s];
            if (UPD) {
                const uint32_t cd = P.code[tv.cb + (uint32_t)h * kLanes + j];
                avS[h] = averaged_term(mm, tv.pb, cd, mm[s], w);
            }
        }
    }
    __syncthreads();

    double lbacc = 0.0;   // lane 0 of the group only
    T energy = INF;
    if (DIR == 0) {
        // SP(v, top) under the current multipliers
        for (int h = K - 1; h >= 0; --h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            if (live) {
                const T l = lamS[h];
                for (uint32_t q = t; q < W; q += LPB) {
                    const uint32_t c = Wd[noff + q];
                    Bk[noff + q] = tmin(head(c & 0xFFFFu, noffn), head(c >> 16, noffn) + l);
                }
            }
            __syncthreads();
        }
        if (live && t == 0) F[0] = T(0);
        __syncthreads();
        T top = INF;
        for (int h = 0; h < K; ++h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            const uint32_t Wn = h + 1 < K ? (uni(layers[h + 1]) >> 16) : 0u;
            T lu = T(0);
            if (live) {
                const T l = lamS[h];
                T m0 = INF, m1 = INF;
                for (uint32_t q = t; q < W; q += LPB) {
                    const T f = F[noff + q];
                    const uint32_t c = Wd[noff + q];
                    const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                    if (lo != kBot) m0 = tmin(m0, f + head(lo, noffn));
                    if (hi != kBot) m1 = tmin(m1, (f + l) + head(hi, noffn));
                }
                m0 = group_min<LPB>(m0);
                m1 = group_min<LPB>(m1);
                const T M = m1 - m0;
                lu = UPD ? (l - omega * M) + avS[h] : l;
                if (t == 0) {
                    const uint32_t s = tv.pb + (uint32_t)h * kLanes + j;
                    mm[s] = M;
                    if (UPD) {
                        lam[s] = lu;
                        lbacc += (double)(M < T(0) ? M : T(0));
                    }
                }
                for (uint32_t q = t; q < Wn; q += LPB) F[noffn + q] = INF;
            }
            __syncthreads();
            if (live) {
                for (uint32_t q = t; q < W; q += LPB) {
                    const T f = F[noff + q];
                    const uint32_t c = Wd[noff + q];
                    const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                    if (lo != kBot) {
                        if (lo == kTop) top = tmin(top, f);
                        else lds_min(&F[noffn + lo], f);
                    }
                    if (hi != kBot) {
                        const T v = f + lu;
                        if (hi == kTop) top = tmin(top, v);
                        else lds_min(&F[noffn + hi], v);
                    }
                }
            }
            __syncthreads();
        }
        energy = group_min<LPB>(top);
    } else {
        // SP(root, v) under the current multipliers
        if (live && t == 0) F[0] = T(0);
        __syncthreads();
        for (int h = 0; h + 1 < K; ++h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            const uint32_t Wn = uni(layers[h + 1]) >> 16;
            if (live)
                for (uint32_t q = t; q < Wn; q += LPB) F[noffn + q] = INF;
            __syncthreads();
            if (live) {
                const T l = lamS[h];
                for (uint32_t q = t; q < W; q += LPB) {
                    const T f = F[noff + q];
                    const uint32_t c = Wd[noff + q];
                    const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                    if (lo < kTop) lds_min(&F[noffn + lo], f);
                    if (hi < kTop) lds_min(&F[noffn + hi], f + l);
                }
            }
            __syncthreads();
        }
        // backward sweep with updates
        for (int h = K - 1; h >= 0; --h) {
            const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
            if (live) {
                const T l = lamS[h];
                T m0 = INF, m1 = INF;
                for (uint32_t q = t; q < W; q += LPB) {
                    const T f = F[noff + q];
                    const uint32_t c = Wd[noff + q];
                    const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
                    if (lo != kBot) m0 = tmin(m0, f + head(lo, noffn));
                    if (hi != kBot) m1 = tmin(m1, (f + l) + head(hi, noffn));
                }
                m0 = group_min<LPB>(m0);
                m1 = group_min<LPB>(m1);
                const T M = m1 - m0;
                const T lu = UPD ? (l - omega * M) + avS[h] : l;
                if (t == 0) {
                    const uint32_t s = tv.pb + (uint32_t)h * kLanes + j;
                    mm[s] = M;
                    if (UPD) {
                        lam[s] = lu;
                        lbacc += (double)(M < T(0) ? M : T(0));
                    }
                }
                for (uint32_t q = t; q < W; q += LPB) {
                    const uint32_t c = Wd[noff + q];
                    Bk[noff + q] = tmin(head(c & 0xFFFFu, noffn), head(c >> 16, noffn) + lu);
                }
            }
            __syncthreads();
        }
        energy = Bk[0];
    }
    if (UPD && t == 0) *part = live ? (double)energy + (double)omega * lbacc : 0.0;
}

__global__ __launch_bounds__(kLanes) void k_wide_lb(const double *__restrict__ part,
                                                   const int32_t *__restrict__ list, double *__restrict__ tile_lb)
{
    const double e = wave_sum<float>(part[(int64_t)blockIdx.x * kLanes + threadIdx.x]);
    if (threadIdx.x == 0) tile_lb[list[blockIdx.x]] = e;
}

// E^j(t') of every lane in FP64, summed per tile: t' = lambda + omega M -
// share[i], the terminated multipliers made dual feasible (share[i] = r_i /
// |J_i| from the residual kernel, share[n_vars] = 0 for padding slots)
template <typename T, bool LDS>
__global__ __launch_bounds__(kThreads) void k_cert(DevProblem P, const T *__restrict__ lam,
                                                    const T *__restrict__ mm, double omega,
                                                    const double *__restrict__ share,
                                                    double *__restrict__ tile_e, const int32_t *__restrict__ list,
                                                    int64_t tile_count)
{
    extern __shared__ unsigned char smem_raw[];
    const int lane = threadIdx.x & (kLanes - 1);
    const uint32_t wave = uni(threadIdx.x >> 6);
    const int64_t lt = xcd_block() * kWavesPerBlock + wave;
    if (lt >= tile_count) return;
    const int64_t tile = (int64_t)uni((uint32_t)list[lt]);
    const TileView tv = load_tile(P.tiles + tile);
    const uint32_t *__restrict__ layers = P.layers + tv.lb;
    double *F;
    if (LDS) {
        const size_t per_lane = (size_t)P.lds_lane_elems * sizeof(T) / sizeof(double);
        F = reinterpret_cast<double *>(smem_raw) + (size_t)wave * kLanes * per_lane + lane;
    } else {
        F = reinterpret_cast<double *>(reinterpret_cast<T *>(P.scratch) + (size_t)P.tiles[tile].scratch_base) + lane;
    }
    const double INF = __builtin_huge_val();
    F[0] = 0.0;
    double top = INF;
    for (uint32_t h = 0; h < tv.K; ++h) {
        const uint32_t le = uni(layers[h]), noff = le & 0xFFFFu, W = le >> 16, noffn = noff + W;
        const uint32_t Wn = (h + 1 < tv.K) ? (uni(layers[h + 1]) >> 16) : 0u;
        const uint32_t s = tv.pb + h * kLanes + lane;
        const double cost = ((double)lam[s] + omega * (double)mm[s]) - share[P.pair_var[s]];
        for (uint32_t q = 0; q < Wn; ++q) F[(size_t)(noffn + q) * kLanes] = INF;
        for (uint32_t q = 0; q < W; ++q) {
            const double f = F[(size_t)(noff + q) * kLanes];
            const uint32_t c = node_word(P.child, tv, noff + q, lane);
            const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
            if (lo != kBot) {
                if (lo == kTop) top = tmin(top, f);
                else {
                    double &d = F[(size_t)(noffn + lo) * kLanes];
                    d = tmin(d, f);
                }
            }
            if (hi != kBot) {
                const double v = f + cost;
                if (hi == kTop) top = tmin(top, v);
                else {
                    double &d = F[(size_t)(noffn + hi) * kLanes];
                    d = tmin(d, v);
                }
            }
        }
    }
    const double e = wave_sum<T>(top);
    if (lane == 0) tile_e[tile] = e;
}

// fixed-order two-stage sum: stage 1 writes one partial per block
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

__device__ __forceinline__ double block_max(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_sum_stage1(const double *__restrict__ part, int64_t n,
                                                            double *__restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * per, b = a + per < n ? a + per : n;
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) s += part[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedThreads) void k_sum_stage2(const double *__restrict__ part, int n, double offset,
                                                            double *__restrict__ out)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kRedThreads) s += part[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = t + offset;
}


// a_i = (omega / |J_i|) * sum_{k in J_i} M_ik, summed in ascending row order,
// for the variables the sweep does not average in-tile; the term replaces M_ik
// at every slot of i (each thread owns the slots of its variable).  Blocks are
// assigned to degree buckets (layout.hpp).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_average(AvgBucketSet bs, const int32_t *__restrict__ gslot,
                                                         const int32_t *__restrict__ vptr,
                                                         const int32_t *__restrict__ vslot, T *__restrict__ mm,
                                                         double omega)
{
    // bucket of this block (uniform; the descriptors are kernel arguments)
    int bi = -1;
    for (int j = 0; j < bs.n; ++j)
        if ((int)blockIdx.x >= bs.b[j].block_begin) bi = j;
    if (bi >= 0) {
        const AvgBucket bk = bs.b[bi];
        const int64_t i = (int64_t)((int)blockIdx.x - bk.block_begin) * kRedThreads + threadIdx.x;
        if (i < bk.count) {
            if (bk.deg > 0) {
                // slots of the variable, coalesced across the block, then its M-bar values
                int32_t sl[kEllMaxDeg];
                T mv[kEllMaxDeg];
#pragma unroll
                for (int k = 0; k < kEllMaxDeg; ++k)
                    if (k < bk.deg) sl[k] = gslot[bk.base + (int64_t)k * bk.count + i];
#pragma unroll
                for (int k = 0; k < kEllMaxDeg; ++k)
                    if (k < bk.deg) mv[k] = mm[sl[k]];
                T s = T(0);
#pragma unroll
                for (int k = 0; k < kEllMaxDeg; ++k)
                    if (k < bk.deg) s += mv[k];
                const T av = (T)(omega / (double)bk.deg) * s;
#pragma unroll
                for (int k = 0; k < kEllMaxDeg; ++k)
                    if (k < bk.deg) mm[sl[k]] = av;
            } else {
                const int32_t v = gslot[bk.base + i];
                const int32_t a = vptr[v], b = vptr[v + 1];
                T s = T(0);
                for (int32_t q = a; q < b; ++q) s += mm[vslot[q]];
                const T av = (T)(omega / (double)(b - a)) * s;
                for (int32_t q = a; q < b; ++q) mm[vslot[q]] = av;
            }
        }
    }
}

// Bound of each of the recorded sweeps from its per-tile partials (row r of
// `part`): one block per sweep, fixed summation order, so the value does not
// depend on scheduling.  out[r] = offset + sum.
__global__ __launch_bounds__(kRedThreads) void k_lb_many(const double *__restrict__ part, int64_t n_tiles,
                                                         double offset, double *__restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const double *row = part + (int64_t)blockIdx.x * n_tiles;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t t = threadIdx.x;
    for (; t + 3 * kRedThreads < n_tiles; t += 4 * kRedThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += row[t + u * kRedThreads];
    }
    for (int u = 0; t < n_tiles; t += kRedThreads, ++u) acc[u & 3] += row[t];
    const double tot = block_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), sh);
    if (threadIdx.x == 0) out[blockIdx.x] = tot + offset;
}

// per-variable a_i of every variable (state export)
template <typename T>
__global__ __launch_bounds__(256) void k_average_all(const int32_t *__restrict__ vptr,
                                                     const int32_t *__restrict__ vslot, const T *__restrict__ mm,
                                                     T *__restrict__ avg, double omega, int64_t V)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int32_t a = vptr[v], b = vptr[v + 1];
    if (a == b) {
        avg[v] = T(0);
        return;
    }
    T s = T(0);
    for (int32_t q = a; q < b; ++q) s += mm[vslot[q]];
    avg[v] = (T)(omega / (double)(b - a)) * s;
}

// per-variable copy of the differences for the fused averaging
template <typename T>
__global__ __launch_bounds__(256) void k_gather_refresh(const int32_t *__restrict__ gsrc, const T *__restrict__ mm,
                                                        T *__restrict__ g, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) g[e] = mm[gsrc[e]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_init(DevProblem P, T *__restrict__ lam, T *__restrict__ mm)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.n_slots) return;
    const int32_t v = P.pair_var[s];
    T l = T(0);
    if (v < P.n_vars) {
        const int32_t d = P.vptr[v + 1] - P.vptr[v];
        l = (T)(P.cost[v] / (double)d);   // lambda_i^j = c_i / |J_i|
    }
    lam[s] = l;
    mm[s] = T(0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_terminate(int64_t n, T *__restrict__ lam, const T *__restrict__ mm, T omega)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) lam[s] = lam[s] + omega * mm[s];
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_residual(DevProblem P, const T *__restrict__ lam,
                                                          const T *__restrict__ mm, double omega,
                                                          double *__restrict__ red, double *__restrict__ share)
{
    __shared__ double sh[kRedThreads];
    const int64_t per = (P.n_vars + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * per, b = a + per < P.n_vars ? a + per : P.n_vars;
    double pos = 0.0, mx = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) share[P.n_vars] = 0.0;
    for (int64_t v = a + threadIdx.x; v < b; v += kRedThreads) {
        const int32_t q0 = P.vptr[v], q1 = P.vptr[v + 1];
        if (q0 == q1) continue;
        double s = 0.0;
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t sl = P.vslot[q];
            s += (double)lam[sl] + omega * (double)mm[sl];
        }
        const double r = s - P.cost[v];
        share[v] = r / (double)(q1 - q0);
        if (r > 0.0) pos += r;
        mx = fmax(mx, fabs(r));
    }
    const double tp = block_sum(pos, sh);
    const double tm = block_max(mx, sh);
    if (threadIdx.x == 0) {
        red[2 + blockIdx.x] = tp;
        red[2 + gridDim.x + blockIdx.x] = tm;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_residual_stage2(double *__restrict__ red, int nb)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nb; i += kRedThreads) {
        s += red[2 + i];
        m = fmax(m, red[2 + nb + i]);
    }
    const double ts = block_sum(s, sh);
    const double tm = block_max(m, sh);
    if (threadIdx.x == 0) {
        red[0] = ts;
        red[1] = tm;
    }
}

// Slots and differences of a variable's first kVarBatch subproblems (q0 ..
// q1-1 in ascending row order), loaded together: all slot ids, then all
// values, so a thread waits for two trips to memory instead of two per
// subproblem.  Later subproblems, if any, are read one by one by the caller.
// (The perturbation, which also rewrites the multipliers, gains from it:
// 83 against 94 us on the 256 x 256 grid; the conflict count does not.)
constexpr int kVarBatch = 4;

template <typename T>
__device__ __forceinline__ int var_batch(const DevProblem &P, const T *__restrict__ mm, int32_t q0, int32_t q1,
                                         int32_t (&sl)[kVarBatch], T (&mv)[kVarBatch])
{
    const int n = q1 - q0 < kVarBatch ? q1 - q0 : kVarBatch;
#pragma unroll
    for (int k = 0; k < kVarBatch; ++k)
        if (k < n) sl[k] = P.vslot[q0 + k];
#pragma unroll
    for (int k = 0; k < kVarBatch; ++k)
        if (k < n) mv[k] = mm[sl[k]];
    return n;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_conflicts(DevProblem P, const T *__restrict__ mm, double tau,
                                                           const uint8_t *__restrict__ flag, int32_t *counter)
{
    __shared__ double sh[kRedThreads];
    const int64_t v = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    int c = 0;
    if (v < P.n_vars) {
        const int32_t q0 = P.vptr[v], q1 = P.vptr[v + 1];
        if (P.inst_tau) tau = P.inst_tau[P.var_inst[v]];
        if (q0 != q1) {
            bool pos = true, neg = true;
            for (int32_t q = q0; q < q1; ++q) {
                const double m = (double)mm[P.vslot[q]];
                pos = pos && m > tau;
                neg = neg && m < -tau;
            }
            c = (flag[v] || !(pos || neg)) ? 1 : 0;
        }
    }
    if (P.var_inst) {
        // batch: one count per instance
        if (c) atomicAdd(counter + P.var_inst[v], 1);
        return;
    }
    const double t = block_sum((double)c, sh);
    if (threadIdx.x == 0 && t > 0.0) atomicAdd(counter, (int32_t)t);
}

// SplitMix64 output function (Steele, Lea & Flood 2014) of seed ^ round*K1 ^ i*K2 -> [0, 1)
__device__ __forceinline__ double u01(uint64_t seed, uint64_t round, uint64_t i)
{
    uint64_t z = seed ^ (round * 0xD1B54A32D192ED03ull) ^ (i * 0x8CB92BA72F3D8DD7ull);
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Alg. 2 perturbation: all M > 0 -> +delta, all M < 0 -> -delta, all M = 0 ->
// r*delta, mixed -> sign(sum M)*|r|*delta; flagged variables take r*delta.
// r ~ U[-delta, delta] (scale 0) or U[-1, 1] (scale 1).
template <typename T>
__global__ __launch_bounds__(256) void k_perturb(DevProblem P, T *__restrict__ lam, const T *__restrict__ mm,
                                                 double tau, double delta, uint64_t seed, uint64_t round, int scale,
                                                 const uint8_t *__restrict__ flag)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= P.n_vars) return;
    const int32_t q0 = P.vptr[v], q1 = P.vptr[v + 1];
    if (q0 == q1) return;
    // the draw depends on the variable's index inside its instance only
    const uint64_t li = P.var_inst ? (uint64_t)(v - P.inst_var[P.var_inst[v]]) : (uint64_t)v;
    if (P.inst_tau) tau = P.inst_tau[P.var_inst[v]];
    double r = 2.0 * u01(seed, round, li) - 1.0;
    if (scale == 0) r = r * delta;
    bool pos = true, neg = true, zero = true;
    double sum = 0.0;
    int32_t sl[kVarBatch];
    T mv[kVarBatch];
    const int n = var_batch(P, mm, q0, q1, sl, mv);
    auto take = [&](double m) {
        pos = pos && m > tau;
        neg = neg && m < -tau;
        zero = zero && fabs(m) <= tau;
        sum += m;
    };
#pragma unroll
    for (int k = 0; k < kVarBatch; ++k)
        if (k < n) take((double)mv[k]);
    for (int32_t q = q0 + n; q < q1; ++q) take((double)mm[P.vslot[q]]);
    double pert;
    if (flag[v]) pert = r * delta;
    else if (pos) pert = delta;
    else if (neg) pert = -delta;
    else if (zero) pert = r * delta;
    else {
        const double mag = fabs(r) * delta;
        const int sg = sum > 0.0 ? 1 : sum < 0.0 ? -1 : (r >= 0.0 ? 1 : -1);
        pert = sg > 0 ? mag : -mag;
    }
    const T p = (T)pert;
    T lv[kVarBatch];
#pragma unroll
    for (int k = 0; k < kVarBatch; ++k)
        if (k < n) lv[k] = lam[sl[k]];
#pragma unroll
    for (int k = 0; k < kVarBatch; ++k)
        if (k < n) lam[sl[k]] = lv[k] + p;
    for (int32_t q = q0 + n; q < q1; ++q) {
        const int32_t s = P.vslot[q];
        lam[s] = lam[s] + p;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_decode(DevProblem P, const T *__restrict__ mm, uint8_t *__restrict__ x)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= P.n_vars) return;
    const int32_t q0 = P.vptr[v], q1 = P.vptr[v + 1];
    x[v] = (q0 != q1 && mm[P.vslot[q0]] < T(0)) ? 1 : 0;
}

// Exact feasibility of a decoded 0-1 point (Sec. 5, constraint set
// correspondence): walk every BDD along x; a BDD rejects x when the walk
// reaches the rejecting terminal.  Padding layers point at variable n_vars,
// whose x entry is 0 and whose chain nodes accept either value.
__global__ __launch_bounds__(kThreads) void k_check(DevProblem P, const uint8_t *__restrict__ x,
                                                    uint8_t *__restrict__ flag, int32_t *counter,
                                                    const uint8_t *__restrict__ only,
                                                    const int32_t *__restrict__ list, int64_t tile_count)
{
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t lt = xcd_block() * kWavesPerBlock + uni(threadIdx.x >> 6);
    if (lt >= tile_count) return;
    const int64_t tile = (int64_t)uni((uint32_t)list[lt]);
    const int32_t inst = P.tile_inst ? P.tile_inst[tile] : 0;
    if (only && !only[inst]) return;
    const TileView tv = load_tile(P.tiles + tile);
    // unused lanes of a partially filled tile carry the padding variable at
    // layer 0; they stand for no row
    if (P.pair_var[tv.pb + lane] >= P.n_vars) return;
    uint32_t node = 0;        // index inside the current layer
    bool ok = true;
    for (uint32_t h = 0; h < tv.K; ++h) {
        const uint32_t noff = uni(P.layers[tv.lb + h]) & 0xFFFFu;
        const uint32_t s = tv.pb + h * kLanes + lane;
        const uint32_t wd = node_word(P.child, tv, noff + (ok ? node : 0u), lane);
        const uint32_t nxt = x[P.pair_var[s]] ? (wd >> 16) : (wd & 0xFFFFu);
        if (nxt == kBot) ok = false;
        node = nxt;
    }
    ok = ok && node == kTop;
    if (!ok) {
        atomicAdd(counter + inst, 1);
        for (uint32_t h = 0; h < tv.K; ++h) flag[P.pair_var[tv.pb + h * kLanes + lane]] = 1;
    }
}

__global__ __launch_bounds__(256) void k_finalize_x(const int8_t *__restrict__ preset,
                                                   const uint8_t *__restrict__ xdec, uint8_t *__restrict__ xfull,
                                                   int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xfull[i] = preset[i] >= 0 ? (uint8_t)preset[i] : xdec[i];
}

// one thread per original row: sum_k a_k x_{c_k} (sense) b in int64
__global__ __launch_bounds__(kRedThreads) void k_row_check(DevRows R, const uint8_t *__restrict__ x,
                                                           int32_t *counter)
{
    __shared__ double sh[kRedThreads];
    const int64_t r = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    int bad = 0;
    if (r < R.n_rows) {
        int64_t lhs = 0;
        for (int64_t e = R.row_ptr[r]; e < R.row_ptr[r + 1]; ++e) lhs += (int64_t)R.coef[e] * (int64_t)x[R.col[e]];
        const int sn = R.sense[r];
        const int64_t b = R.rhs[r];
        bad = !(sn < 0 ? lhs <= b : sn > 0 ? lhs >= b : lhs == b);
    }
    if (R.row_inst) {
        if (bad) atomicAdd(counter + R.row_inst[r], 1);
        return;
    }
    const double t = block_sum((double)bad, sh);
    if (threadIdx.x == 0 && t > 0.0) atomicAdd(counter, (int32_t)t);
}

// objective of one chunk of variables [b, b + kObjChunk) (clipped to the
// chunk list's next start), fixed order
__global__ __launch_bounds__(kRedThreads) void k_obj_chunk(const double *__restrict__ cost,
                                                           const uint8_t *__restrict__ x,
                                                           const int64_t *__restrict__ chunk_begin,
                                                           double *__restrict__ part)
{
    __shared__ double sh[kRedThreads];
    const int64_t a = chunk_begin[blockIdx.x], b = chunk_begin[blockIdx.x + 1];
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) s += x[i] ? cost[i] : 0.0;
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[k] = max of part[seg[k] .. seg[k+1]) (0 for an empty segment); one block per segment
__global__ __launch_bounds__(kRedThreads) void k_seg_max(const double *__restrict__ part,
                                                         const int64_t *__restrict__ seg, double *__restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const int64_t a = seg[blockIdx.x], b = seg[blockIdx.x + 1];
    double m = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) m = fmax(m, part[i]);
    const double t = block_max(m, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// out[k] = offset[k] + sum of part[seg[k] .. seg[k+1]), fixed order; one block per segment
__global__ __launch_bounds__(kRedThreads) void k_seg_sum(const double *__restrict__ part,
                                                         const int64_t *__restrict__ seg,
                                                         const double *__restrict__ offset, double *__restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const int64_t a = seg[blockIdx.x], b = seg[blockIdx.x + 1];
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) s += part[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t + (offset ? offset[blockIdx.x] : 0.0);
}

__global__ __launch_bounds__(256) void k_take_x(const int32_t *__restrict__ var_inst, const uint8_t *__restrict__ x,
                                                uint8_t *__restrict__ xbest, const uint8_t *__restrict__ take,
                                                int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && take[var_inst ? var_inst[i] : 0]) xbest[i] = x[i];
}

// residual r_i = sum_j (lam + omega M) - c_i over one chunk of variables
// [chunk_begin[c], chunk_begin[c+1]) per block: sum of max(r_i, 0) and max |r_i|
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_residual_chunk(DevProblem P, const T *__restrict__ lam,
                                                                const T *__restrict__ mm, double omega,
                                                                const int64_t *__restrict__ chunk_begin,
                                                                double *__restrict__ pos_out,
                                                                double *__restrict__ max_out,
                                                                double *__restrict__ share)
{
    __shared__ double sh[kRedThreads];
    const int64_t a = chunk_begin[blockIdx.x], b = chunk_begin[blockIdx.x + 1];
    double pos = 0.0, mx = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) share[P.n_vars] = 0.0;
    for (int64_t v = a + threadIdx.x; v < b; v += kRedThreads) {
        const int32_t q0 = P.vptr[v], q1 = P.vptr[v + 1];
        if (q0 == q1) continue;
        double s = 0.0;
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t sl = P.vslot[q];
            s += (double)lam[sl] + omega * (double)mm[sl];
        }
        const double r = s - P.cost[v];
        share[v] = r / (double)(q1 - q0);
        if (r > 0.0) pos += r;
        mx = fmax(mx, fabs(r));
    }
    const double tp = block_sum(pos, sh);
    const double tm = block_max(mx, sh);
    if (threadIdx.x == 0) {
        pos_out[blockIdx.x] = tp;
        max_out[blockIdx.x] = tm;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *__restrict__ d, T v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(T *__restrict__ d, const T *__restrict__ s, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

inline unsigned grid8(int64_t tiles, int per_block)
{
    return (unsigned)((((tiles + per_block - 1) / per_block) + 7) & ~int64_t(7));
}

template <typename T, int DIR, int MODE>
void launch_general(const DevProblem &p, int list_lds, int list_glob, T *lam, T *mm, double *tile_lb, Omega<T> w,
                    hipStream_t st)
{
    const int64_t nl = p.list_off[list_lds + 1] - p.list_off[list_lds];
    const int64_t ng = p.list_off[list_glob + 1] - p.list_off[list_glob];
    if (nl > 0) {
        const size_t lds = (size_t)kWavesPerBlock * kLanes * p.lds_lane_elems * sizeof(T);
        hipLaunchKernelGGL((k_sweep<T, DIR, MODE, true>), dim3(grid8(nl, kWavesPerBlock)), dim3(kThreads), lds, st, p,
                           lam, mm, tile_lb, w, p.lists + p.list_off[list_lds], nl);
    }
    if (ng > 0)
        hipLaunchKernelGGL((k_sweep<T, DIR, MODE, false>), dim3(grid8(ng, kWavesPerBlock)), dim3(kThreads), 0, st, p,
                           lam, mm, tile_lb, w, p.lists + p.list_off[list_glob], ng);
}

}  // namespace

template <typename T, int DIR, bool UPD>
void launch_wide(const DevProblem &p, T *lam, T *mm, double *tile_lb, Omega<T> w, hipStream_t st)
{
    const int64_t n = p.list_off[LIST_WIDE + 1] - p.list_off[LIST_WIDE];
    if (n == 0) return;
    const int32_t *list = p.lists + p.list_off[LIST_WIDE];
    // a BDD's LDS region: distances, multipliers and terms (wide_elems
    // values), then its node words (4 B per node, at most wide_elems / 2
    // nodes); a block holds 64 / lanes regions within kWideBlockLds
    const size_t region = ((size_t)p.wide_elems * (sizeof(T) + 2) + 15) & ~(size_t)15;
    int lanes = p.wide_lanes;
    while (lanes < kLanes && (size_t)(kLanes / lanes) * region > (size_t)kWideBlockLds) lanes *= 2;
    const dim3 grid((unsigned)(n * lanes)), block(kLanes);
    const size_t lds = (size_t)(kLanes / lanes) * region;
    if (lanes == 16)
        hipLaunchKernelGGL((k_sweep_wide<T, DIR, UPD, 16>), grid, block, lds, st, p, lam, mm, w, list, n,
                           (uint32_t)region);
    else if (lanes == 32)
        hipLaunchKernelGGL((k_sweep_wide<T, DIR, UPD, 32>), grid, block, lds, st, p, lam, mm, w, list, n,
                           (uint32_t)region);
    else
        hipLaunchKernelGGL((k_sweep_wide<T, DIR, UPD, 64>), grid, block, lds, st, p, lam, mm, w, list, n,
                           (uint32_t)region);
    if (UPD && tile_lb)
        hipLaunchKernelGGL(k_wide_lb, dim3((unsigned)n), dim3(kLanes), 0, st, p.wide_part, list, tile_lb);
}

template <typename T>
void launch_sweep(const DevProblem &p, T *lam, T *mm, double *tile_lb, Omega<T> w, int dir, int mode, hipStream_t st)
{
    if (mode == MODE_UPDATE) {
        if (dir == 0) launch_wide<T, 0, true>(p, lam, mm, tile_lb, w, st);
        else launch_wide<T, 1, true>(p, lam, mm, tile_lb, w, st);
    } else {
        if (dir == 0) launch_wide<T, 0, false>(p, lam, mm, nullptr, w, st);
        else launch_wide<T, 1, false>(p, lam, mm, nullptr, w, st);
    }
    if (mode == MODE_UPDATE) {
        if (dir == 0) {
            launch_reg<T, 0, 2, true>(p, 0, lam, mm, tile_lb, w, st);
            launch_reg<T, 0, 4, true>(p, 1, lam, mm, tile_lb, w, st);
            launch_general<T, 0, MODE_UPDATE>(p, LIST_GEN_LDS_REST, LIST_GEN_GLOB_REST, lam, mm, tile_lb, w, st);
        } else {
            launch_reg<T, 1, 2, true>(p, 0, lam, mm, tile_lb, w, st);
            launch_reg<T, 1, 4, true>(p, 1, lam, mm, tile_lb, w, st);
            launch_general<T, 1, MODE_UPDATE>(p, LIST_GEN_LDS_REST, LIST_GEN_GLOB_REST, lam, mm, tile_lb, w, st);
        }
    } else {
        if (dir == 0) {
            launch_reg<T, 0, 2, false>(p, 0, lam, mm, nullptr, w, st);
            launch_reg<T, 0, 4, false>(p, 1, lam, mm, nullptr, w, st);
            launch_general<T, 0, MODE_FIXED>(p, LIST_GEN_LDS_REST, LIST_GEN_GLOB_REST, lam, mm, nullptr, w, st);
        } else {
            launch_reg<T, 1, 2, false>(p, 0, lam, mm, nullptr, w, st);
            launch_reg<T, 1, 4, false>(p, 1, lam, mm, nullptr, w, st);
            launch_general<T, 1, MODE_FIXED>(p, LIST_GEN_LDS_REST, LIST_GEN_GLOB_REST, lam, mm, nullptr, w, st);
        }
    }
}

template <typename T>
void launch_cert(const DevProblem &p, const T *lam, const T *mm, double omega, const double *share, double *tile_e,
                 hipStream_t st)
{
    const int64_t nl = p.list_off[LIST_GEN_LDS_ALL + 1] - p.list_off[LIST_GEN_LDS_ALL];
    const int64_t ng = p.list_off[LIST_GEN_GLOB_ALL + 1] - p.list_off[LIST_GEN_GLOB_ALL];
    if (nl > 0) {
        const size_t lds = (size_t)kWavesPerBlock * kLanes * p.lds_lane_elems * sizeof(T);
        hipLaunchKernelGGL((k_cert<T, true>), dim3(grid8(nl, kWavesPerBlock)), dim3(kThreads), lds, st, p, lam, mm,
                           omega, share, tile_e, p.lists + p.list_off[LIST_GEN_LDS_ALL], nl);
    }
    if (ng > 0)
        hipLaunchKernelGGL((k_cert<T, false>), dim3(grid8(ng, kWavesPerBlock)), dim3(kThreads), 0, st, p, lam, mm,
                           omega, share, tile_e, p.lists + p.list_off[LIST_GEN_GLOB_ALL], ng);
}

template <typename T>
void launch_average(const DevProblem &p, T *mm, double omega, hipStream_t st)
{
    if (p.gblocks == 0 || p.gmeta) return;
    hipLaunchKernelGGL((k_average<T>), dim3((unsigned)p.gblocks), dim3(kRedThreads), 0, st, p.gbucket_set,
                       p.gslot, p.vptr, p.vslot, mm, omega);
}

template <typename T>
void launch_gather_refresh(const DevProblem &p, const T *mm, int dir, hipStream_t st)
{
    if (!p.gmeta || p.n_g == 0) return;
    T *g = static_cast<T *>(p.gbuf) + (dir ? p.n_g : 0);
    hipLaunchKernelGGL((k_gather_refresh<T>), dim3(blocks_for(p.n_g, 256)), dim3(256), 0, st, p.gsrc, mm, g, p.n_g);
}

void launch_lb_many(const double *part, int64_t n_tiles, int64_t n, double offset, double *out, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_lb_many, dim3((unsigned)n), dim3(kRedThreads), 0, st, part, n_tiles, offset, out);
}

template <typename T>
void launch_average_all(const DevProblem &p, const T *mm, T *avg, double omega, hipStream_t st)
{
    if (p.n_vars > 0)
        hipLaunchKernelGGL((k_average_all<T>), dim3(blocks_for(p.n_vars, 256)), dim3(256), 0, st, p.vptr, p.vslot, mm,
                           avg, omega, p.n_vars);
}

void launch_reduce_sum(const double *part, int64_t n, double offset, double *scratch, double *out, hipStream_t st)
{
    const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 1023) / 1024));
    hipLaunchKernelGGL(k_sum_stage1, dim3(nb), dim3(kRedThreads), 0, st, part, n, scratch);
    hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(kRedThreads), 0, st, scratch, nb, offset, out);
}

template <typename T>
void launch_init(const DevProblem &p, T *lam, T *mm, hipStream_t st)
{
    if (p.n_slots > 0)
        hipLaunchKernelGGL((k_init<T>), dim3(blocks_for(p.n_slots, 256)), dim3(256), 0, st, p, lam, mm);
}

template <typename T>
void launch_terminate(const DevProblem &p, T *lam, const T *mm, T omega, hipStream_t st)
{
    if (p.n_slots > 0)
        hipLaunchKernelGGL((k_terminate<T>), dim3(blocks_for(p.n_slots, 256)), dim3(256), 0, st, p.n_slots, lam, mm,
                           omega);
}

template <typename T>
void launch_residual(const DevProblem &p, const T *lam, const T *mm, double omega, double *red, double *share,
                     hipStream_t st)
{
    // about two variables per thread: each thread's variables are dependent
    // loads (slots, then values), so parallelism hides them
    const int nb = (int)std::min<int64_t>(kResidualBlocks, std::max<int64_t>(1, (p.n_vars + 511) / 512));
    hipLaunchKernelGGL((k_residual<T>), dim3(nb), dim3(kRedThreads), 0, st, p, lam, mm, omega, red, share);
    hipLaunchKernelGGL(k_residual_stage2, dim3(1), dim3(kRedThreads), 0, st, red, nb);
}

template <typename T>
void launch_conflicts(const DevProblem &p, const T *mm, double tau, const uint8_t *flag, int32_t *counter,
                      int64_t n_inst, hipStream_t st)
{
    launch_fill<int32_t>(counter, 0, n_inst, st);
    if (p.n_vars > 0)
        hipLaunchKernelGGL((k_conflicts<T>), dim3(blocks_for(p.n_vars, kRedThreads)), dim3(kRedThreads), 0, st, p, mm,
                           tau, flag, counter);
}

template <typename T>
void launch_perturb(const DevProblem &p, T *lam, const T *mm, double tau, double delta, uint64_t seed,
                    uint64_t round, int scale, const uint8_t *flag, hipStream_t st)
{
    if (p.n_vars > 0)
        hipLaunchKernelGGL((k_perturb<T>), dim3(blocks_for(p.n_vars, 256)), dim3(256), 0, st, p, lam, mm, tau, delta,
                           seed, round, scale, flag);
}

template <typename T>
void launch_decode(const DevProblem &p, const T *mm, uint8_t *x, hipStream_t st)
{
    if (p.n_vars > 0)
        hipLaunchKernelGGL((k_decode<T>), dim3(blocks_for(p.n_vars, 256)), dim3(256), 0, st, p, mm, x);
}

void launch_finalize_x(const DevRows &r, int64_t n_vars, const uint8_t *xdec, uint8_t *xfull, hipStream_t st)
{
    if (n_vars > 0)
        hipLaunchKernelGGL(k_finalize_x, dim3(blocks_for(n_vars, 256)), dim3(256), 0, st, r.preset, xdec, xfull, n_vars);
}

void launch_row_check(const DevRows &r, const uint8_t *xfull, int32_t *counter, int64_t n_inst, hipStream_t st)
{
    launch_fill<int32_t>(counter, 0, n_inst, st);
    if (r.n_rows > 0)
        hipLaunchKernelGGL(k_row_check, dim3(blocks_for(r.n_rows, kRedThreads)), dim3(kRedThreads), 0, st, r, xfull,
                           counter);
}

void launch_obj_chunks(const double *cost, const uint8_t *x, const int64_t *chunk_begin, int64_t n_chunks,
                       int64_t n_vars, double *part, hipStream_t st)
{
    (void)n_vars;
    if (n_chunks > 0)
        hipLaunchKernelGGL(k_obj_chunk, dim3((unsigned)n_chunks), dim3(kRedThreads), 0, st, cost, x, chunk_begin, part);
}

void launch_seg_sum(const double *part, const int64_t *seg, int64_t n_seg, const double *offset, double *out,
                    hipStream_t st)
{
    if (n_seg > 0) hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)n_seg), dim3(kRedThreads), 0, st, part, seg, offset, out);
}

void launch_take_x(const DevProblem &p, const uint8_t *x, uint8_t *xbest, const uint8_t *take, hipStream_t st)
{
    if (p.n_vars > 0)
        hipLaunchKernelGGL(k_take_x, dim3(blocks_for(p.n_vars, 256)), dim3(256), 0, st, p.var_inst, x, xbest, take,
                           p.n_vars);
}

template <typename T>
void launch_residual_seg(const DevProblem &p, const T *lam, const T *mm, double omega, const int64_t *chunk_begin,
                         int64_t n_chunks, const int64_t *seg, int64_t n_inst, double *part_pos, double *part_max,
                         double *pos, double *mx, double *share, hipStream_t st)
{
    if (n_chunks > 0)
        hipLaunchKernelGGL((k_residual_chunk<T>), dim3((unsigned)n_chunks), dim3(kRedThreads), 0, st, p, lam, mm,
                           omega, chunk_begin, part_pos, part_max, share);
    if (n_inst > 0) {
        hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)n_inst), dim3(kRedThreads), 0, st, part_pos, seg,
                           (const double *)nullptr, pos);
        hipLaunchKernelGGL(k_seg_max, dim3((unsigned)n_inst), dim3(kRedThreads), 0, st, part_max, seg, mx);
    }
}

void launch_check(const DevProblem &p, const uint8_t *x, uint8_t *flag, int32_t *counter, const uint8_t *only,
                  int64_t n_inst, hipStream_t st)
{
    launch_fill<int32_t>(counter, 0, n_inst, st);
    for (int l : {(int)LIST_GEN_LDS_ALL, (int)LIST_GEN_GLOB_ALL}) {
        const int64_t n = p.list_off[l + 1] - p.list_off[l];
        if (n > 0)
            hipLaunchKernelGGL(k_check, dim3(grid8(n, kWavesPerBlock)), dim3(kThreads), 0, st, p, x, flag, counter,
                               only, p.lists + p.list_off[l], n);
    }
}

// pair_var from the variable -> slot lists (thread per variable); the
// padding slots keep the value the caller filled in before (n_vars)
__global__ __launch_bounds__(256) void k_pair_var(const int32_t *__restrict__ vptr,
                                                  const int32_t *__restrict__ vslot, int64_t n_vars,
                                                  int32_t *__restrict__ pair_var)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vars) return;
    for (int32_t q = vptr[v]; q < vptr[v + 1]; ++q) pair_var[vslot[q]] = (int32_t)v;
}

// instance of every variable from the instances' first variables:
// var_inst[v] = k with inst_var[k] <= v < inst_var[k + 1]
__global__ __launch_bounds__(256) void k_var_inst(const int64_t *__restrict__ inst_var, int64_t n_inst,
                                                  int64_t n_vars, int32_t *__restrict__ var_inst)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vars) return;
    int64_t lo = 0, hi = n_inst;   // inst_var[lo] <= v < inst_var[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (inst_var[mid] <= v) lo = mid;
        else hi = mid;
    }
    var_inst[v] = (int32_t)lo;
}

void launch_pair_var(const int32_t *vptr, const int32_t *vslot, int64_t n_vars, int64_t n_slots, int32_t *pair_var,
                     hipStream_t st)
{
    launch_fill<int32_t>(pair_var, (int32_t)n_vars, n_slots, st);
    if (n_vars > 0)
        hipLaunchKernelGGL(k_pair_var, dim3(blocks_for(n_vars, 256)), dim3(256), 0, st, vptr, vslot, n_vars, pair_var);
}

void launch_var_inst(const int64_t *inst_var, int64_t n_inst, int64_t n_vars, int32_t *var_inst, hipStream_t st)
{
    if (n_vars > 0 && n_inst > 0)
        hipLaunchKernelGGL(k_var_inst, dim3(blocks_for(n_vars, 256)), dim3(256), 0, st, inst_var, n_inst, n_vars,
                           var_inst);
}

template <typename T>
void launch_fill(T *dst, T value, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, dst, value, n);
}

template <typename T>
void launch_copy(T *dst, const T *src, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL((k_copy<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, dst, src, n);
}

#define BDDMMA_INSTANTIATE(T)                                                                                        \
    template void launch_sweep<T>(const DevProblem &, T *, T *, double *, Omega<T>, int, int, hipStream_t);         \
    template void launch_cert<T>(const DevProblem &, const T *, const T *, double, const double *, double *,        \
                                 hipStream_t);                                                                       \
    template void launch_average<T>(const DevProblem &, T *, double, hipStream_t);                                  \
    template void launch_gather_refresh<T>(const DevProblem &, const T *, int, hipStream_t);                        \
    template void launch_average_all<T>(const DevProblem &, const T *, T *, double, hipStream_t);                   \
    template void launch_init<T>(const DevProblem &, T *, T *, hipStream_t);                                        \
    template void launch_terminate<T>(const DevProblem &, T *, const T *, T, hipStream_t);                          \
    template void launch_residual<T>(const DevProblem &, const T *, const T *, double, double *, double *,          \
                                     hipStream_t);                                                                   \
    template void launch_conflicts<T>(const DevProblem &, const T *, double, const uint8_t *, int32_t *, int64_t,   \
                                      hipStream_t);                                                                  \
    template void launch_residual_seg<T>(const DevProblem &, const T *, const T *, double, const int64_t *,         \
                                         int64_t, const int64_t *, int64_t, double *, double *, double *, double *, \
                                         double *, hipStream_t);                                                     \
    template void launch_perturb<T>(const DevProblem &, T *, const T *, double, double, uint64_t, uint64_t, int,    \
                                    const uint8_t *, hipStream_t);                                                   \
    template void launch_decode<T>(const DevProblem &, const T *, uint8_t *, hipStream_t);                          \
    template void launch_fill<T>(T *, T, int64_t, hipStream_t);                                                      \
    template void launch_copy<T>(T *, const T *, int64_t, hipStream_t);

BDDMMA_INSTANTIATE(float)
BDDMMA_INSTANTIATE(double)
template void launch_fill<int32_t>(int32_t *, int32_t, int64_t, hipStream_t);
template void launch_fill<uint8_t>(uint8_t *, uint8_t, int64_t, hipStream_t);
template void launch_copy<uint8_t>(uint8_t *, const uint8_t *, int64_t, hipStream_t);

}  // namespace bddmma
