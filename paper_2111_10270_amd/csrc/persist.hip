// Persistent sweep kernel: a block of Alg. 1 sweeps in one cooperative
// launch, with a grid-wide barrier between consecutive sweeps instead of a
// kernel boundary.  Used (option `persistent`) for problems whose tiles all
// belong to one mixed register class and whose cross-tile averaging runs
// inside the sweep (fused averaging), so a sweep has no other launch.  Each
// wave keeps the same tiles in every sweep.  Compiled once per precision
// (BDDMMA_PERSIST_T).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <utility>

#include "device_common.hpp"
#include "kernels.hpp"
#include "sweep_tile.hpp"

#ifndef BDDMMA_PERSIST_T
#define BDDMMA_PERSIST_T float
#endif

namespace bddmma {

namespace {

// n_sweeps sweeps from direction dir0 over the tiles of `list`; sweep s writes
// its per-tile bound partials to row s of lbpart (rows of lb_stride doubles)
template <typename T, int KMAX, bool GAT>
__global__ __launch_bounds__(kLanes) void k_persist(DevProblem P, T *__restrict__ lam, T *__restrict__ mm,
                                                     double *__restrict__ lbpart, int64_t lb_stride, Omega<T> w,
                                                     const int32_t *__restrict__ list, int64_t tile_count,
                                                     int32_t first, int32_t n_sweeps, int32_t dir0)
{
    extern __shared__ __align__(16) unsigned char lds_bytes[];
    T *sh = reinterpret_cast<T *>(lds_bytes);
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int64_t stride = gridDim.x;
    for (int32_t s = 0; s < n_sweeps; ++s) {
        double *tile_lb = lbpart + (int64_t)s * lb_stride;
        const bool fwd = ((dir0 + s) & 1) == 0;
        for (int64_t lt = xcd_block(); lt < tile_count; lt += stride) {
            const int64_t tile = first >= 0 ? first + lt : (int64_t)uni((uint32_t)list[lt]);
            if (fwd) sweep_tile<T, 0, 2, KMAX, true, false, GAT>(P, lam, mm, tile_lb, w, tile, sh);
            else sweep_tile<T, 1, 2, KMAX, true, false, GAT>(P, lam, mm, tile_lb, w, tile, sh);
        }
        // every tile's new differences (and their per-variable copies) are
        // visible to every wave before the next sweep reads them
        if (s + 1 < n_sweeps) grid.sync();
    }
}

template <typename T, int KI>
const void *persist_fn(bool fused)
{
    constexpr bool can_fuse = fuse_class_ok(sizeof(T), kKClass[KI]);
    if (fused && !can_fuse) return nullptr;
    return fused ? reinterpret_cast<const void *>(&k_persist<T, kKClass[KI], can_fuse>)
                 : reinterpret_cast<const void *>(&k_persist<T, kKClass[KI], false>);
}

// kernel and LDS bytes of layer class ki
template <typename T, int... KI>
const void *persist_fn_of(int ki, bool fused, size_t &lds, std::integer_sequence<int, KI...>)
{
    const void *f = nullptr;
    ((ki == KI ? (void)(f = persist_fn<T, KI>(fused), lds = sweep_lds_bytes<T, kKClass[KI]>()) : (void)0), ...);
    return f;
}

}  // namespace

template <typename T>
int launch_persist(const DevProblem &p, int ki, T *lam, T *mm, double *lbpart, int64_t lb_stride, Omega<T> w,
                   int32_t n_sweeps, int32_t dir0, hipStream_t st)
{
    const int l = mix_list(ki);
    int64_t tile_count = p.list_off[l + 1] - p.list_off[l];
    if (tile_count == 0 || n_sweeps <= 0) return 0;
    size_t lds = 0;
    const void *f = persist_fn_of<T>(ki, p.gmeta != nullptr, lds, std::make_integer_sequence<int, kNumKClasses>{});
    if (!f) return -1;
    // every block must be resident at once: at most the co-resident blocks,
    // a multiple of 8 (one eighth per XCD); waves loop over further tiles
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kLanes, lds) != hipSuccess)
        return -1;
    const int64_t resident = ((int64_t)cus * per_cu) & ~int64_t(7);
    if (resident < 8) return -1;
    const int64_t grid = std::min<int64_t>((tile_count + 7) & ~int64_t(7), resident);
    const int32_t *list = p.lists + p.list_off[l];
    DevProblem pp = p;
    int32_t first = p.list_first[l];
    void *args[] = {&pp, &lam, &mm, &lbpart, &lb_stride, &w, &list, &tile_count, &first, &n_sweeps, &dir0};
    return hipLaunchCooperativeKernel(f, dim3((unsigned)grid), dim3(kLanes), args, (unsigned)lds, st) == hipSuccess ? 0
                                                                                                               : -1;
}

template int launch_persist<BDDMMA_PERSIST_T>(const DevProblem &, int, BDDMMA_PERSIST_T *, BDDMMA_PERSIST_T *,
                                              double *, int64_t, Omega<BDDMMA_PERSIST_T>, int32_t, int32_t,
                                              hipStream_t);

}  // namespace bddmma
