// Serial min-marginal averaging (the sequential update of Sec. 3 that the
// deferred scheme replaces), for ablation.  A sweep visits the variables
// level by level (levels in problem.hpp): one launch per level, one thread
// per variable of the level, which computes the min-marginal differences of
// the variable in every BDD containing it (from the distances kept in device
// memory), averages them, updates the multipliers and propagates the
// distances of those BDDs past the variable's layer.  Variables of a level
// share no BDD, so the threads write disjoint nodes and multipliers.
#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace bddmma {

namespace {

template <typename T>
__device__ __forceinline__ T inf_val() { return (T)__builtin_huge_val(); }

// SP(child, top): 0 for the accepting terminal, +inf for the rejecting one
template <typename T>
__device__ __forceinline__ T child_to_top(uint32_t c, int32_t next, const T *Bk)
{
    return c == kTop ? T(0) : c == kBot ? inf_val<T>() : Bk[next + (int32_t)c];
}

// terminated multipliers of every pair: lambda + omega M-bar (the state the
// serial scheme starts from)
template <typename T>
__global__ __launch_bounds__(256) void k_ser_gather(int64_t n, const int32_t *__restrict__ slot,
                                                    const T *__restrict__ lam, const T *__restrict__ mm, T w,
                                                    T *__restrict__ lam_p)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) lam_p[q] = lam[slot[q]] + w * mm[slot[q]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_ser_scatter(int64_t n, const int32_t *__restrict__ slot,
                                                     const T *__restrict__ lam_p, T *__restrict__ lam)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) lam[slot[q]] = lam_p[q];
}

// Start of a sweep, one thread per BDD.  DIR 0 (ascending variables):
// SP(., top) of every node at the current multipliers, SP(r, .) reset to +inf
// except at the root, energy reset.  DIR 1: SP(r, .) of every node.
template <typename T, int DIR>
__global__ __launch_bounds__(256) void k_ser_prep(int64_t nb, const int32_t *__restrict__ bpair,
                                                  const int4 *__restrict__ pinfo, const uint32_t *__restrict__ child,
                                                  const T *__restrict__ lam_p, T *__restrict__ F, T *__restrict__ Bk,
                                                  double *__restrict__ E)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t q0 = bpair[b], q1 = bpair[b + 1];
    if (q0 == q1) return;
    const int32_t root = pinfo[q0].x;
    const int4 last = pinfo[q1 - 1];
    const int32_t end = last.x + last.y;
    for (int32_t v = root; v < end; ++v) F[v] = inf_val<T>();
    F[root] = T(0);
    if (DIR == 0) {
        for (int32_t q = q1 - 1; q >= q0; --q) {
            const int4 L = pinfo[q];
            const T l = lam_p[q];
            for (int32_t v = L.x; v < L.x + L.y; ++v) {
                const uint32_t w = child[v];
                const T b0 = child_to_top<T>(w & 0xFFFFu, L.z, Bk);
                const T b1 = child_to_top<T>(w >> 16, L.z, Bk) + l;
                Bk[v] = b0 < b1 ? b0 : b1;
            }
        }
        E[b] = __builtin_huge_val();
    } else {
        for (int32_t q = q0; q < q1; ++q) {
            const int4 L = pinfo[q];
            const T l = lam_p[q];
            for (int32_t v = L.x; v < L.x + L.y; ++v) {
                const uint32_t w = child[v];
                for (int t = 0; t < 2; ++t) {
                    const uint32_t c = t ? (w >> 16) : (w & 0xFFFFu);
                    const T val = t ? F[v] + l : F[v];
                    if (c == kBot || c == kTop) continue;
                    T &dst = F[L.z + (int32_t)c];
                    if (val < dst) dst = val;
                }
            }
        }
    }
}

// One level: each thread takes one variable of the level.
template <typename T, int DIR>
__global__ __launch_bounds__(256) void k_ser_level(int64_t n, const int32_t *__restrict__ vars,
                                                   const int32_t *__restrict__ vptr, const int32_t *__restrict__ vpair,
                                                   const int32_t *__restrict__ bpair, const int4 *__restrict__ pinfo,
                                                   const uint32_t *__restrict__ child, T *__restrict__ lam_p,
                                                   T *__restrict__ mm_p, T *__restrict__ F, T *__restrict__ Bk,
                                                   double *__restrict__ E)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t i = vars[t];
    const int32_t a = vptr[i], z = vptr[i + 1];
    T sum = T(0);
    for (int32_t k = a; k < z; ++k) {
        const int32_t q = vpair[k];
        const int4 L = pinfo[q];
        const T l = lam_p[q];
        T m0 = inf_val<T>(), m1 = inf_val<T>();
        for (int32_t v = L.x; v < L.x + L.y; ++v) {
            const uint32_t w = child[v];
            const uint32_t lo = w & 0xFFFFu, hi = w >> 16;
            if (lo != kBot) {
                const T s0 = F[v] + child_to_top<T>(lo, L.z, Bk);
                if (s0 < m0) m0 = s0;
            }
            if (hi != kBot) {
                const T s1 = (F[v] + l) + child_to_top<T>(hi, L.z, Bk);
                if (s1 < m1) m1 = s1;
            }
        }
        const T M = m1 - m0;
        mm_p[q] = M;
        sum += M;
    }
    const T avg = (T)(1.0 / (double)(z - a)) * sum;
    for (int32_t k = a; k < z; ++k) {
        const int32_t q = vpair[k];
        const int4 L = pinfo[q];
        const T l = (lam_p[q] - mm_p[q]) + avg;
        lam_p[q] = l;
        if (DIR == 0) {
            double e = E[L.w];
            for (int32_t v = L.x; v < L.x + L.y; ++v) {
                const uint32_t w = child[v];
                for (int u = 0; u < 2; ++u) {
                    const uint32_t c = u ? (w >> 16) : (w & 0xFFFFu);
                    const T val = u ? F[v] + l : F[v];
                    if (c == kBot) continue;
                    if (c == kTop) {
                        if ((double)val < e) e = (double)val;
                    } else {
                        T &dst = F[L.z + (int32_t)c];
                        if (val < dst) dst = val;
                    }
                }
            }
            E[L.w] = e;
        } else {
            for (int32_t v = L.x; v < L.x + L.y; ++v) {
                const uint32_t w = child[v];
                const T b0 = child_to_top<T>(w & 0xFFFFu, L.z, Bk);
                const T b1 = child_to_top<T>(w >> 16, L.z, Bk) + l;
                Bk[v] = b0 < b1 ? b0 : b1;
            }
            if (q == bpair[L.w]) E[L.w] = (double)Bk[L.x];
        }
    }
}

unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
void launch_ser_gather(int64_t n, const int32_t *slot, const T *lam, const T *mm, T w, T *lam_p, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL((k_ser_gather<T>), dim3(blocks256(n)), dim3(256), 0, st, n, slot, lam, mm, w, lam_p);
}

template <typename T>
void launch_ser_scatter(int64_t n, const int32_t *slot, const T *lam_p, T *lam, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL((k_ser_scatter<T>), dim3(blocks256(n)), dim3(256), 0, st, n, slot, lam_p, lam);
}

template <typename T>
void launch_ser_prep(int dir, int64_t nb, const int32_t *bpair, const int32_t *pinfo, const uint32_t *child,
                     const T *lam_p, T *F, T *Bk, double *E, hipStream_t st)
{
    if (nb <= 0) return;
    const int4 *pi = reinterpret_cast<const int4 *>(pinfo);
    if (dir == 0)
        hipLaunchKernelGGL((k_ser_prep<T, 0>), dim3(blocks256(nb)), dim3(256), 0, st, nb, bpair, pi, child, lam_p, F,
                           Bk, E);
    else
        hipLaunchKernelGGL((k_ser_prep<T, 1>), dim3(blocks256(nb)), dim3(256), 0, st, nb, bpair, pi, child, lam_p, F,
                           Bk, E);
}

template <typename T>
void launch_ser_level(int dir, int64_t n, const int32_t *vars, const int32_t *vptr, const int32_t *vpair,
                      const int32_t *bpair, const int32_t *pinfo, const uint32_t *child, T *lam_p, T *mm_p, T *F,
                      T *Bk, double *E, hipStream_t st)
{
    if (n <= 0) return;
    const int4 *pi = reinterpret_cast<const int4 *>(pinfo);
    if (dir == 0)
        hipLaunchKernelGGL((k_ser_level<T, 0>), dim3(blocks256(n)), dim3(256), 0, st, n, vars, vptr, vpair, bpair, pi,
                           child, lam_p, mm_p, F, Bk, E);
    else
        hipLaunchKernelGGL((k_ser_level<T, 1>), dim3(blocks256(n)), dim3(256), 0, st, n, vars, vptr, vpair, bpair, pi,
                           child, lam_p, mm_p, F, Bk, E);
}

#define BDDMMA_SERIAL_INST(T)                                                                                         \
    template void launch_ser_gather<T>(int64_t, const int32_t *, const T *, const T *, T, T *, hipStream_t);           \
    template void launch_ser_scatter<T>(int64_t, const int32_t *, const T *, T *, hipStream_t);                        \
    template void launch_ser_prep<T>(int, int64_t, const int32_t *, const int32_t *, const uint32_t *, const T *, T *, \
                                     T *, double *, hipStream_t);                                                     \
    template void launch_ser_level<T>(int, int64_t, const int32_t *, const int32_t *, const int32_t *,                 \
                                      const int32_t *, const int32_t *, const uint32_t *, T *, T *, T *, T *, double *, \
                                      hipStream_t);
BDDMMA_SERIAL_INST(float)
BDDMMA_SERIAL_INST(double)

}  // namespace bddmma
