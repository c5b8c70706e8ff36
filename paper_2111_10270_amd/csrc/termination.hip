// Termination step of Alg. 1 in its averaging form: lambda_i^j +
// (omega/|J_i|) sum_k M-bar_ik, the averaged term coming from the averaging of
// all variables (avg[i], ascending row order); padding slots keep lambda.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bddmma {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_add_term(int64_t n_slots, int64_t n_vars, const int32_t *__restrict__ pair_var,
                                                  const T *lam, const T *__restrict__ avg, T *dst)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    const int32_t v = pair_var[s];
    dst[s] = v < n_vars ? lam[s] + avg[v] : lam[s];
}

}  // namespace

// dst may equal lam (in place)
template <typename T>
void launch_add_term(int64_t n_slots, int64_t n_vars, const int32_t *pair_var, const T *lam, const T *avg, T *dst,
                     hipStream_t st)
{
    if (n_slots > 0)
        hipLaunchKernelGGL((k_add_term<T>), dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st, n_slots, n_vars,
                           pair_var, lam, avg, dst);
}

template void launch_add_term<float>(int64_t, int64_t, const int32_t *, const float *, const float *, float *,
                                     hipStream_t);
template void launch_add_term<double>(int64_t, int64_t, const int32_t *, const double *, const double *, double *,
                                      hipStream_t);

}  // namespace bddmma
