// Renumbering of dats on the device (a plain gather through a permutation),
// and the small helper kernels of the static-scratch execution entry point:
// clearing words (a kernel, not a memset, so that the call can be captured
// in a HIP graph) and adding a device count into another.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace um {
namespace {

template <typename T, int LAYOUT>
__global__ __launch_bounds__(256) void gather_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                     const int32_t *__restrict__ idx, int64_t n,
                                                     int32_t dim) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * dim) return;
    if constexpr (LAYOUT == UM_AOS) {
        // consecutive lanes take consecutive components of consecutive rows
        const int64_t k = t / dim, c = t - k * dim;
        dst[t] = src[int64_t(idx[k]) * dim + c];
    } else {
        const int64_t c = t / n, k = t - c * n;
        dst[t] = src[c * n + idx[k]];
    }
}

template <typename T>
hipError_t gather(const void *src, void *dst, const int32_t *idx, int64_t n, int32_t dim,
                  int32_t layout, hipStream_t stream) {
    const int64_t total = n * dim;
    if (total == 0) return hipSuccess;
    dim3 block(256), grid(unsigned((total + 255) / 256));
    clear_stale_error();
    if (layout == UM_AOS)
        hipLaunchKernelGGL((gather_kernel<T, UM_AOS>), grid, block, 0, stream,
                           static_cast<const T *>(src), static_cast<T *>(dst), idx, n, dim);
    else
        hipLaunchKernelGGL((gather_kernel<T, UM_SOA>), grid, block, 0, stream,
                           static_cast<const T *>(src), static_cast<T *>(dst), idx, n, dim);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void zero_kernel(int32_t *__restrict__ p, int64_t n) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

__global__ void add_count_kernel(int32_t *dst, const int32_t *__restrict__ src) {
    if (threadIdx.x == 0 && src[0] != 0)
        __hip_atomic_fetch_add(dst, src[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

hipError_t zero_words(int32_t *p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    clear_stale_error();
    hipLaunchKernelGGL(zero_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t add_count(int32_t *dst, const int32_t *src, hipStream_t stream) {
    clear_stale_error();
    hipLaunchKernelGGL(add_count_kernel, dim3(1), dim3(64), 0, stream, dst, src);
    return hipGetLastError();
}

hipError_t permute_gather(const void *src, void *dst, const int32_t *idx, int64_t n, int32_t dim,
                          int32_t dtype, int32_t layout, hipStream_t stream) {
    if (dtype == UM_F64) return gather<double>(src, dst, idx, n, dim, layout, stream);
    return gather<float>(src, dst, idx, n, dim, layout, stream);
}

}  // namespace um
