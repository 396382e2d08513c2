// probe.hip -- memory-system microbenchmarks for gfx950, used by bench.py to
// put the hot-path kernels next to what the hardware sustains for their access
// patterns: a streaming copy (the HBM ceiling of the streaming kernels) and
// random 8-byte gathers and scatters through a precomputed index permutation
// (the ceiling of the rank-scatter and LCP kernels, whose cost is one random
// cache line per access).  Not part of the query path.

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__global__ __launch_bounds__(256) void copy_kernel(const int4 *__restrict__ src,
                                                   int4 *__restrict__ dst, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void gather_kernel(const uint32_t *__restrict__ idx,
                                                     const uint64_t *__restrict__ table,
                                                     uint64_t tn, uint64_t *__restrict__ out,
                                                     int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const uint64_t j = idx[i];
        out[i] = j < tn ? table[j] : 0;
    }
}

__global__ __launch_bounds__(256) void scatter_kernel(const uint32_t *__restrict__ idx,
                                                      const uint64_t *__restrict__ val,
                                                      uint64_t *__restrict__ table, uint64_t tn,
                                                      int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const uint64_t j = idx[i];
        if (j < tn) table[j] = val[i];
    }
}

unsigned grid(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return unsigned(b < 65536 ? b : 65536);
}

}  // namespace

extern "C" {

// All pointers are device pointers; sizes in elements; returns a hipError_t.
int probe_copy(const void *src, void *dst, int64_t n16, void *stream) {
    hipLaunchKernelGGL(copy_kernel, dim3(grid(n16)), dim3(256), 0, (hipStream_t)stream,
                       (const int4 *)src, (int4 *)dst, n16);
    return int(hipGetLastError());
}

int probe_gather(const uint32_t *idx, const uint64_t *table, int64_t tn, uint64_t *out, int64_t n,
                 void *stream) {
    hipLaunchKernelGGL(gather_kernel, dim3(grid(n)), dim3(256), 0, (hipStream_t)stream, idx, table,
                       uint64_t(tn), out, n);
    return int(hipGetLastError());
}

int probe_scatter(const uint32_t *idx, const uint64_t *val, uint64_t *table, int64_t tn, int64_t n,
                  void *stream) {
    hipLaunchKernelGGL(scatter_kernel, dim3(grid(n)), dim3(256), 0, (hipStream_t)stream, idx, val,
                       table, uint64_t(tn), n);
    return int(hipGetLastError());
}

}  // extern "C"
