// Micro-benchmarks that set the measured ceilings of the tally roofline:
// FP64 atomic adds at random bins of an array the size of a tally, and a
// streaming copy for the HBM ceiling.  Not part of the transport path.
#include "mcdc_runtime.hpp"

namespace mcdc {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // integer hash (xorshift-multiply finaliser); only spreads indices
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Each work-item performs `per_item` updates in runs of `run` consecutive
// bins starting at a hashed position (run = 1: fully random).
__global__ void __launch_bounds__(256) k_atomic_ceiling(double *__restrict__ buf, uint32_t n_bins,
                                                        uint32_t n_items, uint32_t per_item,
                                                        uint32_t run) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= n_items) return;
    uint32_t h = mix32(tid * 2654435761u + 12345u);
    for (uint32_t k = 0; k < per_item; k += run) {
        h = mix32(h + k);
        const uint32_t base = h % n_bins;
        for (uint32_t r = 0; r < run && k + r < per_item; ++r) {
            uint32_t i = base + r;
            if (i >= n_bins) i -= n_bins;
            unsafeAtomicAdd(buf + i, 1.0);
        }
    }
}

__global__ void __launch_bounds__(256) k_stream_copy(const double4 *__restrict__ src,
                                                     double4 *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace mcdc

using namespace mcdc;

extern "C" {

int mcdc_micro_atomics(double *dev_buf, uint64_t n_bins, uint64_t n_items, uint32_t per_item,
                       uint32_t run, void *stream) {
    if (!dev_buf || n_bins == 0 || n_bins > 0xFFFFFFFFull || per_item == 0 || run == 0)
        return fail(MCDC_E_INVALID, "micro_atomics arguments");
    if (n_items == 0 || n_items > (1ull << 31)) return fail(MCDC_E_INVALID, "micro_atomics item count");
    const int block = 256;
    const uint64_t grid = (n_items + block - 1) / block;
    hipLaunchKernelGGL(k_atomic_ceiling, dim3((uint32_t)grid), dim3(block), 0, (hipStream_t)stream,
                       dev_buf, (uint32_t)n_bins, (uint32_t)n_items, per_item, run);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "micro_atomics");
}

int mcdc_micro_copy(const void *dev_src, void *dev_dst, size_t bytes, void *stream) {
    if (!dev_src || !dev_dst || bytes % 32) return fail(MCDC_E_INVALID, "micro_copy: 32-byte multiple");
    const size_t n = bytes / 32;
    int dev = 0, n_cu = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        n_cu = prop.multiProcessorCount;
    hipLaunchKernelGGL(k_stream_copy, dim3(n_cu * 8), dim3(256), 0, (hipStream_t)stream,
                       (const double4 *)dev_src, (double4 *)dev_dst, n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "micro_copy");
}

}  // extern "C"
