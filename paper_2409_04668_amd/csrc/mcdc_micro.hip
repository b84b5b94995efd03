// Micro-benchmarks that set the measured ceilings of the tally roofline:
// FP64 atomic adds at random bins of an array the size of a tally (HBM), the
// same adds into a workgroup's LDS array the size of a hot tile (ds_add_f64),
// and a streaming copy for the HBM ceiling.  Not part of the transport path.
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

// Each work-item performs `per_item` LDS adds into its workgroup's array of
// n_bins doubles: it starts at a hashed bin and walks with its own odd
// stride modulo the largest power of two not above n_bins (an add and a mask
// per update, so the loop is bound by the ds_add_f64, not by the index
// arithmetic; the lanes of a wave hit scattered bins).  The array is zeroed
// first; at the end the workgroup's total is added to out[0] (one atomic per
// workgroup), which shows that no update was lost.
typedef __attribute__((address_space(3))) double lds_f64_t;
__global__ void __launch_bounds__(1024) k_lds_atomic_ceiling(double *__restrict__ out,
                                                             uint32_t n_bins, uint32_t n_items,
                                                             uint32_t per_item) {
    extern __shared__ double s_bins[];
    __shared__ double s_wave[16];
    for (uint32_t i = threadIdx.x; i < n_bins; i += blockDim.x) s_bins[i] = 0.0;
    __syncthreads();
    const uint32_t mask = (1u << (31 - __clz(n_bins))) - 1u;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n_items) {
        uint32_t i = mix32(tid * 2654435761u + 777u) & mask;
        const uint32_t step = (mix32(tid + 99u) | 1u) & mask;
        lds_f64_t *base = (lds_f64_t *)s_bins;
        for (uint32_t k = 0; k < per_item; ++k) {
            __hip_atomic_fetch_add(base + i, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            i = (i + step) & mask;
        }
    }
    __syncthreads();
    double t = 0.0;
    for (uint32_t i = threadIdx.x; i < n_bins; i += blockDim.x) t += s_bins[i];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w = 0.0;
        for (uint32_t k = 0; k < blockDim.x / 64; ++k) w += s_wave[k];
        if (w != 0.0) unsafeAtomicAdd(out, w);
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

int mcdc_micro_lds_atomics(double *dev_out, uint32_t n_bins, uint64_t n_items, uint32_t per_item,
                           void *stream) {
    if (!dev_out || n_bins < 2 || n_bins > MCDC_MAX_TILE_BINS || per_item == 0)
        return fail(MCDC_E_INVALID, "micro_lds_atomics arguments");
    if (n_items == 0 || n_items > (1ull << 31)) return fail(MCDC_E_INVALID, "micro_lds_atomics item count");
    const int block = 1024;
    const uint64_t grid = (n_items + block - 1) / block;
    const size_t shm = (size_t)n_bins * sizeof(double);
    if (shm > 65536)
        (void)hipFuncSetAttribute((const void *)k_lds_atomic_ceiling,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_lds_atomic_ceiling, dim3((uint32_t)grid), dim3(block), shm,
                       (hipStream_t)stream, dev_out, n_bins, (uint32_t)n_items, per_item);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "micro_lds_atomics");
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
