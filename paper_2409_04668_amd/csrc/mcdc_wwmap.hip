// Weight-window map: the log-importance network evaluated once at the centre
// of every cell of a regular (x, y, z, t) map per group, stored as the window
// target w_T, so that a check in the transport loop is one table read instead
// of a 64x64 network evaluation.  The map is a piecewise-constant version of
// the same importance function; splitting and roulette stay unbiased for any
// positive w_T, so only the variance changes.
#include "mcdc_runtime.hpp"
#include "transport_stages.hpp"

namespace mcdc {

// One thread per map cell, layout [g][t][z][y][x]; cell-centre inputs
// 2 (i + 1/2) / n - 1 per axis, rounded to float once.
__global__ void __launch_bounds__(256) k_ww_bake(DevProblem, const float *__restrict__ prm,
                                                 int32_t nx, int32_t ny, int32_t nz, int32_t nt,
                                                 uint64_t cells, double *__restrict__ out) {
    CP &P = kernel_problem();
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    uint64_t r = c;
    const int32_t n[4] = {nx, ny, nz, nt};
    int32_t idx[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        idx[a] = (int32_t)(r % (uint64_t)n[a]);
        r /= (uint64_t)n[a];
    }
    const int g = (int)r;
    float xt[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xt[a] = (float)(2.0 * (((double)idx[a] + 0.5) / (double)n[a]) - 1.0);
    out[c] = ww_net_target(P, prm, xt, g);
}

}  // namespace mcdc

using namespace mcdc;

extern "C" {

int mcdc_set_ww_map(mcdc_handle h, const int32_t n[4], double *dev_map, size_t capacity,
                    void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle has no weight windows");
    if (!dev_map) {
        h->P.ww_map = nullptr;
        for (int a = 0; a < 4; ++a) h->P.ww_map_n[a] = 0;
        return MCDC_OK;
    }
    if (!h->P.ww_on) return fail(MCDC_E_STATE, "set the network with mcdc_set_ww_mlp first");
    if (!n) return fail(MCDC_E_INVALID, "null map dimensions");
    uint64_t cells = (uint64_t)h->desc.G;
    for (int a = 0; a < 4; ++a) {
        if (n[a] < 1 || n[a] > (1 << 16)) return fail(MCDC_E_INVALID, "map dimensions must lie in [1, 65536]");
        cells *= (uint64_t)n[a];
    }
    if (cells > ((uint64_t)1 << 26)) return fail(MCDC_E_INVALID, "map larger than 2^26 cells");
    if (capacity < cells) return fail(MCDC_E_NOMEM, "map buffer smaller than G*nx*ny*nz*nt doubles");
    hipStream_t s = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL(k_ww_bake, dim3(blocks), dim3(256), 0, s, h->P,
                       (const float *)(h->ws + h->L.ww_params), n[0], n[1], n[2], n[3], cells,
                       dev_map);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "set_ww_map");
    h->P.ww_map = dev_map;
    for (int a = 0; a < 4; ++a) h->P.ww_map_n[a] = n[a];
    return MCDC_OK;
}

}  // extern "C"
