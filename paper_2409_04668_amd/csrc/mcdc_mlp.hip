// Log-importance MLP (in -> 64 -> 64 -> 1, ReLU, FP32): forward, backward and
// Adam, trained full-batch on importance estimates that the transport itself
// produced.  Parameter layout: W1[64][in], b1[64], W2[64][64], b2[64], W3[64], b3.
//
// One training step is two launches:
//   k_mlp_step  one workgroup per 64 consecutive points: forward pass, loss,
//               backward pass and the gradient summed over its points into
//               partial[workgroup][param]; every contraction (layer 1, the
//               hidden layer forward and backward, the W1 and W2 gradients)
//               runs on the FP32 matrix cores;
//   k_mlp_adam  sums the workgroup partials in workgroup order (so a step is
//               reproducible bit for bit) and applies Adam.
// Inference (k_mlp_point) is one work-item per point.
#include <mutex>

#include "mcdc_runtime.hpp"

namespace mcdc {

constexpr int kPts = 64;                  // points per workgroup of a training step
constexpr int kLd = kH + 1;               // padded 64-wide row in LDS (fewer bank conflicts)

__host__ __device__ inline int mlp_np(int in_dim) { return kH * in_dim + kH + kH * kH + kH + kH + 1; }

struct MlpScratch {
    float *partial;                        // [workgroups][np]
    float *wsum;                           // [1]
    int groups;                            // workgroups of a step: ceil(n / kPts)
};

static int mlp_groups(size_t n) { return (int)((n + kPts - 1) / kPts); }

static size_t mlp_scratch_floats(size_t n, int in_dim) {
    return (size_t)mlp_groups(n) * mlp_np(in_dim) + 64;
}

static MlpScratch carve(float *base, size_t n, int in_dim) {
    MlpScratch s;
    s.partial = base;
    s.groups = mlp_groups(n);
    s.wsum = s.partial + (size_t)s.groups * mlp_np(in_dim);
    return s;
}

// Parameters are read-only and the same for every lane of a wave: they are
// read through the constant address space (uniform scalar loads into SGPRs).
typedef const __attribute__((address_space(4))) float cparam_t;

// Forward pass, one work-item per point.
__global__ void __launch_bounds__(256) k_mlp_point(const float *__restrict__ prm, int in_dim,
                                                   const float *__restrict__ X, size_t n,
                                                   float *__restrict__ out) {
    cparam_t *W1 = (cparam_t *)(uintptr_t)prm;
    cparam_t *b1 = W1 + kH * in_dim;
    cparam_t *W2 = b1 + kH;
    cparam_t *b2 = W2 + kH * kH;
    cparam_t *W3 = b2 + kH;
    const float b3 = W3[kH];
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float x[4 + kMaxG];
#pragma unroll
    for (int k = 0; k < 4 + kMaxG; ++k) x[k] = k < in_dim ? X[p * in_dim + k] : 0.0f;
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = b1[j];
#pragma unroll
        for (int k = 0; k < 4 + kMaxG; ++k)
            if (k < in_dim) acc = acc + W1[j * in_dim + k] * x[k];
        h1[j] = acc > 0.0f ? acc : 0.0f;
    }
    float o = b3;
    for (int j = 0; j < kH; ++j) {
        float acc = b2[j];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = acc + W2[j * kH + i] * h1[i];
        const float h2 = acc > 0.0f ? acc : 0.0f;
        o = o + W3[j] * h2;
    }
    out[p] = o;
}

// One block's gradient: points [64 b, 64 b + 64), 512 work-items.  The
// parameters are staged in LDS with the points' inputs and four per-point
// rows (h1, h2, dL/dz2, dL/dz1).  Inputs and W1 are padded to 16 columns: the
// input row gets a 1 in column in_dim and W1's row the bias b1 there, so one
// product gives layer 1 with its bias and one product the W1 and b1
// gradient.  The contractions run as 16 x 16 tiles of v_mfma_f32_16x16x4f32
// (lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of each 16 x 4 by
// 4 x 16 slice; result element r of lane l is D[4 (l / 16) + r][l % 16]):
// in the 64 x 64 products wave w takes row tile w % 4 and column tiles
// 2 (w / 4) and 2 (w / 4) + 1.  For the per-point work lane l of every wave is
// point 64 b + l and wave w owns hidden units [8 w, 8 w + 8).  Points past n
// contribute nothing (their dL/dout is zero).  Every sum runs in a fixed
// order.
constexpr int kStepThreads = 512;
constexpr int kWaves = kStepThreads / 64;
constexpr int kUnits = kH / kWaves;                 // hidden units per wave
constexpr int kXc = 16;                             // padded input columns
constexpr int kXs = kXc + 1;                        // their LDS row stride
static_assert(kH == 64 && kPts == 64 && kWaves == 8, "tiling assumes 64 x 64 blocks, 8 waves");
static_assert(4 + kMaxG < kXc, "the bias column follows the inputs");

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr size_t mlp_step_lds_floats() {             // 94.7 KiB
    return (size_t)2 * kH * kXs + (size_t)kH * kLd + kH + kH + 1 + 4 * kPts * kLd + kWaves * kPts + kPts;
}

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void block_grad(const float *prm, int in_dim, const float *__restrict__ X,
                                           const float *__restrict__ y,
                                           const float *__restrict__ wt, size_t n, float wsum,
                                           size_t blk, float *__restrict__ part, float *loss,
                                           float *sm) {
    const int np = mlp_np(in_dim);
    const int ob1 = kH * in_dim, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
    float *s_W1 = sm;                                // [64][kXs]: W1 | b1 | 0
    float *s_W2 = s_W1 + kH * kXs;                   // [64][kLd]
    float *s_b2 = s_W2 + kH * kLd;
    float *s_W3 = s_b2 + kH;                         // W3[64], then b3
    float *s_x = s_W3 + kH + 1;                      // [64][kXs]: x | 1 | 0
    float *s_h1 = s_x + kPts * kXs;                  // [64][kLd]
    float *s_h2 = s_h1 + kPts * kLd;
    float *s_dz2 = s_h2 + kPts * kLd;
    float *s_dz1 = s_dz2 + kPts * kLd;
    float *s_op = s_dz1 + kPts * kLd;                // [waves][64] output partials
    float *s_dout = s_op + kWaves * kPts;            // [64]
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int u0 = kUnits * w;
    const int m16 = l & 15, k4 = l >> 4;
    const int rt = w & 3, ct = (w >> 2) * 2;         // row tile, first column tile
    const size_t p0 = blk * kPts;
    const size_t p = p0 + l;
    // this point's target and weight, loaded early (first wave only)
    float yp = 0.0f, wp = 0.0f;
    if (w == 0 && p < n) {
        yp = y[p];
        wp = wt[p];
    }
    // staging, every load issued before the first store: the padded W1 and
    // input rows (64 x 16 each), then W2 (rows padded to kLd), b2, W3, b3
    constexpr int kPad = kH * kXc / kStepThreads;
    constexpr int kRest = (kH * kH + kH + kH + 1 + kStepThreads - 1) / kStepThreads;
    const int n_rest = np - oW2;
    float vw[kPad], vx[kPad], vr[kRest];
#pragma unroll
    for (int k = 0; k < kPad; ++k) {
        const int e = tid + k * kStepThreads, i = e / kXc, c = e % kXc;
        vw[k] = c < in_dim ? prm[i * in_dim + c] : c == in_dim ? prm[ob1 + i] : 0.0f;
        vx[k] = c < in_dim ? (p0 + i < n ? X[(p0 + i) * in_dim + c] : 0.0f) : c == in_dim ? 1.0f : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kRest; ++k) {
        const int j = tid + k * kStepThreads;
        vr[k] = j < n_rest ? prm[oW2 + j] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kPad; ++k) {
        const int e = tid + k * kStepThreads, i = e / kXc, c = e % kXc;
        s_W1[i * kXs + c] = vw[k];
        s_x[i * kXs + c] = vx[k];
    }
#pragma unroll
    for (int k = 0; k < kRest; ++k) {
        const int j = tid + k * kStepThreads;
        if (j < n_rest) s_W2[j < kH * kH ? (j >> 6) * kLd + (j & 63) : j + kH * (kLd - kH)] = vr[k];
    }
    __syncthreads();
    // layer 1: z1[p][i] = sum_c x[p][c] W1[i][c] (the bias through the 1 column)
    {
        f32x4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
        for (int kk = 0; kk < kXc / 4; ++kk) {
            const float a = s_x[(16 * rt + m16) * kXs + 4 * kk + k4];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = mfma4(a, s_W1[(16 * (ct + t) + m16) * kXs + 4 * kk + k4], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[t][r];
                s_h1[(16 * rt + 4 * k4 + r) * kLd + 16 * (ct + t) + m16] = z > 0.0f ? z : 0.0f;
            }
    }
    __syncthreads();
    // layer 2: z2[p][j] = sum_i h1[p][i] W2[j][i] (+ b2[j])
    {
        f32x4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
        for (int kk = 0; kk < kH / 4; ++kk) {
            const float a = s_h1[(16 * rt + m16) * kLd + 4 * kk + k4];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = mfma4(a, s_W2[(16 * (ct + t) + m16) * kLd + 4 * kk + k4], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = 16 * rt + 4 * k4 + r, j = 16 * (ct + t) + m16;
                const float z = acc[t][r] + s_b2[j];
                s_h2[pp * kLd + j] = z > 0.0f ? z : 0.0f;
            }
    }
    __syncthreads();
    // this wave's units' share of the output of point l
    float op = 0.0f;
#pragma unroll
    for (int u = 0; u < kUnits; ++u) op = op + s_W3[u0 + u] * s_h2[l * kLd + u0 + u];
    s_op[w * kPts + l] = op;
    __syncthreads();
    // output (wave partials added in wave order), loss term and dL/dout:
    // wave 0 for every point
    float lterm = 0.0f;
    if (w == 0) {
        float o = s_W3[kH];
        for (int v = 0; v < kWaves; ++v) o = o + s_op[v * kPts + l];
        float dout = 0.0f;
        if (p < n) {
            const float inv = 1.0f / wsum;
            const float r = o - yp;
            lterm = wp * r * r * inv;
            dout = 2.0f * wp * r * inv;
        }
        s_dout[l] = dout;
    }
    __syncthreads();
    const float dout = s_dout[l];
#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
        const int j = u0 + u;
        s_dz2[l * kLd + j] = s_h2[l * kLd + j] > 0.0f ? dout * s_W3[j] : 0.0f;
    }
    __syncthreads();
    // dL/dz1[p][i] = [h1 > 0] sum_j dz2[p][j] W2[j][i], and the W2 gradient
    // g[j][i] = sum_p dz2[p][j] h1[p][i] (row tile over j, the sum over points)
    {
        f32x4 d1[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
        f32x4 g2[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll 8
        for (int kk = 0; kk < kH / 4; ++kk) {
            const float a1 = s_dz2[(16 * rt + m16) * kLd + 4 * kk + k4];
            const float a2 = s_dz2[(4 * kk + k4) * kLd + 16 * rt + m16];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int c = 16 * (ct + t) + m16;
                d1[t] = mfma4(a1, s_W2[(4 * kk + k4) * kLd + c], d1[t]);
                g2[t] = mfma4(a2, s_h1[(4 * kk + k4) * kLd + c], g2[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rt + 4 * k4 + r, c = 16 * (ct + t) + m16;
                s_dz1[row * kLd + c] = s_h1[row * kLd + c] > 0.0f ? d1[t][r] : 0.0f;
                part[oW2 + row * kH + c] = g2[t][r];
            }
    }
    __syncthreads();
    if (w < 4) {
        // W1 and b1: g[i][c] = sum_p dz1[p][i] x[p][c] (row tile w over i;
        // column in_dim, the 1 column, is the b1 gradient)
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 8
        for (int kk = 0; kk < kPts / 4; ++kk)
            acc = mfma4(s_dz1[(4 * kk + k4) * kLd + 16 * w + m16], s_x[(4 * kk + k4) * kXs + m16], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + 4 * k4 + r;
            if (m16 < in_dim) part[i * in_dim + m16] = acc[r];
            else if (m16 == in_dim) part[ob1 + i] = acc[r];
        }
    } else {
        // b2, W3 and b3, each summed over the 64 points in point order
        for (int t = tid - kStepThreads / 2; t < np - ob2; t += kStepThreads / 2) {
            const int q = ob2 + t;
            float acc = 0.0f;
            if (q < oW3) {
#pragma unroll 16
                for (int r = 0; r < kPts; ++r) acc = acc + s_dz2[r * kLd + t];
            } else if (q < ob3) {
                const int j = q - oW3;
#pragma unroll 16
                for (int r = 0; r < kPts; ++r) acc = acc + s_dout[r] * s_h2[r * kLd + j];
            } else {
#pragma unroll 16
                for (int r = 0; r < kPts; ++r) acc = acc + s_dout[r];
            }
            part[q] = acc;
        }
    }
    if (loss && w == 0) {
        // wave reduction, then one atomic per workgroup
        for (int off = 32; off > 0; off >>= 1) lterm += __shfl_xor(lterm, off);
        if (l == 0 && lterm != 0.0f) atomicAdd(loss, lterm);
    }
}

__global__ void __launch_bounds__(kStepThreads) k_mlp_step(const float *__restrict__ prm, int in_dim,
                                                           const float *__restrict__ X,
                                                           const float *__restrict__ y,
                                                           const float *__restrict__ wt, size_t n,
                                                           MlpScratch S, float *__restrict__ loss) {
    extern __shared__ float sm[];
    block_grad(prm, in_dim, X, y, wt, n, S.wsum[0], blockIdx.x,
               S.partial + (size_t)blockIdx.x * mlp_np(in_dim), loss, sm);
}

__global__ void k_mlp_wsum(const float *__restrict__ wt, size_t n, float *__restrict__ wsum) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) acc += wt[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsum[0] = red[0];
}

struct AdamArgs {
    float lr, b1, b2, eps;
};

// Parameter q: the gradient as the sum of the workgroup partials (workgroup
// order); with `adam`, Adam step number `step` on it (bias corrections
// 1 - beta^step, taken on the device).
__device__ __forceinline__ void adam_param(int q, int np, const MlpScratch &S, float *grad, float *prm,
                                           float *m, float *v, const AdamArgs &A, int step, bool adam) {
    // the moments and the parameter first, then up to 96 partials in flight;
    // eight interleaved running sums, a[k] over the partials c = k mod 8 in
    // increasing c (zeros past the last one), added in a fixed order at the end
    float mq = 0.0f, vq = 0.0f, pq = 0.0f;
    if (adam) {
        mq = m[q];
        vq = v[q];
        pq = prm[q];
    }
    constexpr int kBatch = 96;
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.0f;
    for (int c = 0; c < S.groups; c += kBatch) {
        float t[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) t[k] = c + k < S.groups ? S.partial[(size_t)(c + k) * np + q] : 0.0f;
#pragma unroll
        for (int k = 0; k < kBatch; ++k) a[k & 7] += t[k];
    }
    const float g = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    if (grad) grad[q] = g;
    if (adam) {
        const float c1 = 1.0f - powf(A.b1, (float)step);
        const float c2 = 1.0f - powf(A.b2, (float)step);
        mq = A.b1 * mq + (1.0f - A.b1) * g;
        vq = A.b2 * vq + (1.0f - A.b2) * g * g;
        m[q] = mq;
        v[q] = vq;
        const float mh = mq / c1;
        const float vh = vq / c2;
        prm[q] = pq - A.lr * mh / (sqrtf(vh) + A.eps);
    }
}

// gradient = sum of the workgroup partials; optional Adam update
__global__ void k_mlp_adam(int np, MlpScratch S, float *__restrict__ grad, float *__restrict__ prm,
                           float *__restrict__ m, float *__restrict__ v, AdamArgs A, int step,
                           int do_adam) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < np) adam_param(q, np, S, grad, prm, m, v, A, step, do_adam != 0);
}

static int mlp_check(int in_dim, size_t n) {
    if (in_dim < 5 || in_dim > 4 + kMaxG) return fail(MCDC_E_INVALID, "in_dim must be 4 + G, G in 1..8");
    if (n == 0) return fail(MCDC_E_INVALID, "no training points");
    if (n > (1u << 26)) return fail(MCDC_E_INVALID, "too many training points");
    return MCDC_OK;
}

static hipError_t step_grad(const float *prm, int in_dim, const float *X, const float *y,
                            const float *wt, size_t n, MlpScratch S, float *loss, hipStream_t s) {
    const size_t shm = mlp_step_lds_floats() * sizeof(float);
    if (shm > 65536)
        (void)hipFuncSetAttribute((const void *)k_mlp_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shm);
    hipLaunchKernelGGL(k_mlp_step, dim3(S.groups), dim3(kStepThreads), shm, s, prm, in_dim, X, y, wt,
                       n, S, loss);
    return hipGetLastError();
}

// Training scratch of mcdc_mlp_train_noalloc, for callers that cannot
// allocate: a static array in device memory (each GPU the library runs on
// holds its own copy until the process ends).  In host code the array's name
// is not a device address; its address on the current device comes from
// hipGetSymbolAddress, taken once per device on the entry point's first call
// there and kept.  Calls that overlap on one GPU share the array and race.
constexpr size_t kStaticScratchFloats = (size_t)1 << 22;      // 16 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[kMaxDevices];

static int static_scratch(float **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "mlp_train_noalloc: current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(MCDC_E_INVALID, "mlp_train_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "mlp_train_noalloc: scratch address");
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return MCDC_OK;
}

__global__ void k_zero_f32(float *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// `steps` Adam steps with the scratch S; the loss history is cleared by a
// memset (the scratch entry point, as it always did) or by a fill kernel
// (the entry point that allocates nothing, which a caller may capture in a
// graph).
static hipError_t train_steps(float *prm, int in_dim, const float *X, const float *y,
                              const float *wt, size_t n, float *m, float *v, float *grad,
                              const mcdc_train_opts *o, int32_t *step_io, float *loss_hist,
                              MlpScratch S, bool fill_kernel, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (loss_hist && o->steps > 0) {
        if (fill_kernel)
            hipLaunchKernelGGL(k_zero_f32, dim3((o->steps + 255) / 256), dim3(256), 0, s, loss_hist,
                               o->steps);
        else
            e = hipMemsetAsync(loss_hist, 0, o->steps * sizeof(float), s);
    }
    hipLaunchKernelGGL(k_mlp_wsum, dim3(1), dim3(256), 0, s, wt, n, S.wsum);
    const int np = mlp_np(in_dim);
    const AdamArgs A{o->lr, o->beta1, o->beta2, o->eps};
    const int step0 = *step_io;
    int done = 0;
    for (; done < o->steps && e == hipSuccess; ++done) {
        e = step_grad(prm, in_dim, X, y, wt, n, S, loss_hist ? loss_hist + done : nullptr, s);
        hipLaunchKernelGGL(k_mlp_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, S, grad, prm, m,
                           v, A, step0 + done + 1, 1);
        if (e == hipSuccess) e = hipGetLastError();
    }
    *step_io = step0 + done;
    return e;
}

}  // namespace mcdc

using namespace mcdc;

extern "C" {

size_t mcdc_mlp_scratch_bytes(int32_t in_dim, size_t n) {
    return mlp_scratch_floats(n, in_dim) * sizeof(float);
}

int mcdc_mlp_forward(const float *prm, int32_t in_dim, const float *X, size_t n, float *out,
                     void *stream) {
    int st = mlp_check(in_dim, n);
    if (st) return st;
    if (!prm || !X || !out) return fail(MCDC_E_INVALID, "null buffer");
    const int block = 256;
    hipLaunchKernelGGL(k_mlp_point, dim3((n + block - 1) / block), dim3(block), 0,
                       (hipStream_t)stream, prm, in_dim, X, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp_forward");
}

int mcdc_mlp_grad(const float *prm, int32_t in_dim, const float *X, const float *y,
                  const float *wt, size_t n, float *grad, float *loss, void *scratch,
                  void *stream) {
    int st = mlp_check(in_dim, n);
    if (st) return st;
    if (!prm || !X || !y || !wt || !grad || !scratch) return fail(MCDC_E_INVALID, "null buffer");
    hipStream_t s = (hipStream_t)stream;
    MlpScratch S = carve((float *)scratch, n, in_dim);
    hipError_t e = hipSuccess;
    if (loss) e = hipMemsetAsync(loss, 0, sizeof(float), s);
    hipLaunchKernelGGL(k_mlp_wsum, dim3(1), dim3(256), 0, s, wt, n, S.wsum);
    if (e == hipSuccess) e = step_grad(prm, in_dim, X, y, wt, n, S, loss, s);
    const int np = mlp_np(in_dim);
    hipLaunchKernelGGL(k_mlp_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, S, grad,
                       (float *)nullptr, (float *)nullptr, (float *)nullptr, AdamArgs{0.f, 0.f, 0.f, 0.f},
                       0, 0);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp_grad");
}

int mcdc_mlp_train(float *prm, int32_t in_dim, const float *X, const float *y, const float *wt,
                   size_t n, float *m, float *v, float *grad, const mcdc_train_opts *o,
                   int32_t *step_io, float *loss_hist, void *scratch, void *stream) {
    int st = mlp_check(in_dim, n);
    if (st) return st;
    if (!prm || !X || !y || !wt || !m || !v || !o || !step_io || !scratch)
        return fail(MCDC_E_INVALID, "null buffer");
    if (o->steps < 0) return fail(MCDC_E_INVALID, "negative step count");
    MlpScratch S = carve((float *)scratch, n, in_dim);
    hipError_t e = train_steps(prm, in_dim, X, y, wt, n, m, v, grad, o, step_io, loss_hist, S, false,
                               (hipStream_t)stream);
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp_train");
}

int mcdc_mlp_train_noalloc(float *prm, int32_t in_dim, const float *X, const float *y,
                           const float *wt, size_t n, float *m, float *v, float *grad,
                           const mcdc_train_opts *o, int32_t *step_io, float *loss_hist,
                           void *stream) {
    int st = mlp_check(in_dim, n);
    if (st) return st;
    if (!prm || !X || !y || !wt || !m || !v || !o || !step_io) return fail(MCDC_E_INVALID, "null buffer");
    if (o->steps < 0) return fail(MCDC_E_INVALID, "negative step count");
    if (mlp_scratch_floats(n, in_dim) > kStaticScratchFloats)
        return fail(MCDC_E_INVALID, "mlp_train_noalloc: " + std::to_string(n) + " points need " +
                                        std::to_string(mlp_scratch_floats(n, in_dim) * sizeof(float)) +
                                        " bytes of scratch, more than its static 16 MiB");
    float *base = nullptr;
    if ((st = static_scratch(&base))) return st;
    MlpScratch S = carve(base, n, in_dim);
    hipError_t e = train_steps(prm, in_dim, X, y, wt, n, m, v, grad, o, step_io, loss_hist, S, true,
                               (hipStream_t)stream);
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp_train_noalloc");
}

}  // extern "C"
