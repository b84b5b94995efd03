// Log-importance MLP (in -> 64 -> 64 -> 1, ReLU, FP32): forward, backward and
// Adam, trained full-batch on importance estimates that the transport itself
// produced.  Parameter layout: W1[64][in], b1[64], W2[64][64], b2[64], W3[64], b3.
//
// One training step is two launches:
//   k_mlp_step  one workgroup per 64 consecutive points: forward pass, loss,
//               backward pass and the gradient summed over its points (in
//               point order) into partial[workgroup][param];
//   k_mlp_adam  sums the workgroup partials in workgroup order (so a step is
//               reproducible bit for bit) and applies Adam.
// Inference (k_mlp_point) is one work-item per point.
#include <mutex>

#include "mcdc_runtime.hpp"

namespace mcdc {

constexpr int kPts = 64;                  // points per workgroup of a training step
constexpr int kLd = kH + 1;               // padded per-point row in LDS (no bank conflicts)

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

// One training step's gradient for points [64 b, 64 b + 64): 512 work-items,
// lane l of every wave is point 64 b + l, and wave w owns hidden units
// [8 w, 8 w + 8) of both layers.  Per-point activations and backward
// quantities live in LDS; parameters come through scalar loads.  Points past
// n contribute nothing (their dL/dout is zero).
constexpr int kStepThreads = 512;
constexpr int kUnits = kH / (kStepThreads / 64);   // hidden units per wave
constexpr size_t mlp_step_lds_floats(int in_dim) {
    return (size_t)kPts * in_dim + 4 * kPts * kLd + (kStepThreads / 64) * kPts + kPts;
}

__global__ void __launch_bounds__(kStepThreads) k_mlp_step(const float *__restrict__ prm, int in_dim,
                                                           const float *__restrict__ X,
                                                           const float *__restrict__ y,
                                                           const float *__restrict__ wt, size_t n,
                                                           MlpScratch S, float *__restrict__ loss) {
    constexpr int kWaves = kStepThreads / 64;
    extern __shared__ float sm[];
    float *s_x = sm;                                 // [64][in_dim]
    float *s_h1 = s_x + kPts * in_dim;               // [64][kLd]
    float *s_h2 = s_h1 + kPts * kLd;
    float *s_dz1 = s_h2 + kPts * kLd;
    float *s_dz2 = s_dz1 + kPts * kLd;
    float *s_op = s_dz2 + kPts * kLd;                // [waves][64] output partials
    float *s_dout = s_op + kWaves * kPts;            // [64]
    cparam_t *W1 = (cparam_t *)(uintptr_t)prm;
    cparam_t *b1 = W1 + kH * in_dim;
    cparam_t *W2 = b1 + kH;
    cparam_t *b2 = W2 + kH * kH;
    cparam_t *W3 = b2 + kH;
    const float b3 = W3[kH];
    const int np = mlp_np(in_dim);
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int u0 = kUnits * w;
    const size_t p0 = (size_t)blockIdx.x * kPts;
    for (int i = tid; i < kPts * in_dim; i += kStepThreads) {
        const size_t pi = p0 + (size_t)(i / in_dim);
        s_x[i] = pi < n ? X[p0 * in_dim + i] : 0.0f;
    }
    __syncthreads();
    const size_t p = p0 + l;
    // layer 1: this wave's units of point l
    for (int u = 0; u < kUnits; ++u) {
        const int i = u0 + u;
        float acc = b1[i];
        for (int k = 0; k < in_dim; ++k) acc = acc + W1[i * in_dim + k] * s_x[l * in_dim + k];
        s_h1[l * kLd + i] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // layer 2 (this wave's units) and its share of the output
    float a2[kUnits];
#pragma unroll
    for (int u = 0; u < kUnits; ++u) a2[u] = b2[u0 + u];
    for (int i = 0; i < kH; ++i) {
        const float h = s_h1[l * kLd + i];
#pragma unroll
        for (int u = 0; u < kUnits; ++u) a2[u] = a2[u] + W2[(u0 + u) * kH + i] * h;
    }
    float op = 0.0f;
#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
        const float h2 = a2[u] > 0.0f ? a2[u] : 0.0f;
        s_h2[l * kLd + u0 + u] = h2;
        op = op + W3[u0 + u] * h2;
    }
    s_op[w * kPts + l] = op;
    __syncthreads();
    // output (wave partials added in wave order), loss term and dL/dout
    float o = b3;
    for (int v = 0; v < kWaves; ++v) o = o + s_op[v * kPts + l];
    float lterm = 0.0f, dout = 0.0f;
    if (p < n) {
        const float inv = 1.0f / S.wsum[0];
        const float r = o - y[p];
        lterm = wt[p] * r * r * inv;
        dout = 2.0f * wt[p] * r * inv;
    }
    if (w == 0) s_dout[l] = dout;
#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
        const int j = u0 + u;
        s_dz2[l * kLd + j] = s_h2[l * kLd + j] > 0.0f ? dout * W3[j] : 0.0f;
    }
    __syncthreads();
    // dL/dz1 for this wave's units
    float a1[kUnits];
#pragma unroll
    for (int u = 0; u < kUnits; ++u) a1[u] = 0.0f;
    for (int j = 0; j < kH; ++j) {
        const float dz = s_dz2[l * kLd + j];
#pragma unroll
        for (int u = 0; u < kUnits; ++u) a1[u] = a1[u] + dz * W2[j * kH + u0 + u];
    }
#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
        const int i = u0 + u;
        s_dz1[l * kLd + i] = s_h1[l * kLd + i] > 0.0f ? a1[u] : 0.0f;
    }
    __syncthreads();
    // the workgroup's gradient, each parameter summed over its 64 points in
    // point order.  W2[j][i]: work-item (i = lane, wave w) takes rows
    // j = w, w + 8, ..., sharing each h1 read among them.
    float *part = S.partial + (size_t)blockIdx.x * np;
    const int ob1 = kH * in_dim, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
    {
        constexpr int kRows = kH / kWaves;
        float g2[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) g2[k] = 0.0f;
        for (int r = 0; r < kPts; ++r) {
            const float h = s_h1[r * kLd + l];
#pragma unroll
            for (int k = 0; k < kRows; ++k) g2[k] = g2[k] + s_dz2[r * kLd + w + kWaves * k] * h;
        }
#pragma unroll
        for (int k = 0; k < kRows; ++k) part[oW2 + (w + kWaves * k) * kH + l] = g2[k];
    }
    // every other parameter: W1, b1 (indices below oW2) and b2, W3, b3 (from ob2)
    const int n_small = oW2 + (np - ob2);
    for (int t = tid; t < n_small; t += kStepThreads) {
        const int q = t < oW2 ? t : ob2 + (t - oW2);
        float acc = 0.0f;
        if (q < ob1) {
            const int i = q / in_dim, k = q % in_dim;
            for (int r = 0; r < kPts; ++r) acc = acc + s_dz1[r * kLd + i] * s_x[r * in_dim + k];
        } else if (q < oW2) {
            const int i = q - ob1;
            for (int r = 0; r < kPts; ++r) acc = acc + s_dz1[r * kLd + i];
        } else if (q < oW3) {
            const int j = q - ob2;
            for (int r = 0; r < kPts; ++r) acc = acc + s_dz2[r * kLd + j];
        } else if (q < ob3) {
            const int j = q - oW3;
            for (int r = 0; r < kPts; ++r) acc = acc + s_dout[r] * s_h2[r * kLd + j];
        } else {
            for (int r = 0; r < kPts; ++r) acc = acc + s_dout[r];
        }
        part[q] = acc;
    }
    if (loss && w == 0) {
        // wave reduction, then one atomic per workgroup
        for (int off = 32; off > 0; off >>= 1) lterm += __shfl_xor(lterm, off);
        if (l == 0 && lterm != 0.0f) atomicAdd(loss, lterm);
    }
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

// gradient = sum of the workgroup partials (workgroup order); optional Adam
// update
__global__ void k_mlp_adam(int np, MlpScratch S, float *__restrict__ grad, float *__restrict__ prm,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                           float b2, float eps, float c1, float c2, int do_adam) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    // eight interleaved running sums (independent loads in flight), added
    // in a fixed order at the end
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.0f;
    int c = 0;
    for (; c + 8 <= S.groups; c += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] += S.partial[(size_t)(c + k) * np + q];
    }
    for (int k = 0; c < S.groups; ++c, ++k) a[k] += S.partial[(size_t)c * np + q];
    const float g = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    if (grad) grad[q] = g;
    if (do_adam) {
        const float mq = b1 * m[q] + (1.0f - b1) * g;
        const float vq = b2 * v[q] + (1.0f - b2) * g * g;
        m[q] = mq;
        v[q] = vq;
        const float mh = mq / c1;
        const float vh = vq / c2;
        prm[q] = prm[q] - lr * mh / (sqrtf(vh) + eps);
    }
}

static int mlp_check(int in_dim, size_t n) {
    if (in_dim < 5 || in_dim > 4 + kMaxG) return fail(MCDC_E_INVALID, "in_dim must be 4 + G, G in 1..8");
    if (n == 0) return fail(MCDC_E_INVALID, "no training points");
    if (n > (1u << 26)) return fail(MCDC_E_INVALID, "too many training points");
    return MCDC_OK;
}

static hipError_t step_grad(const float *prm, int in_dim, const float *X, const float *y,
                            const float *wt, size_t n, MlpScratch S, float *loss, hipStream_t s) {
    const size_t shm = mlp_step_lds_floats(in_dim) * sizeof(float);   // up to 71 KiB
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
    int step = *step_io;
    for (int i = 0; i < o->steps && e == hipSuccess; ++i) {
        step += 1;
        e = step_grad(prm, in_dim, X, y, wt, n, S, loss_hist ? loss_hist + i : nullptr, s);
        const float c1 = 1.0f - powf(o->beta1, (float)step);
        const float c2 = 1.0f - powf(o->beta2, (float)step);
        hipLaunchKernelGGL(k_mlp_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, S, grad, prm, m,
                           v, o->lr, o->beta1, o->beta2, o->eps, c1, c2, 1);
        if (e == hipSuccess) e = hipGetLastError();
    }
    *step_io = step;
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
                       (float *)nullptr, (float *)nullptr, (float *)nullptr, 0.f, 0.f, 0.f, 0.f,
                       1.f, 1.f, 0);
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
