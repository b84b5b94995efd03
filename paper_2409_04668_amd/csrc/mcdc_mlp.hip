// Log-importance MLP (in -> 64 -> 64 -> 1, ReLU, FP32): forward, backward and
// Adam, trained full-batch on importance estimates that the transport itself
// produced.  Parameter layout: W1[64][in], b1[64], W2[64][64], b2[64], W3[64], b3.
//
// One training step is three launches:
//   k_mlp_point   one work-item per point: forward pass, loss term, and the
//                 per-point backward quantities dL/dout, dL/dz2 (64), dL/dz1 (64),
//                 stored with h1, h2 in a caller-provided scratch buffer;
//   k_mlp_partial each work-item owns one parameter and sums its gradient over
//                 a contiguous chunk of points (fixed order: reproducible);
//   k_mlp_adam    sums the chunk partials in chunk order and applies Adam.
#include "mcdc_runtime.hpp"

namespace mcdc {

constexpr int kMlpChunks = 32;

__host__ __device__ inline int mlp_np(int in_dim) { return kH * in_dim + kH + kH * kH + kH + kH + 1; }

struct MlpScratch {
    float *h1, *h2, *dz1, *dz2, *dout;     // [n][64] x4, [n]
    float *partial;                        // [kMlpChunks][np]
    float *wsum;                           // [1]
};

static size_t mlp_scratch_floats(size_t n, int in_dim) {
    return 4 * n * kH + n + (size_t)kMlpChunks * mlp_np(in_dim) + 64;
}

static MlpScratch carve(float *base, size_t n, int in_dim) {
    MlpScratch s;
    s.h1 = base;
    s.h2 = s.h1 + n * kH;
    s.dz1 = s.h2 + n * kH;
    s.dz2 = s.dz1 + n * kH;
    s.dout = s.dz2 + n * kH;
    s.partial = s.dout + n;
    s.wsum = s.partial + (size_t)kMlpChunks * mlp_np(in_dim);
    return s;
}

// Forward (and, when y != nullptr, the per-point backward quantities).
template <bool BWD>
__global__ void __launch_bounds__(256) k_mlp_point(const float *__restrict__ prm, int in_dim,
                                                   const float *__restrict__ X,
                                                   const float *__restrict__ y,
                                                   const float *__restrict__ wt, size_t n,
                                                   float *__restrict__ out, MlpScratch S,
                                                   float *__restrict__ loss) {
    extern __shared__ float s_prm[];
    const int np = mlp_np(in_dim);
    for (int i = threadIdx.x; i < np; i += blockDim.x) s_prm[i] = prm[i];
    __syncthreads();
    const float *W1 = s_prm;
    const float *b1 = W1 + kH * in_dim;
    const float *W2 = b1 + kH;
    const float *b2 = W2 + kH * kH;
    const float *W3 = b2 + kH;
    const float b3 = W3[kH];
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    float lterm = 0.0f;
    if (p < n) {
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
            if (BWD) S.h2[p * kH + j] = h2;
            o = o + W3[j] * h2;
        }
        if (out) out[p] = o;
        if (BWD) {
#pragma unroll
            for (int i = 0; i < kH; ++i) S.h1[p * kH + i] = h1[i];
            const float inv = 1.0f / S.wsum[0];
            const float r = o - y[p];
            lterm = wt[p] * r * r * inv;
            const float dout = 2.0f * wt[p] * r * inv;
            S.dout[p] = dout;
            float dh1[kH];
#pragma unroll
            for (int i = 0; i < kH; ++i) dh1[i] = 0.0f;
            for (int j = 0; j < kH; ++j) {
                const float h2 = S.h2[p * kH + j];
                const float dz2 = h2 > 0.0f ? dout * W3[j] : 0.0f;
                S.dz2[p * kH + j] = dz2;
#pragma unroll
                for (int i = 0; i < kH; ++i) dh1[i] = dh1[i] + dz2 * W2[j * kH + i];
            }
#pragma unroll
            for (int i = 0; i < kH; ++i) S.dz1[p * kH + i] = h1[i] > 0.0f ? dh1[i] : 0.0f;
        }
    }
    if (BWD && loss) {
        // wave reduction, then one atomic per wave
        for (int off = 32; off > 0; off >>= 1) lterm += __shfl_xor(lterm, off);
        if ((threadIdx.x & 63) == 0 && lterm != 0.0f) atomicAdd(loss, lterm);
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

// partial[c][q] = sum over points of chunk c of dL/dparam_q (point order)
__global__ void __launch_bounds__(256) k_mlp_partial(int in_dim, const float *__restrict__ X,
                                                     size_t n, MlpScratch S) {
    const int np = mlp_np(in_dim);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (q >= np) return;
    const size_t per = (n + kMlpChunks - 1) / kMlpChunks;
    const size_t p0 = (size_t)c * per;
    const size_t p1 = p0 + per < n ? p0 + per : n;
    float acc = 0.0f;
    const int oW1 = 0, ob1 = kH * in_dim, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH;
    if (q < ob1) {
        const int i = q / in_dim, k = q % in_dim;
        for (size_t p = p0; p < p1; ++p) acc += S.dz1[p * kH + i] * X[p * in_dim + k];
    } else if (q < oW2) {
        const int i = q - ob1;
        for (size_t p = p0; p < p1; ++p) acc += S.dz1[p * kH + i];
    } else if (q < ob2) {
        const int j = (q - oW2) / kH, i = (q - oW2) % kH;
        for (size_t p = p0; p < p1; ++p) acc += S.dz2[p * kH + j] * S.h1[p * kH + i];
    } else if (q < oW3) {
        const int j = q - ob2;
        for (size_t p = p0; p < p1; ++p) acc += S.dz2[p * kH + j];
    } else if (q < ob3) {
        const int j = q - oW3;
        for (size_t p = p0; p < p1; ++p) acc += S.dout[p] * S.h2[p * kH + j];
    } else {
        for (size_t p = p0; p < p1; ++p) acc += S.dout[p];
    }
    (void)oW1;
    S.partial[(size_t)c * np + q] = acc;
}

// gradient = sum of chunk partials (chunk order); optional Adam update
__global__ void k_mlp_adam(int np, MlpScratch S, float *__restrict__ grad, float *__restrict__ prm,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                           float b2, float eps, float c1, float c2, int do_adam) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    float g = 0.0f;
    for (int c = 0; c < kMlpChunks; ++c) g += S.partial[(size_t)c * np + q];
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
    const int np = mlp_np(in_dim);
    const int block = 256;
    const int grid = (int)((n + block - 1) / block);
    hipLaunchKernelGGL((k_mlp_point<true>), dim3(grid), dim3(block), np * sizeof(float), s, prm,
                       in_dim, X, y, wt, n, (float *)nullptr, S, loss);
    hipLaunchKernelGGL(k_mlp_partial, dim3((np + block - 1) / block, kMlpChunks), dim3(block), 0, s,
                       in_dim, X, n, S);
    return hipGetLastError();
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
    MlpScratch S{};
    hipLaunchKernelGGL((k_mlp_point<false>), dim3((n + block - 1) / block), dim3(block),
                       mlp_np(in_dim) * sizeof(float), (hipStream_t)stream, prm, in_dim, X,
                       (const float *)nullptr, (const float *)nullptr, n, out, S, (float *)nullptr);
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
    hipStream_t s = (hipStream_t)stream;
    MlpScratch S = carve((float *)scratch, n, in_dim);
    hipError_t e = hipSuccess;
    if (loss_hist && o->steps > 0) e = hipMemsetAsync(loss_hist, 0, o->steps * sizeof(float), s);
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
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp_train");
}

}  // extern "C"
