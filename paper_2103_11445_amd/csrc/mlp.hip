// mlp.hip -- the learned cost model of the rewrite policy: a 6 -> 64 -> 64 -> 1
// perceptron in FP32 (tanh hidden layers, linear output), its forward pass,
// the gradient of the mean squared error, and Adam updates, on gfx950.
//
// The paper chooses the rows to rewrite by hand (Sec. IV-V); this model
// predicts the time of one executed level of a rewritten schedule from its
// shape, and the LEARNED policy absorbs a level into the current stage when
// the predicted cost of the merged stage beats opening a new one.
//
// Parameter vector (kParams floats): W1[64][6], b1[64], W2[64][64], b2[64],
// w3[64], b3.  Inputs x[m][6], row-major.
//
// The layers are 6x64 and 64x64 per sample: too small to pay for matrix
// cores at the batch sizes used (a training minibatch is a few thousand
// samples), so every kernel is plain FP32 vector code with the weights in
// LDS, read as broadcasts.  Sums run in a fixed order (no atomics), so the
// gradient is deterministic.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>

#include "sptrsv.h"

namespace {

constexpr int kIn = 6, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;
static_assert(kParams == 4673, "parameter layout");
constexpr int kBlock = 256;
constexpr int kChunk = 256;  // samples per partial-gradient block
constexpr int kSub = 32;     // samples staged in LDS at a time

__device__ inline void load_params(const float *__restrict__ p, float *w) {
    for (int q = threadIdx.x; q < kParams; q += blockDim.x) w[q] = p[q];
    __syncthreads();
}

// Hidden activations of one sample.
__device__ inline void hidden1(const float *w, const float *x, float *h1) {
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float z = w[oB1 + i];
#pragma unroll
        for (int k = 0; k < kIn; ++k) z = fmaf(w[oW1 + i * kIn + k], x[k], z);
        h1[i] = tanhf(z);
    }
}

__device__ inline float hidden2(const float *w, const float *h1, int j) {
    float z = w[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) z = fmaf(w[oW2 + j * kH + i], h1[i], z);
    return tanhf(z);
}

__global__ void __launch_bounds__(kBlock) mlp_forward(const float *__restrict__ params, const float *__restrict__ X,
                                                     float *__restrict__ Y, int32_t m) {
    __shared__ float w[kParams];
    load_params(params, w);
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= m) return;
    float x[kIn], h1[kH];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = X[(size_t)s * kIn + k];
    hidden1(w, x, h1);
    float y = w[oB3];
    for (int j = 0; j < kH; ++j) y = fmaf(w[oW3 + j], hidden2(w, h1, j), y);
    Y[s] = y;
}

// Workspace of the gradient (feature-major, m samples):
//   H1[64][m], H2[64][m], D1[64][m], D2[64][m], G[m], E[m], partial[nchunks][kParams + 1]
struct GradWs {
    float *h1, *h2, *d1, *d2, *g, *e, *part;
};

__host__ __device__ inline GradWs grad_ws(void *base, int32_t m) {
    float *f = static_cast<float *>(base);
    GradWs w;
    w.h1 = f;
    w.h2 = w.h1 + (size_t)kH * m;
    w.d1 = w.h2 + (size_t)kH * m;
    w.d2 = w.d1 + (size_t)kH * m;
    w.g = w.d2 + (size_t)kH * m;
    w.e = w.g + m;
    w.part = w.e + m;
    return w;
}

// Per sample: activations, output error and the back-propagated deltas
//   g = 2 (y - t) / m,  d2_j = g w3_j (1 - h2_j^2),  d1_i = (1 - h1_i^2) sum_j W2_ji d2_j.
__global__ void __launch_bounds__(kBlock) mlp_backprop(const float *__restrict__ params, const float *__restrict__ X,
                                                      const float *__restrict__ T, int32_t m, GradWs ws) {
    __shared__ float w[kParams];
    load_params(params, w);
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= m) return;
    float x[kIn], h1[kH], d2[kH];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = X[(size_t)s * kIn + k];
    hidden1(w, x, h1);
    float y = w[oB3];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        const float h2 = hidden2(w, h1, j);
        ws.h2[(size_t)j * m + s] = h2;
        d2[j] = h2;
        y = fmaf(w[oW3 + j], h2, y);
    }
    const float err = y - T[s];
    const float g = 2.0f * err / (float)m;
    ws.g[s] = g;
    ws.e[s] = err * err;
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        d2[j] = g * w[oW3 + j] * (1.0f - d2[j] * d2[j]);
        ws.d2[(size_t)j * m + s] = d2[j];
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc = fmaf(w[oW2 + j * kH + i], d2[j], acc);
        ws.h1[(size_t)i * m + s] = h1[i];
        ws.d1[(size_t)i * m + s] = (1.0f - h1[i] * h1[i]) * acc;
    }
}

// Partial sums over one chunk of kChunk samples of every parameter's
// gradient (and of the squared errors, at index kParams).  Thread t owns 16
// entries of dW2 (row t/4, columns (t%4)*16 ..) and up to three of the 577
// other parameters.
__global__ void __launch_bounds__(kBlock) mlp_grad_partial(const float *__restrict__ X, int32_t m, GradWs ws) {
    __shared__ float sh1[kSub][kH], sh2[kSub][kH], sd1[kSub][kH], sd2[kSub][kH];
    __shared__ float sx[kSub][kIn], sg[kSub], se[kSub], sone[kSub];
    const int t = threadIdx.x;
    const int j = t >> 2, i0 = (t & 3) * 16;
    float acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0f;
    // The other parameters -- W1 (384), b1 (64), b2 (64), w3 (64), b3 (1) --
    // and the squared errors: each a sum over samples of a product of two
    // staged columns (A at stride sa, B at stride sb; B = ones for biases).
    constexpr int kOther = kH * kIn + kH + kH + kH + 1 + 1;
    const float *pa[3], *pb[3];
    int sa[3], sb[3], dst[3];
    float oacc[3];
    for (int v = 0; v < 3; ++v) {
        const int e = t + v * kBlock;
        oacc[v] = 0.0f;
        sb[v] = 1;
        pb[v] = sone;
        if (e < kH * kIn) {
            pa[v] = &sd1[0][e / kIn], sa[v] = kH, pb[v] = &sx[0][e % kIn], sb[v] = kIn, dst[v] = oW1 + e;
        } else if (e < kH * kIn + kH) {
            pa[v] = &sd1[0][e - kH * kIn], sa[v] = kH, dst[v] = oB1 + e - kH * kIn;
        } else if (e < kH * kIn + 2 * kH) {
            pa[v] = &sd2[0][e - kH * kIn - kH], sa[v] = kH, dst[v] = oB2 + e - kH * kIn - kH;
        } else if (e < kH * kIn + 3 * kH) {
            pa[v] = &sh2[0][e - kH * kIn - 2 * kH], sa[v] = kH, pb[v] = sg, dst[v] = oW3 + e - kH * kIn - 2 * kH;
        } else if (e < kH * kIn + 3 * kH + 1) {
            pa[v] = sg, sa[v] = 1, dst[v] = oB3;
        } else {
            pa[v] = se, sa[v] = 1, dst[v] = kParams;  // squared errors
        }
    }
    if (t < kSub) sone[t] = 1.0f;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    const int64_t c1 = c0 + kChunk < m ? c0 + kChunk : m;
    for (int64_t s0 = c0; s0 < c1; s0 += kSub) {
        const int cnt = (int)(c1 - s0 < kSub ? c1 - s0 : kSub);
        for (int q = t; q < kSub * kH; q += kBlock) {
            const int r = q / kH, f = q % kH;
            const bool ok = r < cnt;
            const size_t idx = (size_t)f * m + (size_t)(s0 + (ok ? r : 0));
            sh1[r][f] = ok ? ws.h1[idx] : 0.0f;
            sh2[r][f] = ok ? ws.h2[idx] : 0.0f;
            sd1[r][f] = ok ? ws.d1[idx] : 0.0f;
            sd2[r][f] = ok ? ws.d2[idx] : 0.0f;
        }
        for (int q = t; q < kSub * kIn; q += kBlock) {
            const int r = q / kIn, k = q % kIn;
            sx[r][k] = r < cnt ? X[(size_t)(s0 + r) * kIn + k] : 0.0f;
        }
        if (t < kSub) {
            sg[t] = t < cnt ? ws.g[s0 + t] : 0.0f;
            se[t] = t < cnt ? ws.e[s0 + t] : 0.0f;
        }
        __syncthreads();
        for (int r = 0; r < kSub; ++r) {
            const float d = sd2[r][j];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = fmaf(d, sh1[r][i0 + u], acc[u]);
        }
#pragma unroll 1
        for (int v = 0; v < 3; ++v) {
            if (t + v * kBlock >= kOther) break;
            float a = oacc[v];
            for (int r = 0; r < kSub; ++r) a = fmaf(pa[v][r * sa[v]], pb[v][r * sb[v]], a);
            oacc[v] = a;
        }
        __syncthreads();
    }
    float *out = ws.part + (size_t)blockIdx.x * (kParams + 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) out[oW2 + j * kH + i0 + u] = acc[u];
    for (int v = 0; v < 3; ++v)
        if (t + v * kBlock < kOther) out[dst[v]] = oacc[v];
}

// grad[p] = sum over chunks in order; loss = (sum of squared errors) / m.
__global__ void __launch_bounds__(kBlock) mlp_grad_reduce(const float *__restrict__ part, int32_t nchunks, int32_t m,
                                                         float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p > kParams) return;
    float a = 0.0f;
    for (int c = 0; c < nchunks; ++c) a += part[(size_t)c * (kParams + 1) + p];
    if (p < kParams) grad[p] = a;
    else if (loss) *loss = a / (float)m;
}

// Adam (Kingma and Ba, 2015) with bias-corrected moments.
__global__ void __launch_bounds__(kBlock) mlp_adam(float *__restrict__ params, const float *__restrict__ grad,
                                                  float *__restrict__ m1, float *__restrict__ m2, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float a = beta1 * m1[p] + (1.0f - beta1) * g;
    const float b = beta2 * m2[p] + (1.0f - beta2) * g * g;
    m1[p] = a;
    m2[p] = b;
    params[p] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

int blocks_for(int64_t count) { return (int)((count + kBlock - 1) / kBlock); }

}  // namespace

namespace {

// ---- workspace without allocation ----------------------------------------
//
// For callers that cannot allocate device memory: the gradient's workspace
// for up to SPTRSV_MLP_NOALLOC_MAX_SAMPLES samples as a file-scope device
// array.  Each GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, not the device
// copy: the device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels.  Every
// word of the workspace is written by the gradient's kernels before it is
// read, so nothing needs clearing between calls; calls that overlap on one
// GPU share the array and race.
constexpr int32_t kStaticSamples = SPTRSV_MLP_NOALLOC_MAX_SAMPLES;
constexpr size_t kStaticBytes =
    sizeof(float) * ((size_t)(4 * kH + 2) * kStaticSamples +
                     ((size_t)kStaticSamples + kChunk - 1) / kChunk * (kParams + 1));
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (guarded by g_scratch_mu)

}  // namespace

extern "C" int sptrsv_mlp_static_workspace(void **ptr, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *ptr = g_scratch_dev[dev];
    *bytes = kStaticBytes;
    return 0;
}

extern "C" size_t sptrsv_launch_mlp_workspace(int32_t m) {
    const size_t nchunks = ((size_t)m + kChunk - 1) / kChunk;
    return sizeof(float) * ((size_t)(4 * kH + 2) * (size_t)m + nchunks * (kParams + 1));
}

extern "C" int sptrsv_launch_mlp_forward(const float *params, const float *X, float *Y, int32_t m, void *stream) {
    hipLaunchKernelGGL(mlp_forward, dim3(blocks_for(m)), dim3(kBlock), 0, static_cast<hipStream_t>(stream), params,
                       X, Y, m);
    return (int)hipGetLastError();
}

extern "C" int sptrsv_launch_mlp_grad(const float *params, const float *X, const float *T, int32_t m, float *grad,
                                      float *loss, void *workspace, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const GradWs ws = grad_ws(workspace, m);
    const int nchunks = (int)(((int64_t)m + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(mlp_backprop, dim3(blocks_for(m)), dim3(kBlock), 0, s, params, X, T, m, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(mlp_grad_partial, dim3(nchunks), dim3(kBlock), 0, s, X, m, ws);
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    hipLaunchKernelGGL(mlp_grad_reduce, dim3(blocks_for(kParams + 1)), dim3(kBlock), 0, s, ws.part, nchunks, m,
                       grad, loss);
    return (int)hipGetLastError();
}

extern "C" int sptrsv_launch_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t step,
                                      float lr, float beta1, float beta2, float eps, void *stream) {
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam, dim3(blocks_for(kParams)), dim3(kBlock), 0, static_cast<hipStream_t>(stream), params,
                       grad, m1, m2, lr, beta1, beta2, eps, c1, c2);
    return (int)hipGetLastError();
}
