// HIP kernels of the parameter predictor (include/hdc_mlp.h): a strided tiled
// FP32 product for the forward and both backward products of a linear layer,
// column sums for bias gradients, fused softmax / cross-entropy, relu backward
// and Adam.  Sizes are small (rows <= a few thousand, widths <= 128), so a
// 16 x 16 LDS tiling is enough; every reduction has a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/hdc_mlp.h"
#include "hdc_internal.h"

namespace hdc {

constexpr int TS = 16;

// C[mi, ni] = sum_k A[mi*sam + k*sak] * Bm[k*sbk + ni*sbn] (+ bias[ni]) (relu)
__global__ void __launch_bounds__(256) k_gemm(const float* __restrict__ A, int64_t sam, int64_t sak,
                                             const float* __restrict__ Bm, int64_t sbk, int64_t sbn,
                                             float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                             const float* __restrict__ bias, int relu) {
    __shared__ float As[TS][TS + 1];
    __shared__ float Bs[TS][TS + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int mi = blockIdx.y * TS + ty;
    const int ni = blockIdx.x * TS + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += TS) {
        const int ka = k0 + tx;  // A tile: row ty of this block, column ka
        const int am = blockIdx.y * TS + ty;
        As[ty][tx] = (am < M && ka < K) ? A[am * sam + ka * sak] : 0.f;
        const int kb = k0 + ty;  // B tile: row kb, column tx of this block
        const int bn = blockIdx.x * TS + tx;
        Bs[ty][tx] = (kb < K && bn < N) ? Bm[kb * sbk + bn * sbn] : 0.f;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TS; ++kk) acc = fmaf(As[ty][kk], Bs[kk][tx], acc);
        __syncthreads();
    }
    if (mi < M && ni < N) {
        if (bias) acc += bias[ni];
        if (relu) acc = acc > 0.f ? acc : 0.f;
        C[mi * ldc + ni] = acc;
    }
}

// db[o] = sum_b dY[b, o]  (one thread per column, rows in order)
__global__ void k_colsum(const float* __restrict__ dY, float* __restrict__ db, int B, int Out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= Out) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dY[(int64_t)b * Out + o];
    db[o] = s;
}

__global__ void k_relu_bwd(float* __restrict__ dA, const float* __restrict__ A, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (!(A[i] > 0.f)) dA[i] = 0.f;
}

// One thread per row: P = softmax(Z) and dZ = (P - onehot) / B.
__global__ void k_softmax_xent(const float* __restrict__ Z, const int32_t* __restrict__ y, float* __restrict__ P,
                               float* __restrict__ dZ, int B, int K) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* z = Z + (int64_t)b * K;
    float mx = z[0];
    for (int k = 1; k < K; ++k) mx = fmaxf(mx, z[k]);
    float s = 0.f;
    for (int k = 0; k < K; ++k) s += expf(z[k] - mx);
    const float inv = 1.f / s;
    for (int k = 0; k < K; ++k) P[(int64_t)b * K + k] = expf(z[k] - mx) * inv;
    if (y) {
        const int lab = y[b];
        if (dZ) {
            const float invB = 1.f / (float)B;
            for (int k = 0; k < K; ++k)
                dZ[(int64_t)b * K + k] = (P[(int64_t)b * K + k] - (k == lab ? 1.f : 0.f)) * invB;
        }
    }
}

// loss = mean_b (logsumexp(Z_b) - Z_b[y_b]); one workgroup, fixed-order sums.
__global__ void __launch_bounds__(256) k_xent_mean(const float* __restrict__ Z, const int32_t* __restrict__ y,
                                                  float* __restrict__ out, int B, int K) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float* z = Z + (int64_t)b * K;
        float mx = z[0];
        for (int k = 1; k < K; ++k) mx = fmaxf(mx, z[k]);
        float e = 0.f;
        for (int k = 0; k < K; ++k) e += expf(z[k] - mx);
        s += logf(e) + mx - z[y[b]];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / (float)B;
}

// Soft targets: P = softmax(Z), dZ = (P - T) / B (one thread per row).
__global__ void k_softmax_soft(const float* __restrict__ Z, const float* __restrict__ T, float* __restrict__ P,
                               float* __restrict__ dZ, int B, int K) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* z = Z + (int64_t)b * K;
    float mx = z[0];
    for (int k = 1; k < K; ++k) mx = fmaxf(mx, z[k]);
    float s = 0.f;
    for (int k = 0; k < K; ++k) s += expf(z[k] - mx);
    const float inv = 1.f / s;
    const float invB = 1.f / (float)B;
    for (int k = 0; k < K; ++k) {
        const float pk = expf(z[k] - mx) * inv;
        P[(int64_t)b * K + k] = pk;
        if (dZ) dZ[(int64_t)b * K + k] = (pk - T[(int64_t)b * K + k]) * invB;
    }
}

// loss = mean_b sum_k -T[b,k] (Z[b,k] - logsumexp(Z_b)); one workgroup, fixed-order sums.
__global__ void __launch_bounds__(256) k_soft_mean(const float* __restrict__ Z, const float* __restrict__ T,
                                                  float* __restrict__ out, int B, int K) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float* z = Z + (int64_t)b * K;
        float mx = z[0];
        for (int k = 1; k < K; ++k) mx = fmaxf(mx, z[k]);
        float e = 0.f;
        for (int k = 0; k < K; ++k) e += expf(z[k] - mx);
        const float lse = logf(e) + mx;
        for (int k = 0; k < K; ++k) s += T[(int64_t)b * K + k] * (lse - z[k]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / (float)B;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

static hipError_t gemm(const float* A, int64_t sam, int64_t sak, const float* Bm, int64_t sbk, int64_t sbn, float* C,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, const float* bias, int relu, hipStream_t s) {
    dim3 grid((unsigned)((N + TS - 1) / TS), (unsigned)((M + TS - 1) / TS));
    hipLaunchKernelGGL(k_gemm, grid, dim3(TS, TS), 0, s, A, sam, sak, Bm, sbk, sbn, C, ldc, (int)M, (int)N, (int)K,
                       bias, relu);
    return hipGetLastError();
}

static unsigned blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace hdc

using namespace hdc;

static bool sizes_ok(int64_t a, int64_t b, int64_t c) {
    return a > 0 && b > 0 && c > 0 && a < (int64_t(1) << 30) && b < (int64_t(1) << 30) && c < (int64_t(1) << 30);
}

extern "C" {

hdc_status hdc_mlp_linear_forward(const float* X, const float* W, const float* b, float* Y, int64_t B, int64_t in,
                                  int64_t out, int relu, hipStream_t s) {
    if (!X || !W || !Y || !sizes_ok(B, in, out)) return set_error(HDC_ERR_INVALID_ARG, "mlp forward: bad arguments");
    hipError_t e = gemm(X, in, 1, W, 1, in, Y, out, B, out, in, b, relu, s);
    return e == hipSuccess ? HDC_OK : set_error(HDC_ERR_HIP, hipGetErrorString(e));
}

hdc_status hdc_mlp_linear_backward(const float* X, const float* W, const float* dY, float* dX, float* dW, float* db,
                                   int64_t B, int64_t in, int64_t out, hipStream_t s) {
    if (!X || !W || !dY || !dW || !db || !sizes_ok(B, in, out))
        return set_error(HDC_ERR_INVALID_ARG, "mlp backward: bad arguments");
    // dW[o, i] = sum_b dY[b, o] X[b, i]
    hipError_t e = gemm(dY, 1, out, X, in, 1, dW, in, out, in, B, nullptr, 0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colsum, dim3(blocks_for(out)), dim3(256), 0, s, dY, db, (int)B, (int)out);
        e = hipGetLastError();
    }
    // dX[b, i] = sum_o dY[b, o] W[o, i]
    if (e == hipSuccess && dX) e = gemm(dY, out, 1, W, in, 1, dX, in, B, in, out, nullptr, 0, s);
    return e == hipSuccess ? HDC_OK : set_error(HDC_ERR_HIP, hipGetErrorString(e));
}

hdc_status hdc_mlp_relu_backward(float* dA, const float* A, int64_t n, hipStream_t s) {
    if (!dA || !A || n <= 0) return set_error(HDC_ERR_INVALID_ARG, "mlp relu backward: bad arguments");
    hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(n)), dim3(256), 0, s, dA, A, n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HDC_OK : set_error(HDC_ERR_HIP, hipGetErrorString(e));
}

hdc_status hdc_mlp_softmax_xent(const float* Z, const int32_t* y, float* P, float* dZ, float* loss, int64_t B,
                                int64_t K, hipStream_t s) {
    if (!Z || !P || !sizes_ok(B, K, 1)) return set_error(HDC_ERR_INVALID_ARG, "mlp softmax: bad arguments");
    hipLaunchKernelGGL(k_softmax_xent, dim3(blocks_for(B)), dim3(256), 0, s, Z, y, P, dZ, (int)B, (int)K);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && y && loss) {
        hipLaunchKernelGGL(k_xent_mean, dim3(1), dim3(256), 0, s, Z, y, loss, (int)B, (int)K);
        e = hipGetLastError();
    }
    return e == hipSuccess ? HDC_OK : set_error(HDC_ERR_HIP, hipGetErrorString(e));
}

hdc_status hdc_mlp_softmax_xent_soft(const float* Z, const float* T, float* P, float* dZ, float* loss, int64_t B,
                                     int64_t K, hipStream_t s) {
    if (!Z || !T || !P || !sizes_ok(B, K, 1)) return set_error(HDC_ERR_INVALID_ARG, "mlp soft softmax: bad arguments");
    hipLaunchKernelGGL(k_softmax_soft, dim3(blocks_for(B)), dim3(256), 0, s, Z, T, P, dZ, (int)B, (int)K);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && loss) {
        hipLaunchKernelGGL(k_soft_mean, dim3(1), dim3(256), 0, s, Z, T, loss, (int)B, (int)K);
        e = hipGetLastError();
    }
    return e == hipSuccess ? HDC_OK : set_error(HDC_ERR_HIP, hipGetErrorString(e));
}

hdc_status hdc_mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                        float eps, int64_t t, hipStream_t s) {
    if (!p || !g || !m || !v || n <= 0 || t < 1) return set_error(HDC_ERR_INVALID_ARG, "mlp adam: bad arguments");
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)t));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HDC_OK : set_error(HDC_ERR_HIP, hipGetErrorString(e));
}

}  // extern "C"
