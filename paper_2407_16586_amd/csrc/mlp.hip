// Training and evaluation kernels of the quartet-contribution estimator (mlp.hpp):
// BF16 matrix-core forward and backward passes with FP32 accumulation, FP32 master
// weights and an Adam update, and the model's C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/tdgrad.h"
#include "mlp.hpp"

using namespace tdg;

extern "C" int tdg_set_error_(int code, const char *msg); // defined in tdgrad.hip

#define HIPM_TRY(expr)                                                                                 \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return tdg_set_error_(TDG_EDEVICE, hipGetErrorString(e_));               \
    } while (0)

struct tdg_mlp {
    int device = 0;
    float *w = nullptr;      // FP32 master weights [MLP_NW]
    float *m = nullptr, *v = nullptr, *g = nullptr; // Adam moments and gradient accumulator
    uint16_t *w1b = nullptr, *w2b = nullptr;        // BF16 copies of W1, W2
    float *loss = nullptr;   // accumulated loss of the last step
    long long steps = 0;
};

__global__ void k_mlp_to_bf16(const float *w, uint16_t *w1b, uint16_t *w2b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_H * MLP_IN) w1b[i] = f2bf(w[MLP_W1 + i]);
    if (i < MLP_H * MLP_H) w2b[i] = f2bf(w[MLP_W2 + i]);
}

// forward of n samples (X [n][16] FP32), one wavefront per 64 samples
__global__ void __launch_bounds__(256) k_mlp_forward(const float *w, const uint16_t *w1b, const uint16_t *w2b,
                                                     const float *X, long long n, float *out)
{
    __shared__ MlpShared S;
    __shared__ MlpWave W[4];
    mlp_load_shared(S, w1b, w2b, w);
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const long long s = ((long long)blockIdx.x * 4 + wave) * 64 + lane;
    float x[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = s < n ? X[s * MLP_IN + i] : 0.f;
    const float y = mlp_forward_wave(S, W[wave], x, lane);
    if (s < n) out[s] = y;
}

// loss = mean (pred - y)^2 over the n samples; gradient summed into g.  One wavefront per
// block; a block takes tiles of 64 samples at a grid stride and keeps its partial gradient in
// registers (each lane holds the matrix-core output elements it produces, and the bias and
// output-layer sums of its column), so that it adds into g once at the end instead of once
// per tile.  The layer inputs are rounded to BF16 exactly where the forward pass rounds them.
__global__ void __launch_bounds__(64) k_mlp_grad(const float *w, const uint16_t *w1b, const uint16_t *w2b,
                                                 const float *X, const float *Y, long long n, float *g, float *loss)
{
    __shared__ MlpShared S;
    __shared__ uint16_t x[64 * MLP_IN], h1[64 * MLP_H], d2[64 * MLP_H], d1[64 * MLP_H];
    __shared__ float h2[64 * MLP_H], dout[64];
    mlp_load_shared(S, w1b, w2b, w);
    const int lane = threadIdx.x;
    const int kq = 4 * (lane >> 4), col = lane & 15;
    static_assert(MLP_H == 64, "one hidden unit per lane in the bias and output-layer sums");
    float a_w2[4][4][4], a_w1[4][4], a_w3 = 0.f, a_b2 = 0.f, a_b1 = 0.f, a_b3 = 0.f, a_loss = 0.f;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a_w1[mi][t] = 0.f;
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) a_w2[mi][ni][t] = 0.f;
        }
    for (long long t0 = (long long)blockIdx.x * 64; t0 < n; t0 += (long long)gridDim.x * 64) {
        __syncthreads(); // the previous tile's reads of x, h1, d1, d2 are done (and S is loaded)
        const long long s = t0 + lane;
        const bool ok = s < n;
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) x[lane * MLP_IN + i] = f2bf(ok ? X[s * MLP_IN + i] : 0.f);
        __syncthreads();
        for (int mi = 0; mi < 4; ++mi)
            for (int ni = 0; ni < 4; ++ni) {
                f32x4 d = mfma_tile([&](int m, int k) { return x[m * MLP_IN + k]; },
                                    [&](int k, int nn) { return S.w1[nn * MLP_IN + k]; }, 16 * mi, 16 * ni, 1, lane);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int m = 16 * mi + kq + t, nn = 16 * ni + col;
                    const float z = d[t] + S.b1[nn];
                    h1[m * MLP_H + nn] = f2bf(z > 0.f ? z : 0.f);
                }
            }
        __syncthreads();
        for (int mi = 0; mi < 4; ++mi)
            for (int ni = 0; ni < 4; ++ni) {
                f32x4 d = mfma_tile([&](int m, int k) { return h1[m * MLP_H + k]; },
                                    [&](int k, int nn) { return S.w2[nn * MLP_H + k]; }, 16 * mi, 16 * ni, 4, lane);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int m = 16 * mi + kq + t, nn = 16 * ni + col;
                    const float z = d[t] + S.b2[nn];
                    h2[m * MLP_H + nn] = z > 0.f ? z : 0.f;
                }
            }
        __syncthreads();
        // output, loss and d loss / d out
        float o = S.b3;
        for (int c = 0; c < MLP_H; ++c) o += h2[lane * MLP_H + c] * S.w3[c];
        const float e = ok ? o - Y[s] : 0.f;
        dout[lane] = 2.f * e / (float)n;
        a_loss += e * e / (float)n;
        __syncthreads();
        // layer 3 and dz2 (hidden unit c = lane)
        {
            const int c = lane;
            float gw3 = 0.f, gb2 = 0.f;
            for (int k = 0; k < 64; ++k) {
                const float hv = h2[k * MLP_H + c];
                gw3 += dout[k] * hv;
                const float dz = hv > 0.f ? dout[k] * S.w3[c] : 0.f;
                d2[k * MLP_H + c] = f2bf(dz);
                gb2 += dz;
            }
            a_w3 += gw3;
            a_b2 += gb2;
        }
        if (lane == 0) {
            float gb3 = 0.f;
            for (int k = 0; k < 64; ++k) gb3 += dout[k];
            a_b3 += gb3;
        }
        __syncthreads();
        // dW2[n][k] = sum_s dz2[s][n] h1[s][k];  dh1[s][k] = sum_n dz2[s][n] W2[n][k]
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                f32x4 d = mfma_tile([&](int m, int k) { return d2[k * MLP_H + m]; },
                                    [&](int k, int nn) { return h1[k * MLP_H + nn]; }, 16 * mi, 16 * ni, 4, lane);
#pragma unroll
                for (int t = 0; t < 4; ++t) a_w2[mi][ni][t] += d[t];
                f32x4 e2 = mfma_tile([&](int m, int k) { return d2[m * MLP_H + k]; },
                                     [&](int k, int nn) { return S.w2[k * MLP_H + nn]; }, 16 * mi, 16 * ni, 4, lane);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int m = 16 * mi + kq + t, nn = 16 * ni + col;
                    d1[m * MLP_H + nn] = f2bf(h1[m * MLP_H + nn] != 0 ? e2[t] : 0.f);
                }
            }
        __syncthreads();
        {
            float gb1 = 0.f;
            for (int k = 0; k < 64; ++k) gb1 += bf2f(d1[k * MLP_H + lane]);
            a_b1 += gb1;
        }
        // dW1[n][i] = sum_s dz1[s][n] x[s][i]
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            f32x4 d = mfma_tile([&](int m, int k) { return d1[k * MLP_H + m]; },
                                [&](int k, int nn) { return x[k * MLP_IN + nn]; }, 16 * mi, 0, 4, lane);
#pragma unroll
            for (int t = 0; t < 4; ++t) a_w1[mi][t] += d[t];
        }
    }
    // one addition per gradient element and block
    for (int off = 32; off > 0; off >>= 1) a_loss += __shfl_xor(a_loss, off);
    if (lane == 0) {
        atomicAdd(loss, a_loss);
        atomicAdd(&g[MLP_B3], a_b3);
    }
    atomicAdd(&g[MLP_W3 + lane], a_w3);
    atomicAdd(&g[MLP_B2 + lane], a_b2);
    atomicAdd(&g[MLP_B1 + lane], a_b1);
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            atomicAdd(&g[MLP_W1 + (16 * mi + kq + t) * MLP_IN + col], a_w1[mi][t]);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                atomicAdd(&g[MLP_W2 + (16 * mi + kq + t) * MLP_H + 16 * ni + col], a_w2[mi][ni][t]);
        }
}

// blocks of the gradient launch: one per 64-sample tile up to 1024 (tiles beyond that are
// taken at a grid stride)
static unsigned mlp_grad_blocks(long long n)
{
    const long long tiles = (n + 63) / 64;
    return (unsigned)(tiles < 1024 ? (tiles > 0 ? tiles : 1) : 1024);
}

__global__ void k_mlp_adam(float *w, float *m, float *v, float *g, uint16_t *w1b, uint16_t *w2b, float lr, float b1,
                           float b2, float eps, float c1, float c2, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    g[i] = 0.f;
    if (i >= MLP_W1 && i < MLP_W1 + MLP_H * MLP_IN) w1b[i - MLP_W1] = f2bf(wi);
    if (i >= MLP_W2 && i < MLP_W2 + MLP_H * MLP_H) w2b[i - MLP_W2] = f2bf(wi);
}

__global__ void k_fill(float *p, int n, float v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

int tdg_mlp_create(int device, uint64_t seed, tdg_mlp_t **out)
{
    if (!out) return tdg_set_error_(TDG_EINVAL, "null output");
    *out = nullptr;
    HIPM_TRY(hipSetDevice(device));
    tdg_mlp *m = new (std::nothrow) tdg_mlp();
    if (!m) return tdg_set_error_(TDG_ENOMEM, "host allocation failed");
    m->device = device;
    size_t f = sizeof(float) * MLP_NW;
    if (hipMalloc((void **)&m->w, f) != hipSuccess || hipMalloc((void **)&m->m, f) != hipSuccess ||
        hipMalloc((void **)&m->v, f) != hipSuccess || hipMalloc((void **)&m->g, f) != hipSuccess ||
        hipMalloc((void **)&m->w1b, 2 * MLP_H * MLP_IN) != hipSuccess ||
        hipMalloc((void **)&m->w2b, 2 * MLP_H * MLP_H) != hipSuccess || hipMalloc((void **)&m->loss, 4) != hipSuccess) {
        tdg_mlp_destroy(m);
        return tdg_set_error_(TDG_ENOMEM, "device allocation failed");
    }
    // He-style initialisation (uniform, seeded), zero biases
    std::mt19937_64 rng(seed);
    std::vector<float> w(MLP_NW, 0.f);
    auto fillu = [&](int off, int cnt, float a) {
        std::uniform_real_distribution<float> U(-a, a);
        for (int i = 0; i < cnt; ++i) w[off + i] = U(rng);
    };
    fillu(MLP_W1, MLP_H * MLP_IN, std::sqrt(6.f / 10.f));
    fillu(MLP_W2, MLP_H * MLP_H, std::sqrt(6.f / MLP_H));
    fillu(MLP_W3, MLP_H, std::sqrt(3.f / MLP_H));
    for (int k = 10; k < MLP_IN; ++k)
        for (int o = 0; o < MLP_H; ++o) w[MLP_W1 + o * MLP_IN + k] = 0.f; // padding inputs
    *out = m;
    return tdg_mlp_set_weights(m, w.data());
}

int tdg_mlp_destroy(tdg_mlp_t *m)
{
    if (!m) return TDG_OK;
    hipSetDevice(m->device);
    for (void *p : {(void *)m->w, (void *)m->m, (void *)m->v, (void *)m->g, (void *)m->w1b, (void *)m->w2b,
                    (void *)m->loss})
        if (p) hipFree(p);
    delete m;
    return TDG_OK;
}

int tdg_mlp_set_weights(tdg_mlp_t *m, const float *w)
{
    if (!m || !w) return tdg_set_error_(TDG_EINVAL, "null argument");
    HIPM_TRY(hipSetDevice(m->device));
    HIPM_TRY(hipMemcpy(m->w, w, sizeof(float) * MLP_NW, hipMemcpyHostToDevice));
    HIPM_TRY(hipMemset(m->m, 0, sizeof(float) * MLP_NW));
    HIPM_TRY(hipMemset(m->v, 0, sizeof(float) * MLP_NW));
    HIPM_TRY(hipMemset(m->g, 0, sizeof(float) * MLP_NW));
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((MLP_H * MLP_H + 255) / 256), dim3(256), 0, 0, m->w, m->w1b, m->w2b);
    HIPM_TRY(hipGetLastError());
    HIPM_TRY(hipDeviceSynchronize());
    m->steps = 0;
    return TDG_OK;
}

int tdg_mlp_get_weights(const tdg_mlp_t *m, float *w)
{
    if (!m || !w) return tdg_set_error_(TDG_EINVAL, "null argument");
    HIPM_TRY(hipSetDevice(m->device));
    HIPM_TRY(hipMemcpy(w, m->w, sizeof(float) * MLP_NW, hipMemcpyDeviceToHost));
    return TDG_OK;
}

int tdg_mlp_forward(const tdg_mlp_t *m, const float *X, int64_t n, float *out, void *stream)
{
    if (!m || (!X && n) || (!out && n) || n < 0) return tdg_set_error_(TDG_EINVAL, "bad arguments");
    if (!n) return TDG_OK;
    HIPM_TRY(hipSetDevice(m->device));
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, m->w, m->w1b,
                       m->w2b, X, (long long)n, out);
    HIPM_TRY(hipGetLastError());
    return TDG_OK;
}

int tdg_mlp_grad(tdg_mlp_t *m, const float *X, const float *Y, int64_t n, float *grad_out, float *loss_out,
                 void *stream)
{
    if (!m || !X || !Y || n <= 0) return tdg_set_error_(TDG_EINVAL, "bad arguments");
    HIPM_TRY(hipSetDevice(m->device));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, m->loss, 1, 0.f);
    hipLaunchKernelGGL(k_mlp_grad, dim3(mlp_grad_blocks(n)), dim3(64), 0, st, m->w, m->w1b, m->w2b, X, Y,
                       (long long)n, m->g, m->loss);
    HIPM_TRY(hipGetLastError());
    if (grad_out) {
        HIPM_TRY(hipMemcpyAsync(grad_out, m->g, sizeof(float) * MLP_NW, hipMemcpyDeviceToHost, st));
        hipLaunchKernelGGL(k_fill, dim3((MLP_NW + 255) / 256), dim3(256), 0, st, m->g, MLP_NW, 0.f);
    }
    if (loss_out) HIPM_TRY(hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    if (grad_out || loss_out) HIPM_TRY(hipStreamSynchronize(st));
    return TDG_OK;
}

int tdg_mlp_train_step(tdg_mlp_t *m, const float *X, const float *Y, int64_t n, float lr, float *loss_out,
                       void *stream)
{
    if (!m || !X || !Y || n <= 0 || !(lr > 0.f)) return tdg_set_error_(TDG_EINVAL, "bad arguments");
    HIPM_TRY(hipSetDevice(m->device));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, m->loss, 1, 0.f);
    hipLaunchKernelGGL(k_mlp_grad, dim3(mlp_grad_blocks(n)), dim3(64), 0, st, m->w, m->w1b, m->w2b, X, Y,
                       (long long)n, m->g, m->loss);
    m->steps += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->steps), c2 = 1.f - std::pow(b2, (float)m->steps);
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NW + 255) / 256), dim3(256), 0, st, m->w, m->m, m->v, m->g, m->w1b,
                       m->w2b, lr, b1, b2, 1e-8f, c1, c2, MLP_NW);
    HIPM_TRY(hipGetLastError());
    if (loss_out) {
        HIPM_TRY(hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToHost, st));
        HIPM_TRY(hipStreamSynchronize(st));
    }
    return TDG_OK;
}

int tdg_mlp_nweights(void) { return MLP_NW; }

} // extern "C"

// device access for the screening filter (same library)
namespace tdg {
void mlp_device_ptrs(const tdg_mlp *m, const float **w, const uint16_t **w1b, const uint16_t **w2b)
{
    *w = m->w;
    *w1b = m->w1b;
    *w2b = m->w2b;
}
} // namespace tdg
