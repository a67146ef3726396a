// Quartet-contribution estimator: a 10 -> 64 -> 64 -> 1 ReLU network evaluated with
// BF16 matrix-core instructions (FP32 accumulation), 64 samples per wavefront.
//
// Weight layout (FP32 master copy, MLP_NW floats):
//   W1[64][16]  (out, in)   b1[64]   W2[64][64] (out, in)   b2[64]   W3[64]   b3
// The BF16 copies keep the same (out, in) layout, which is the B-operand layout the
// 16x16x16 instruction reads (4 consecutive inputs per lane).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdg {

constexpr int MLP_IN = 16, MLP_H = 64;
constexpr int MLP_W1 = 0, MLP_B1 = MLP_W1 + MLP_H * MLP_IN, MLP_W2 = MLP_B1 + MLP_H, MLP_B2 = MLP_W2 + MLP_H * MLP_H,
              MLP_W3 = MLP_B2 + MLP_H, MLP_B3 = MLP_W3 + MLP_H, MLP_NW = MLP_B3 + 1;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f)
{
    union { float f; uint32_t u; } x{f};
    const uint32_t lsb = (x.u >> 16) & 1u;
    return (uint16_t)((x.u + 0x7fffu + lsb) >> 16); // round to nearest even (finite inputs)
}
__host__ __device__ inline float bf2f(uint16_t h)
{
    union { uint32_t u; float f; } x{(uint32_t)h << 16};
    return x.f;
}

// One 16x16 tile of D = A * B with K = 16*ksteps; A(m, k) and B(k, n) return BF16 bits.
// Lane l supplies A[m0 + l%16][k0 + 4(l/16) + t] and B[k0 + 4(l/16) + t][n0 + l%16];
// on return acc[t] = D[m0 + 4(l/16) + t][n0 + l%16].
template <class FA, class FB>
__device__ __forceinline__ f32x4 mfma_tile(FA A, FB B, int m0, int n0, int ksteps, int lane)
{
    const int r = lane & 15, kq = 4 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ksteps; ++s) {
        const int k0 = 16 * s + kq;
        bf16x4 a, b;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[t] = (short)A(m0 + r, k0 + t);
            b[t] = (short)B(k0 + t, n0 + r);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Shared-memory image of the network for one block.
struct MlpShared {
    uint16_t w1[MLP_H * MLP_IN]; // [out][in]
    uint16_t w2[MLP_H * MLP_H];  // [out][in]
    float b1[MLP_H], b2[MLP_H], w3[MLP_H], b3;
};

// Per-wavefront scratch of the forward pass.
struct MlpWave {
    uint16_t x[64 * MLP_IN];  // [sample][in]
    uint16_t h1[64 * MLP_H];  // [sample][hidden], BF16 after ReLU
    float out[64];
};

__device__ inline void mlp_load_shared(MlpShared &s, const uint16_t *w1b, const uint16_t *w2b, const float *wf)
{
    for (int i = threadIdx.x; i < MLP_H * MLP_IN; i += blockDim.x) s.w1[i] = w1b[i];
    for (int i = threadIdx.x; i < MLP_H * MLP_H; i += blockDim.x) s.w2[i] = w2b[i];
    for (int i = threadIdx.x; i < MLP_H; i += blockDim.x) {
        s.b1[i] = wf[MLP_B1 + i];
        s.b2[i] = wf[MLP_B2 + i];
        s.w3[i] = wf[MLP_W3 + i];
    }
    if (threadIdx.x == 0) s.b3 = wf[MLP_B3];
}

// Forward pass of the wavefront's 64 samples: lane l supplies x (MLP_IN features of
// sample l) and receives its prediction.  Requires the whole wavefront active.
__device__ inline float mlp_forward_wave(const MlpShared &S, MlpWave &W, const float *x, int lane)
{
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) W.x[lane * MLP_IN + i] = f2bf(x[i]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int kq = 4 * (lane >> 4), col = lane & 15;
    // layer 1: [64 x 16] x [16 x 64]
    for (int mi = 0; mi < 4; ++mi)
        for (int ni = 0; ni < 4; ++ni) {
            f32x4 d = mfma_tile([&](int m, int k) { return W.x[m * MLP_IN + k]; },
                                [&](int k, int n) { return S.w1[n * MLP_IN + k]; }, 16 * mi, 16 * ni, 1, lane);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int m = 16 * mi + kq + t, n = 16 * ni + col;
                const float z = d[t] + S.b1[n];
                W.h1[m * MLP_H + n] = f2bf(z > 0.f ? z : 0.f);
            }
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 2 and the output row sums: lane holds rows 16 mi + kq + t, column 16 ni + col
    float part[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int t = 0; t < 4; ++t) part[mi][t] = 0.f;
    for (int mi = 0; mi < 4; ++mi)
        for (int ni = 0; ni < 4; ++ni) {
            f32x4 d = mfma_tile([&](int m, int k) { return W.h1[m * MLP_H + k]; },
                                [&](int k, int n) { return S.w2[n * MLP_H + k]; }, 16 * mi, 16 * ni, 4, lane);
            const int n = 16 * ni + col;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float z = d[t] + S.b2[n];
                part[mi][t] += (z > 0.f ? z : 0.f) * S.w3[n];
            }
        }
    // reduce over the 16 lanes sharing kq (columns)
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float v = part[mi][t];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
            if (col == 0) W.out[16 * mi + kq + t] = v + S.b3;
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return W.out[lane];
}

} // namespace tdg
