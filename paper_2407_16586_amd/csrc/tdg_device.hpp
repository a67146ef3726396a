// Device-side helpers shared by the tdgrad kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rys_table.inc"

namespace tdg {

constexpr int kWave = 64;

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Cartesian exponents of component i of a shell with angular momentum l,
// ordered lx descending then ly descending (x,y,z; xx,xy,xz,yy,yz,zz).
struct Cart {
    int v[3][6][3];
};
__host__ __device__ constexpr Cart make_cart()
{
    Cart c{};
    for (int l = 0; l <= 2; ++l) {
        int n = 0;
        for (int lx = l; lx >= 0; --lx)
            for (int ly = l - lx; ly >= 0; --ly) {
                c.v[l][n][0] = lx;
                c.v[l][n][1] = ly;
                c.v[l][n][2] = l - lx - ly;
                ++n;
            }
    }
    return c;
}
constexpr Cart kCart = make_cart();

// number of Rys roots for the derivative of a class of total angular momentum L:
// the raised integral has momentum L+1, so floor((L+1)/2) + 1 roots
__host__ __device__ constexpr int nroots_deriv(int L) { return (L + 1) / 2 + 1; }

// Make LDS writes of one lane visible to the other lanes of its wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimate refined by two
// Newton steps (each squares the relative error), cheaper than the IEEE division
// and square-root sequences
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = 0.5 * y, g = x * y;
        y = fma(y, fma(-g, h, 0.5), y);
    }
    return y;
}

// ------------------------------------------------------------------ Rys rule
template <int N> __device__ __forceinline__ const double *rys_poly();
template <> __device__ __forceinline__ const double *rys_poly<1>() { return rys_poly_1; }
template <> __device__ __forceinline__ const double *rys_poly<2>() { return rys_poly_2; }
template <> __device__ __forceinline__ const double *rys_poly<3>() { return rys_poly_3; }
template <> __device__ __forceinline__ const double *rys_poly<4>() { return rys_poly_4; }
template <> __device__ __forceinline__ const double *rys_poly<5>() { return rys_poly_5; }
template <int N> __device__ __forceinline__ const double *rys_hx();
template <> __device__ __forceinline__ const double *rys_hx<1>() { return rys_herm_x_1; }
template <> __device__ __forceinline__ const double *rys_hx<2>() { return rys_herm_x_2; }
template <> __device__ __forceinline__ const double *rys_hx<3>() { return rys_herm_x_3; }
template <> __device__ __forceinline__ const double *rys_hx<4>() { return rys_herm_x_4; }
template <> __device__ __forceinline__ const double *rys_hx<5>() { return rys_herm_x_5; }
template <int N> __device__ __forceinline__ const double *rys_hw();
template <> __device__ __forceinline__ const double *rys_hw<1>() { return rys_herm_w_1; }
template <> __device__ __forceinline__ const double *rys_hw<2>() { return rys_herm_w_2; }
template <> __device__ __forceinline__ const double *rys_hw<3>() { return rys_herm_w_3; }
template <> __device__ __forceinline__ const double *rys_hw<4>() { return rys_herm_w_4; }
template <> __device__ __forceinline__ const double *rys_hw<5>() { return rys_herm_w_5; }

// Polynomial sum_k c[k] x^k of NC coefficients by Estrin's scheme: coefficient pairs
// first, then pairs of pairs with x^2, x^4, ...  The dependency depth is about log2(NC)
// instead of NC - 1 for Horner's rule, for the same number of multiply-adds plus the
// powers of x; with |x| <= 1 (the table's intervals are centred) it is as accurate.
template <int NC>
__device__ __forceinline__ double poly_estrin(const double *c, double x)
{
    double v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = c[k];
    double xp = x;
    int n = NC;
#pragma unroll
    for (int level = 0; level < 8; ++level) {
        if (n <= 1) break;
#pragma unroll
        for (int j = 0; j < (NC + 1) / 2; ++j) {
            if (2 * j + 1 < n) v[j] = fma(v[2 * j + 1], xp, v[2 * j]);
            else if (2 * j < n) v[j] = v[2 * j];
        }
        n = (n + 1) / 2;
        xp = xp * xp;
    }
    return v[0];
}

// Root r (0-based, ascending) and weight of the N-point Rys rule at argument T >= 0:
// sum_r w_r u_r^k = F_k(T) for k < 2N.
template <int N>
__device__ __forceinline__ void rys_root(double T, int r, double &u, double &w)
{
    if (T < RYS_TMAX) {
        const int j = (int)(T * (1.0 / RYS_WIDTH));
        const double x = T - RYS_WIDTH * (j + 0.5);
        const double *cu = rys_poly<N>() + ((j * 2 * N) + r) * RYS_NCOEF;
        const double *cw = cu + N * RYS_NCOEF;
        u = poly_estrin<RYS_NCOEF>(cu, x);
        w = poly_estrin<RYS_NCOEF>(cw, x);
    } else {
        const double st = rsq64(T);
        const double xh = rys_hx<N>()[r] * st;
        u = xh * xh;
        w = rys_hw<N>()[r] * st;
    }
}

// Same rule with the polynomial table of N roots read from a copy in LDS
// (rys_table_to_lds<N> fills it: RYS_NINT * 2N * RYS_NCOEF doubles).
template <int N> constexpr int rys_table_size() { return RYS_NINT * 2 * N * RYS_NCOEF; }

template <int N>
__device__ __forceinline__ void rys_table_to_lds(double *lds)
{
    const double *src = rys_poly<N>();
    for (int i = threadIdx.x; i < rys_table_size<N>(); i += blockDim.x) lds[i] = src[i];
}

template <int N>
__device__ __forceinline__ void rys_root_lds(const double *tab, double T, int r, double &u, double &w)
{
    if (T < RYS_TMAX) {
        const int j = (int)(T * (1.0 / RYS_WIDTH));
        const double x = T - RYS_WIDTH * (j + 0.5);
        const double *cu = tab + ((j * 2 * N) + r) * RYS_NCOEF;
        const double *cw = cu + N * RYS_NCOEF;
        u = poly_estrin<RYS_NCOEF>(cu, x);
        w = poly_estrin<RYS_NCOEF>(cw, x);
    } else {
        const double st = rsq64(T);
        const double xh = rys_hx<N>()[r] * st;
        u = xh * xh;
        w = rys_hw<N>()[r] * st;
    }
}

__device__ __forceinline__ void rys_root_rt(int n, double T, int r, double &u, double &w)
{
    switch (n) {
    case 1: rys_root<1>(T, r, u, w); break;
    case 2: rys_root<2>(T, r, u, w); break;
    case 3: rys_root<3>(T, r, u, w); break;
    case 4: rys_root<4>(T, r, u, w); break;
    default: rys_root<5>(T, r, u, w); break;
    }
}

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ void atomic_add_global(double *p, double v)
{
    unsafeAtomicAdd(p, v); // global_atomic_add_f64 (coarse-grained device memory)
}

} // namespace tdg
