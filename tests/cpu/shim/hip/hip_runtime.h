// Host stand-in for the HIP runtime header, so that the device-side table recursions of the
// library (deriv_kernel.hpp) compile as plain C++ for a CPU test.  Only the table functions
// are called by the test; the kernels in the same header are templates that are never
// instantiated here, so the declarations below only have to satisfy name lookup.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__
#define __align__(x) alignas(x)
struct double2 { double x, y; };
struct int2 { int x, y; };
struct dim3_ { unsigned x = 0, y = 0, z = 0; };
static dim3_ threadIdx, blockIdx, blockDim, gridDim;
inline void __syncthreads() {}
inline double __shfl(double v, int) { return v; }
inline float __shfl(float v, int) { return v; }
inline int __shfl(int v, int) { return v; }
inline double __shfl_xor(double v, int) { return v; }
inline unsigned long long __ballot(int p) { return p ? 1ull : 0ull; }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __all(int p) { return p; }
inline double atomicAdd(double *p, double v) { double o = *p; *p += v; return o; }
inline void unsafeAtomicAdd(double *p, double v) { *p += v; }
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)0)
#define __builtin_amdgcn_readfirstlane(x) (x)
