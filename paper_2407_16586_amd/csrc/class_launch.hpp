// Host-side launchers of the ERI-derivative class kernels; one definition per
// angular class, each in its own translation unit (class_kernels.hip compiled with
// -DTDG_CLASS=c).
#pragma once
#include <hip/hip_runtime.h>

namespace tdg {
struct DerivArgs;
// variant 0: team of lanes per shell quartet (FP64: vertical recursion + transfers;
// FP32: direct four-centre derivative tables), 1: wavefront per shell quartet,
// 2: team of lanes with direct four-centre base tables and the collapsed contraction;
// 3, 4: as 0, 2 with one lane per (quartet, range) looping over the roots (classes with
// <= 27 components; elsewhere they run as 0, 2);
// prec 0: FP64 2D integrals, 1: FP32 2D integrals (FP64 roots and sums)
using LaunchFn = hipError_t (*)(int variant, int prec, const DerivArgs &a, bool lr, hipStream_t st, int grid_max);
// per-lane scratch (private segment) bytes of a variant's kernel; (size_t)-1 if unknown
using ScratchFn = size_t (*)(int variant, int prec, bool lr);
} // namespace tdg

#define TDG_LAUNCH_NAME_(c) tdg_launch_class_##c
#define TDG_LAUNCH_NAME(c) TDG_LAUNCH_NAME_(c)
#define TDG_SCRATCH_NAME_(c) tdg_class_scratch_##c
#define TDG_SCRATCH_NAME(c) TDG_SCRATCH_NAME_(c)
#define TDG_DECL_LAUNCH(c) \
    hipError_t TDG_LAUNCH_NAME(c)(int variant, int prec, const tdg::DerivArgs &a, bool lr, hipStream_t st, int grid_max); \
    size_t TDG_SCRATCH_NAME(c)(int variant, int prec, bool lr);
TDG_DECL_LAUNCH(0) TDG_DECL_LAUNCH(1) TDG_DECL_LAUNCH(2) TDG_DECL_LAUNCH(3) TDG_DECL_LAUNCH(4)
TDG_DECL_LAUNCH(5) TDG_DECL_LAUNCH(6) TDG_DECL_LAUNCH(7) TDG_DECL_LAUNCH(8) TDG_DECL_LAUNCH(9)
TDG_DECL_LAUNCH(10) TDG_DECL_LAUNCH(11) TDG_DECL_LAUNCH(12) TDG_DECL_LAUNCH(13) TDG_DECL_LAUNCH(14)
TDG_DECL_LAUNCH(15) TDG_DECL_LAUNCH(16) TDG_DECL_LAUNCH(17) TDG_DECL_LAUNCH(18) TDG_DECL_LAUNCH(19)
TDG_DECL_LAUNCH(20)
