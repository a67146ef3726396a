// Host-side launchers of the Fock-type matrix kernels; one definition per angular class,
// each in its own translation unit (fock_kernels.hip compiled with -DTDG_CLASS=c).
#pragma once
#include <hip/hip_runtime.h>

namespace tdg {
struct FockArgs;
// lr: the long-range exchange term is evaluated (a second Rys rule per primitive quartet)
using FockFn = hipError_t (*)(const FockArgs &a, bool lr, hipStream_t st, int grid_max);
} // namespace tdg

#define TDG_FOCK_NAME_(c) tdg_fock_class_##c
#define TDG_FOCK_NAME(c) TDG_FOCK_NAME_(c)
#define TDG_DECL_FOCK(c) hipError_t TDG_FOCK_NAME(c)(const tdg::FockArgs &a, bool lr, hipStream_t st, int grid_max);
TDG_DECL_FOCK(0) TDG_DECL_FOCK(1) TDG_DECL_FOCK(2) TDG_DECL_FOCK(3) TDG_DECL_FOCK(4)
TDG_DECL_FOCK(5) TDG_DECL_FOCK(6) TDG_DECL_FOCK(7) TDG_DECL_FOCK(8) TDG_DECL_FOCK(9)
TDG_DECL_FOCK(10) TDG_DECL_FOCK(11) TDG_DECL_FOCK(12) TDG_DECL_FOCK(13) TDG_DECL_FOCK(14)
TDG_DECL_FOCK(15) TDG_DECL_FOCK(16) TDG_DECL_FOCK(17) TDG_DECL_FOCK(18) TDG_DECL_FOCK(19)
TDG_DECL_FOCK(20)
