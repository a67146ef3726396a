// Kernels of one angular class (la lb|lc ld), selected by -DTDG_CLASS=c in the
// library's class order: bra pair class PB >= ket pair class PK over the pair
// classes (ss, ps, pp, ds, dp, dd), the highest momentum on centre A.
#include "class_launch.hpp"
#include "deriv_wave.hpp"

#ifndef TDG_CLASS
#error "compile with -DTDG_CLASS=<0..20>"
#endif

namespace {
constexpr int kPL[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
constexpr int class_pb(int c)
{
    int k = 0;
    for (int b = 0; b < 6; ++b)
        for (int q = 0; q <= b; ++q, ++k)
            if (k == c) return b;
    return -1;
}
constexpr int class_pk(int c)
{
    int k = 0;
    for (int b = 0; b < 6; ++b)
        for (int q = 0; q <= b; ++q, ++k)
            if (k == c) return q;
    return -1;
}
constexpr int LA = kPL[class_pb(TDG_CLASS)][0], LB = kPL[class_pb(TDG_CLASS)][1];
constexpr int LC = kPL[class_pk(TDG_CLASS)][0], LD = kPL[class_pk(TDG_CLASS)][1];
// the per-range team layout (variants 3, 4) exists for classes with <= 27 components
constexpr bool kAllRoots = (LA + 1) * (LA + 2) / 2 * ((LB + 1) * (LB + 2) / 2) * ((LC + 1) * (LC + 2) / 2) *
                               ((LD + 1) * (LD + 2) / 2) <= 27;

// Blocks for ntasks tasks taken `per` at a time by each block round, at most grid_max: when
// the tasks need more rounds than one per block, the grid is shrunk so that every block does
// the same number of rounds (no last round run by a few blocks while the rest of the GPU
// idles).
static int grid_for(long long ntasks, long long per, int grid_max)
{
    const long long blocks = (ntasks + per - 1) / per;
    if (blocks <= grid_max) return (int)blocks;
    const long long rounds = (blocks + grid_max - 1) / grid_max;
    return (int)((blocks + rounds - 1) / rounds);
}

template <bool LR, typename F>
hipError_t go(int variant, const tdg::DerivArgs &a, hipStream_t st, int grid_max)
{
    using namespace tdg;
    const size_t dyn = a.lds_atoms ? (size_t)3 * a.n_atoms * sizeof(double) : 0;
    if constexpr (kAllRoots) {
        if (variant == 3 || variant == 4) {
            using K = DerivClass<LA, LB, LC, LD, LR, F, true>;
            const int grid = grid_for(a.ntasks, K::TPB, grid_max);
            if (variant == 4)
                hipLaunchKernelGGL((k_deriv<LA, LB, LC, LD, LR, F, 2, true>), dim3(grid), dim3(K::BLOCK), dyn,
                                   st, a);
            else if constexpr (sizeof(F) != sizeof(double))
                hipLaunchKernelGGL((k_deriv<LA, LB, LC, LD, LR, F, 1, true>), dim3(grid), dim3(K::BLOCK), dyn,
                                   st, a);
            else
                hipLaunchKernelGGL((k_deriv<LA, LB, LC, LD, LR, F, 0, true>), dim3(grid), dim3(K::BLOCK), dyn,
                                   st, a);
            return hipGetLastError();
        }
    }
    if (variant == 3) variant = 0; // classes without the per-range layout
    if (variant == 4) variant = 2;
    if (variant == 0 || variant == 2) {
        using K = DerivClass<LA, LB, LC, LD, LR, F>;
        const int grid = grid_for(a.ntasks, K::TPB, grid_max);
        if (variant == 2)
            hipLaunchKernelGGL((k_deriv<LA, LB, LC, LD, LR, F, 2>), dim3(grid), dim3(K::BLOCK), dyn, st, a);
        else if constexpr (sizeof(F) != sizeof(double))
            hipLaunchKernelGGL((k_deriv<LA, LB, LC, LD, LR, F, 1>), dim3(grid), dim3(K::BLOCK), dyn, st, a);
        else
            hipLaunchKernelGGL((k_deriv<LA, LB, LC, LD, LR, F, 0>), dim3(grid), dim3(K::BLOCK), dyn, st, a);
    } else {
        using K = WaveClass<LA, LB, LC, LD, LR, F>;
        const int grid = grid_for(a.ntasks, K::WAVES, grid_max);
        hipLaunchKernelGGL((k_deriv_wave<LA, LB, LC, LD, LR, F>), dim3(grid), dim3(K::BLOCK), dyn, st, a);
    }
    return hipGetLastError();
}

template <bool LR, typename F>
const void *kernel_ptr(int variant)
{
    using namespace tdg;
    if constexpr (kAllRoots) {
        if (variant == 4) return reinterpret_cast<const void *>(&k_deriv<LA, LB, LC, LD, LR, F, 2, true>);
        if (variant == 3) {
            if constexpr (sizeof(F) != sizeof(double))
                return reinterpret_cast<const void *>(&k_deriv<LA, LB, LC, LD, LR, F, 1, true>);
            else
                return reinterpret_cast<const void *>(&k_deriv<LA, LB, LC, LD, LR, F, 0, true>);
        }
    }
    if (variant == 3) variant = 0;
    if (variant == 4) variant = 2;
    if (variant == 1) return reinterpret_cast<const void *>(&k_deriv_wave<LA, LB, LC, LD, LR, F>);
    if (variant == 2) return reinterpret_cast<const void *>(&k_deriv<LA, LB, LC, LD, LR, F, 2>);
    if constexpr (sizeof(F) != sizeof(double))
        return reinterpret_cast<const void *>(&k_deriv<LA, LB, LC, LD, LR, F, 1>);
    else
        return reinterpret_cast<const void *>(&k_deriv<LA, LB, LC, LD, LR, F, 0>);
}

template <bool LR, typename F>
size_t scratch_of(int variant)
{
    hipFuncAttributes a1{};
    if (hipFuncGetAttributes(&a1, kernel_ptr<LR, F>(variant)) != hipSuccess) return (size_t)-1;
    return a1.localSizeBytes;
}
} // namespace

size_t TDG_SCRATCH_NAME(TDG_CLASS)(int variant, int prec, bool lr)
{
    return prec ? (lr ? scratch_of<true, float>(variant) : scratch_of<false, float>(variant))
                : (lr ? scratch_of<true, double>(variant) : scratch_of<false, double>(variant));
}

hipError_t TDG_LAUNCH_NAME(TDG_CLASS)(int variant, int prec, const tdg::DerivArgs &a, bool lr, hipStream_t st,
                                      int grid_max)
{
    if (prec) return lr ? go<true, float>(variant, a, st, grid_max) : go<false, float>(variant, a, st, grid_max);
    return lr ? go<true, double>(variant, a, st, grid_max) : go<false, double>(variant, a, st, grid_max);
}
