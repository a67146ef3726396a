// Fock-type matrix kernels of one angular class (la lb|lc ld), selected by
// -DTDG_CLASS=c in the library's class order (that of class_kernels.hip).
#include "fock_kernel.hpp"
#include "fock_launch.hpp"

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

// classes with at most 27 components: one lane per quartet (k_fock_lane); with 28 to 54
// components and the long-range kernel: a pair of lanes per quartet (k_fock_lane, PAIR);
// larger classes: a group of lanes per quartet (k_fock)
constexpr int kN = (LA + 1) * (LA + 2) / 2 * ((LB + 1) * (LB + 2) / 2) * ((LC + 1) * (LC + 2) / 2) *
                   ((LD + 1) * (LD + 2) / 2);
constexpr bool kLane = kN <= 27;
constexpr bool kPair = kN > 27 && kN <= 54;

template <bool LR>
hipError_t go(const tdg::FockArgs &a, hipStream_t st, int grid_max)
{
    using K = tdg::FockClass<LA, LB, LC, LD, LR>;
    constexpr bool pair = kPair && LR;
    const long long per = kLane ? tdg::FockLane<LA, LB, LC, LD, LR>::QPB
                                : (pair ? tdg::FockLane<LA, LB, LC, LD, true, true>::QPB : K::QPB);
    const long long blocks = (a.ntasks + per - 1) / per;
    // equal rounds per block (see class_kernels.hip)
    long long grid = blocks;
    if (blocks > grid_max) {
        const long long rounds = (blocks + grid_max - 1) / grid_max;
        grid = (blocks + rounds - 1) / rounds;
    }
    if (grid < 1) return hipSuccess;
    if constexpr (kLane)
        hipLaunchKernelGGL((tdg::k_fock_lane<LA, LB, LC, LD, LR>), dim3((unsigned)grid),
                           dim3(tdg::FockLane<LA, LB, LC, LD, LR>::BLOCK), 0, st, a);
    else if constexpr (pair)
        hipLaunchKernelGGL((tdg::k_fock_lane<LA, LB, LC, LD, true, true>), dim3((unsigned)grid),
                           dim3(tdg::FockLane<LA, LB, LC, LD, true, true>::BLOCK), 0, st, a);
    else
        hipLaunchKernelGGL((tdg::k_fock<LA, LB, LC, LD, LR>), dim3((unsigned)grid), dim3(K::BLOCK), 0, st, a);
    return hipGetLastError();
}
} // namespace

hipError_t TDG_FOCK_NAME(TDG_CLASS)(const tdg::FockArgs &a, bool lr, hipStream_t st, int grid_max)
{
    return lr ? go<true>(a, st, grid_max) : go<false>(a, st, grid_max);
}
