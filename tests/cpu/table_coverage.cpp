// CPU test of the library's per-lane integral tables (csrc/deriv_kernel.hpp), compiled as host
// code: every table entry that a class kernel reads is written by the recursion first.  A read
// of an entry that the recursion never writes would take whatever the lane's private memory
// (registers or, when a kernel spills, scratch) held before, which makes a result depend on
// earlier launches.
//
// Tables: the vertical-recursion + transfer tables X[i][j][k][l] (Rys2D, team kernels of
// variant 0, FP64) for the momenta that the derivative formulas read: I(i,j,k,l), the raised
// B, C, D entries (j+1, k+1, l+1) and the lowered ones (j-1, k-1, l-1); and the direct
// four-centre base tables (variants 1-4) with their derivative tables.  Each table is filled
// with a sentinel bit pattern, built from random coefficients, and the entries read are
// checked against the sentinel.  Prints "OK <tables checked>" or the first failure.
#include <cstdio>
#include <cstring>
#include <random>

#include "../../paper_2407_16586_amd/csrc/deriv_kernel.hpp"

using namespace tdg;

static const uint64_t kSentinel = 0x7ff4deadbeef0001ull; // a NaN no arithmetic produces
static bool is_sentinel(double v)
{
    uint64_t b;
    std::memcpy(&b, &v, 8);
    return b == kSentinel;
}
static void poison(void *p, size_t bytes)
{
    double s;
    std::memcpy(&s, &kSentinel, 8);
    double *d = static_cast<double *>(p);
    for (size_t i = 0; i < bytes / 8; ++i) d[i] = s;
}

static std::mt19937_64 rng(7);
static double rnd() { return std::uniform_real_distribution<double>(0.1, 1.0)(rng); }
static int failures = 0, checked = 0;

template <int LA, int LB, int LC, int LD>
static void check_class()
{
    // variant 0: vertical recursion on A and C up to the raised momenta, transfers to B and D
    Rys2D<LA + LB + 1, LC + LD + 1, LA, LB + 1, LD + 1, double> g;
    poison(&g, sizeof(g));
    g.build(rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd());
    ++checked;
    for (int i = 0; i <= LA; ++i)
        for (int j = 0; j <= LB; ++j)
            for (int k = 0; k <= LC; ++k)
                for (int l = 0; l <= LD; ++l) {
                    const double reads[7] = {g.X[i][j][k][l], g.X[i][j + 1][k][l], g.X[i][j][k + 1][l],
                                             g.X[i][j][k][l + 1], j ? g.X[i][j - 1][k][l] : 0.0,
                                             k ? g.X[i][j][k - 1][l] : 0.0, l ? g.X[i][j][k][l - 1] : 0.0};
                    for (int r = 0; r < 7; ++r)
                        if (is_sentinel(reads[r])) {
                            if (failures++ < 10)
                                printf("unwritten X read: class (%d%d|%d%d) entry %d,%d,%d,%d read %d\n", LA, LB, LC,
                                       LD, i, j, k, l, r);
                        }
                }
    // variants 1-4: direct base tables and their derivative tables
    constexpr int NBASE = (LA + 1) * (LB + 1) * (LC + 1) * (LD + 1);
    double I[NBASE];
    poison(I, sizeof(I));
    direct_base<LA, LB, LC, LD, double>(I, rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd());
    double T[4 * NBASE];
    poison(T, sizeof(T));
    direct_tables<LA, LB, LC, LD, double>(T, rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(),
                                          rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd(), rnd());
    checked += 2;
    for (int e = 0; e < NBASE; ++e)
        if (is_sentinel(I[e]) && failures++ < 10) printf("unwritten base entry: class (%d%d|%d%d) %d\n", LA, LB, LC, LD, e);
    for (int e = 0; e < 4 * NBASE; ++e)
        if (is_sentinel(T[e]) && failures++ < 10)
            printf("unwritten derivative-table entry: class (%d%d|%d%d) %d\n", LA, LB, LC, LD, e);
}

int main()
{
    // the 21 classes, bra pair class >= ket pair class over (ss, ps, pp, ds, dp, dd)
#define P0 0, 0
#define P1 1, 0
#define P2 1, 1
#define P3 2, 0
#define P4 2, 1
#define P5 2, 2
#define C(b, k) check_class<b, k>();
    C(P0, P0) C(P1, P0) C(P1, P1) C(P2, P0) C(P2, P1) C(P2, P2) C(P3, P0) C(P3, P1) C(P3, P2) C(P3, P3)
    C(P4, P0) C(P4, P1) C(P4, P2) C(P4, P3) C(P4, P4) C(P5, P0) C(P5, P1) C(P5, P2) C(P5, P3) C(P5, P4)
    C(P5, P5)
    if (failures) {
        printf("FAILED %d\n", failures);
        return 1;
    }
    printf("OK %d\n", checked);
    return 0;
}
