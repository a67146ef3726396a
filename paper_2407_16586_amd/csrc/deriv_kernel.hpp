// ERI-derivative class kernels: Rys quadrature, translational invariance,
// on-the-fly contraction with the two-particle densities (section II.C,
// eqs deriv, deri, ti, eriupdate; densities of eq gamma).
#pragma once
#include "tdg_device.hpp"

namespace tdg {

struct DerivArgs {
    const double *coords;   // [n_atoms][3]
    const int *shell_atom;  // [n_shells]
    const int *shell_ao;    // [n_shells]
    const int *pair_sa, *pair_sb, *pair_ppoff, *pair_npp; // sorted shell pairs
    const double2 *pp_rec;  // per primitive pair, 4 x double2: (p, 1/p) (c, za) (zb, Px) (Py, Pz)
    const double *dens;     // shell-blocked P, D, R records with the angular normalisation folded in
    int n_bf;
    const int2 *tasks;      // (bra pair, ket pair) of this class
    long long ntasks;
    double omega, alpha, beta;
    int terms;
    double *grad;           // [n_atoms][3]
    int n_atoms;
    int lds_atoms;          // 1: block-level accumulation in LDS (dynamic shared memory)
    double *task_out;       // optional per-task output [ntasks][12] (canonical centres)
};

// 2D Rys integrals for one root and one Cartesian direction.
// Vertical recursion on centres A (bra) and C (ket) up to n <= NM, m <= MM, then
// horizontal transfer A->B (j <= JE) and C->D (l <= LE).  Entry X[i][j][k][l] is
// defined for i <= IE, j <= JE, k + l <= MM with k <= MM - l.
template <int NM, int MM, int IE, int JE, int LE, typename F = double>
struct Rys2D {
    F X[IE + 1][JE + 1][MM + 1][LE + 1];

    __device__ __forceinline__ void build(F I0, F C00, F D00, F B10, F B01, F B00, F AB, F CD)
    {
        F V[NM + 1][MM + 1];
        V[0][0] = I0;
        if constexpr (NM >= 1) V[1][0] = C00 * I0;
#pragma unroll
        for (int n = 1; n < NM; ++n) V[n + 1][0] = C00 * V[n][0] + (F(n) * B10) * V[n - 1][0];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
#pragma unroll
            for (int n = 0; n <= NM; ++n) {
                F v = D00 * V[n][m];
                if (m > 0) v += (F(m) * B01) * V[n][m > 0 ? m - 1 : 0];
                if (n > 0) v += (F(n) * B00) * V[n > 0 ? n - 1 : 0][m];
                V[n][m + 1] = v;
            }
        }
        F W[NM + 1][JE + 1][MM + 1];
#pragma unroll
        for (int i = 0; i <= NM; ++i)
#pragma unroll
            for (int m = 0; m <= MM; ++m) W[i][0][m] = V[i][m];
#pragma unroll
        for (int j = 0; j < JE; ++j)
#pragma unroll
            for (int i = 0; i < NM - j; ++i)
#pragma unroll
                for (int m = 0; m <= MM; ++m) W[i][j + 1][m] = W[i + 1][j][m] + AB * W[i][j][m];
#pragma unroll
        for (int i = 0; i <= IE; ++i)
#pragma unroll
            for (int j = 0; j <= JE; ++j)
#pragma unroll
                for (int k = 0; k <= MM; ++k) X[i][j][k][0] = W[i][j][k];
#pragma unroll
        for (int l = 0; l < LE; ++l)
#pragma unroll
            for (int i = 0; i <= IE; ++i)
#pragma unroll
                for (int j = 0; j <= JE; ++j)
#pragma unroll
                    for (int k = 0; k < MM - l; ++k) X[i][j][k][l + 1] = X[i][j][k + 1][l] + CD * X[i][j][k][l];
    }
};

// Direct four-centre form used for the FP32 route.  The 2D integrals over the base
// index range (i<=la, j<=lb, k<=lc, l<=ld) are built by raising each index with its
// own centre's displacement,
//   I(.., x+1, ..) = C_X I + B10 [i I(i-1) + j I(j-1)] + B00 [k I(k-1) + l I(l-1)]   (x = i, j)
//   I(.., x+1, ..) = C_X I + B01 [k I(k-1) + l I(l-1)] + B00 [i I(i-1) + j I(j-1)]   (x = k, l)
// with C_A = (P-A) - rho/p PQ u, C_B = (P-B) - rho/p PQ u, C_C = (Q-C) + rho/q PQ u,
// C_D = (Q-D) + rho/q PQ u, so no step transfers momentum across a bond (no
// A->B difference of large terms).  The centre derivatives 2 zeta X(+1) - n X(-1) are
// expanded with the same recurrence, e.g.
//   dB = 2 zb C_B I + 2 zb B10 i I(i-1) + (2 zb B10 - 1) j I(j-1) + 2 zb B00 (k I(k-1) + l I(l-1)),
// whose coefficients (2 zb B10 - 1 = -za/p - zb q u/(p(p+q)) and its C, D analogues) are
// formed in FP64 without cancellation.
struct DirectCoef {
    double e2, e3, e4, f2, f3, f4, g2, g3, g4; // direction-independent derivative coefficients
};

__device__ __forceinline__ DirectCoef direct_coef(double za, double zb, double zc, double zd, double p, double q,
                                                  double ip, double iq, double u, double ipq, double B10, double B01,
                                                  double B00)
{
    DirectCoef c;
    c.e2 = 2.0 * zb * B10;
    c.e3 = -(za + zb * q * u * ipq) * ip;
    c.e4 = 2.0 * zb * B00;
    c.f2 = -(zd + zc * p * u * ipq) * iq;
    c.f3 = 2.0 * zc * B01;
    c.f4 = 2.0 * zc * B00;
    c.g2 = 2.0 * zd * B01;
    c.g3 = -(zc + zd * p * u * ipq) * iq;
    c.g4 = 2.0 * zd * B00;
    return c;
}

// Base-range 2D integrals I[e], e = ((i*(lb+1)+j)*(lc+1)+k)*(ld+1)+l, by the direct
// four-centre recurrence above.
template <int LA, int LB, int LC, int LD, typename F>
__device__ __forceinline__ void direct_base(F *I, F I0, F CA, F CB, F CC, F CDd, F B10, F B01, F B00)
{
    constexpr int NB1 = LB + 1, NC1 = LC + 1, ND1 = LD + 1;
#define IX(i, j, k, l) I[(((i) * NB1 + (j)) * NC1 + (k)) * ND1 + (l)]
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LB; ++j)
#pragma unroll
            for (int k = 0; k <= LC; ++k)
#pragma unroll
                for (int l = 0; l <= LD; ++l) {
                    F v;
                    if (l > 0) {
                        const int l0 = l - 1;
                        v = CDd * IX(i, j, k, l0);
                        if (k > 0) v += F(k) * B01 * IX(i, j, k > 0 ? k - 1 : 0, l0);
                        if (l0 > 0) v += F(l0) * B01 * IX(i, j, k, l0 > 0 ? l0 - 1 : 0);
                        if (i > 0) v += F(i) * B00 * IX(i > 0 ? i - 1 : 0, j, k, l0);
                        if (j > 0) v += F(j) * B00 * IX(i, j > 0 ? j - 1 : 0, k, l0);
                    } else if (k > 0) {
                        const int k0 = k - 1;
                        v = CC * IX(i, j, k0, 0);
                        if (k0 > 0) v += F(k0) * B01 * IX(i, j, k0 > 0 ? k0 - 1 : 0, 0);
                        if (i > 0) v += F(i) * B00 * IX(i > 0 ? i - 1 : 0, j, k0, 0);
                        if (j > 0) v += F(j) * B00 * IX(i, j > 0 ? j - 1 : 0, k0, 0);
                    } else if (j > 0) {
                        const int j0 = j - 1;
                        v = CB * IX(i, j0, 0, 0);
                        if (i > 0) v += F(i) * B10 * IX(i > 0 ? i - 1 : 0, j0, 0, 0);
                        if (j0 > 0) v += F(j0) * B10 * IX(i, j0 > 0 ? j0 - 1 : 0, 0, 0);
                    } else if (i > 0) {
                        const int i0 = i - 1;
                        v = CA * IX(i0, 0, 0, 0);
                        if (i0 > 0) v += F(i0) * B10 * IX(i0 > 0 ? i0 - 1 : 0, 0, 0, 0);
                    } else {
                        v = I0;
                    }
                    IX(i, j, k, l) = v;
                }
#undef IX
}

// out[0][e] = I, out[1][e] = dB, out[2][e] = dC, out[3][e] = dD for the base index
// e = ((i*(lb+1)+j)*(lc+1)+k)*(ld+1)+l; stride between the four kinds is NBASE.
template <int LA, int LB, int LC, int LD, typename F, typename OUT>
__device__ __forceinline__ void direct_tables(OUT &out, F I0, F CA, F CB, F CC, F CDd, F B10, F B01, F B00, F e1, F e2,
                                              F e3, F e4, F f1, F f2, F f3, F f4, F g1, F g2, F g3, F g4)
{
    constexpr int NB1 = LB + 1, NC1 = LC + 1, ND1 = LD + 1;
    constexpr int NBASE = (LA + 1) * NB1 * NC1 * ND1;
    F I[NBASE];
    direct_base<LA, LB, LC, LD, F>(I, I0, CA, CB, CC, CDd, B10, B01, B00);
#define IX(i, j, k, l) I[(((i) * NB1 + (j)) * NC1 + (k)) * ND1 + (l)]
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LB; ++j)
#pragma unroll
            for (int k = 0; k <= LC; ++k)
#pragma unroll
                for (int l = 0; l <= LD; ++l) {
                    const int e = ((i * NB1 + j) * NC1 + k) * ND1 + l;
                    const F v = I[e];
                    const F im = i ? F(i) * IX(i ? i - 1 : 0, j, k, l) : F(0);
                    const F jm = j ? F(j) * IX(i, j ? j - 1 : 0, k, l) : F(0);
                    const F km = k ? F(k) * IX(i, j, k ? k - 1 : 0, l) : F(0);
                    const F lm = l ? F(l) * IX(i, j, k, l ? l - 1 : 0) : F(0);
                    out[e] = v;
                    out[NBASE + e] = e1 * v + e2 * im + e3 * jm + e4 * (km + lm);
                    out[2 * NBASE + e] = f1 * v + f2 * km + f3 * lm + f4 * (im + jm);
                    out[3 * NBASE + e] = g1 * v + g2 * km + g3 * lm + g4 * (im + jm);
                }
#undef IX
}

// Collapsed contraction of one root.  With H_x[e] = sum over the components whose
// x index quadruple is e of Gamma * I_y * I_z (and H_y, H_z alike), the nine
// derivative sums of the root are
//   dB_d = e1_d S0 + e2 Si + e3 Sj + e4 (Sk + Sl)
//   dC_d = f1_d S0 + f2 Sk + f3 Sl + f4 (Si + Sj)
//   dD_d = g1_d S0 + g2 Sk + g3 Sl + g4 (Si + Sj)
// with S0 = sum_e H_d[e] I_d[e] and Si = sum_e H_d[e] i I_d[e - 1_i] (Sj, Sk, Sl
// alike), since the direct derivative tables are those combinations of base
// entries.  The five S sums per direction leave the working precision F here.
template <int LA, int LB, int LC, int LD, typename F>
__device__ __forceinline__ void collapse_sums(const F *H, const F *I, double S[5])
{
    constexpr int NB1 = LB + 1, NC1 = LC + 1, ND1 = LD + 1;
    F s0 = F(0), si = F(0), sj = F(0), sk = F(0), sl = F(0);
#define IX(i, j, k, l) I[(((i) * NB1 + (j)) * NC1 + (k)) * ND1 + (l)]
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LB; ++j)
#pragma unroll
            for (int k = 0; k <= LC; ++k)
#pragma unroll
                for (int l = 0; l <= LD; ++l) {
                    const int e = ((i * NB1 + j) * NC1 + k) * ND1 + l;
                    const F h = H[e];
                    s0 += h * I[e];
                    if (i) si += (F(i) * h) * IX(i ? i - 1 : 0, j, k, l);
                    if (j) sj += (F(j) * h) * IX(i, j ? j - 1 : 0, k, l);
                    if (k) sk += (F(k) * h) * IX(i, j, k ? k - 1 : 0, l);
                    if (l) sl += (F(l) * h) * IX(i, j, k, l ? l - 1 : 0);
                }
#undef IX
    S[0] = double(s0); S[1] = double(si); S[2] = double(sj); S[3] = double(sk); S[4] = double(sl);
}

// Team layout of the team kernels.  ALLR = false: one lane per (root, range) of a
// quartet; ALLR = true: one lane per range, looping over the roots (the primitive-pair
// setup is then done once per range instead of once per root).
template <int LA, int LB, int LC, int LD, bool LR, typename F = double, bool ALLR = false>
struct DerivClass {
    static constexpr int L = LA + LB + LC + LD;
    static constexpr int NR = nroots_deriv(L);
    static constexpr int NSET = LR ? 2 : 1;
    static constexpr int RPL = ALLR ? NR : 1;      // roots per lane
    static constexpr int TEAM = (NR / RPL) * NSET;
    static constexpr int TPW = kWave / TEAM;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int N = NA * NB * NC * ND;
    static constexpr int GSTRIDE = NSET * N + 1;  // odd stride: teams start in different banks
    // Rys table of the class staged in LDS when it fits beside Gamma (n <= 3 roots); the
    // static LDS (Gamma + table) stays within 40 KB so that with the per-atom array
    // (<= 24 KB) a block needs at most 64 KB
    static constexpr bool TAB_LDS = NR <= 3;
    static constexpr int TAB_N = TAB_LDS ? rys_table_size<NR>() : 1;
    static constexpr int LDS_G_BYTES = 40 * 1024 - (TAB_LDS ? TAB_N * 8 : 0);
    static constexpr int GB = (int)sizeof(F);
    static constexpr int TPB_LDS = LDS_G_BYTES / (GSTRIDE * GB) > 0 ? LDS_G_BYTES / (GSTRIDE * GB) : 1;
    // two wavefronts per block (measured on the 60-atom chain: 1, 2, 4 wavefronts give
    // 12.2, 10.8, 11.4 ms of mixed-path class kernels)
    static constexpr int TPB = TPW * 2 < TPB_LDS ? TPW * 2 : TPB_LDS;
    static constexpr int WAVES = (TPB + TPW - 1) / TPW;
    static constexpr int BLOCK = WAVES * kWave;
    // ket primitive records loaded one primitive ahead: pays where a primitive's work is
    // short (few components, one root per lane); elsewhere the extra live registers
    // would cost occupancy
    static constexpr bool EARLY_PREFETCH = !ALLR && N <= 9;
    // per-range lanes evaluate their roots interleaved where the per-root state is small
    static constexpr int ROOT_UNROLL = (ALLR && N <= 9) ? RPL : 1;
};

// Shell-blocked densities: the record of the ordered shell pair (x, y) starts at
// 3 (ao_x n_bf + ncart(l_x) ao_y) and holds the P, D and R blocks (ncart(l_x) x ncart(l_y),
// row-major) back to back, so that every block a quartet reads is contiguous.
__device__ __forceinline__ size_t dens_rec(int n_bf, int ao_x, int nx, int ao_y)
{
    return 3 * ((size_t)ao_x * n_bf + (size_t)nx * ao_y);
}

// Permutation-averaged Gamma and Gamma^lr (eq gamma) of one Cartesian component
// (ia, ib, ic, id) of the quartet (a b | c d) whose shell momenta are LA..LD; rec[]
// holds the records of the ordered pairs ab ba cd dc ac ca ad da bc cb bd db.
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void gamma_sym(const DerivArgs &a, const size_t rec[12], int ia, int ib, int ic, int id,
                                          double deg, double &gf, double &gl)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    const double *B = a.dens;
    // element (i, j) of the P (0), D (1) or R (2) block of the pair record r with row/column sizes nx, ny
#define E_(r, k, nx, ny, i, j) B[rec[r] + (k) * (nx) * (ny) + (i) * (ny) + (j)]
    const double rs_mn = 0.5 * (E_(0, 2, NA, NB, ia, ib) + E_(1, 2, NB, NA, ib, ia));
    const double rs_ls = 0.5 * (E_(2, 2, NC, ND, ic, id) + E_(3, 2, ND, NC, id, ic));
    const double J = 2.0 * rs_mn * rs_ls + 0.25 * (E_(0, 1, NA, NB, ia, ib) * E_(2, 0, NC, ND, ic, id) +
                                                   E_(0, 0, NA, NB, ia, ib) * E_(2, 1, NC, ND, ic, id));
    // D_ms P_nl + D_ns P_ml + D_ml P_ns + D_nl P_ms
    const double KD = E_(6, 1, NA, ND, ia, id) * E_(8, 0, NB, NC, ib, ic) + E_(10, 1, NB, ND, ib, id) * E_(4, 0, NA, NC, ia, ic) +
                      E_(4, 1, NA, NC, ia, ic) * E_(10, 0, NB, ND, ib, id) + E_(8, 1, NB, NC, ib, ic) * E_(6, 0, NA, ND, ia, id);
    // R_sm R_ln + R_sn R_lm + R_ms R_nl + R_ml R_ns
    const double KR = E_(7, 2, ND, NA, id, ia) * E_(9, 2, NC, NB, ic, ib) + E_(11, 2, ND, NB, id, ib) * E_(5, 2, NC, NA, ic, ia) +
                      E_(6, 2, NA, ND, ia, id) * E_(8, 2, NB, NC, ib, ic) + E_(4, 2, NA, NC, ia, ic) * E_(10, 2, NB, ND, ib, id);
#undef E_
    const double K = 0.0625 * KD + 0.25 * KR;
    gf = deg * (((a.terms & 1) ? J : 0.0) - ((a.terms & 2) ? a.alpha * K : 0.0));
    gl = deg * ((a.terms & 4) ? -a.beta * K : 0.0);
}

// Records of the 12 ordered shell pairs of the quartet (a b | c d) with AO offsets oa..od.
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void pair_records(int n_bf, int oa, int ob, int oc, int od, size_t rec[12])
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    rec[0] = dens_rec(n_bf, oa, NA, ob); rec[1] = dens_rec(n_bf, ob, NB, oa);
    rec[2] = dens_rec(n_bf, oc, NC, od); rec[3] = dens_rec(n_bf, od, ND, oc);
    rec[4] = dens_rec(n_bf, oa, NA, oc); rec[5] = dens_rec(n_bf, oc, NC, oa);
    rec[6] = dens_rec(n_bf, oa, NA, od); rec[7] = dens_rec(n_bf, od, ND, oa);
    rec[8] = dens_rec(n_bf, ob, NB, oc); rec[9] = dens_rec(n_bf, oc, NC, ob);
    rec[10] = dens_rec(n_bf, ob, NB, od); rec[11] = dens_rec(n_bf, od, ND, ob);
}

// F: type of the 2D integrals, derivative products and per-primitive partial sums
// (double, or float for the mixed-precision route); roots, weights, prefactors and
// the running sums are FP64 in both.  MODE 0: vertical recursion plus transfers
// (FP64 only); 1: derivative tables from the direct four-centre recurrence; 2: the
// direct base tables with the collapsed contraction (collapse_sums).  ALLR: each lane
// evaluates all roots of its range (see DerivClass).
template <int LA, int LB, int LC, int LD, bool LR, typename F, int MODE, bool ALLR = false>
__global__ void __launch_bounds__((DerivClass<LA, LB, LC, LD, LR, F, ALLR>::BLOCK))
k_deriv(const DerivArgs a)
{
    using K = DerivClass<LA, LB, LC, LD, LR, F, ALLR>;
    constexpr int NR = K::NR, TEAM = K::TEAM, TPW = K::TPW, TPB = K::TPB, RPL = K::RPL;
    constexpr int NA = K::NA, NB = K::NB, NC = K::NC, ND = K::ND, N = K::N;
    // FP32 route: the per-primitive partial sums go to the FP64 sums after every
    // (a, b) component pair (2) or every a component (1) when those groups hold
    // several components, so no FP32 sum runs over more than NC*ND (NB*NC*ND) terms
    constexpr int FLUSH = (sizeof(F) == sizeof(double) || MODE != 1) ? 0 : (NC * ND >= 6 ? 2 : (NB * NC * ND >= 6 ? 1 : 0));
    auto flush = [](double *acc, F *pacc) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            acc[k] += double(pacc[k]);
            pacc[k] = F(0);
        }
    };
    extern __shared__ double s_atoms[];
    __shared__ F s_gam[TPB * K::GSTRIDE];
    __shared__ double s_rys[K::TAB_N];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int tw = lane / TEAM, r = lane % TEAM;
    if constexpr (K::TAB_LDS) {
        rys_table_to_lds<NR>(s_rys);
        __syncthreads();
    }
    const int team = wave * TPW + tw;
    const bool lane_ok = (tw < TPW) && (team < TPB);
    const int set = r / (NR / RPL), ir0 = r % (NR / RPL);
    F *myG = s_gam + (lane_ok ? team : 0) * K::GSTRIDE;

    if (a.lds_atoms) {
        for (int i = tid; i < 3 * a.n_atoms; i += blockDim.x) s_atoms[i] = 0.0;
        __syncthreads();
    }
    const double iom2 = LR ? 1.0 / (a.omega * a.omega) : 0.0;
    // blocks take rounds of TPB consecutive tasks at a fixed grid stride (the host sizes the
    // grid so that every block does the same number of rounds); consecutive blocks run on
    // different XCDs, so every XCD gets an even share of each stretch of the task list
    const long long stride = (long long)gridDim.x * TPB;
    for (long long base = (long long)blockIdx.x * TPB; base < a.ntasks; base += stride) {
        const long long t = base + team;
        const bool valid = lane_ok && t < a.ntasks;
        int bra = 0, ket = 0, sa = 0, sb = 0, sc = 0, sd = 0;
        const DerivArgs &M = a;
        if (valid) {
            const int2 tk = a.tasks[t];
            bra = tk.x;
            ket = tk.y;
            sa = M.pair_sa[bra]; sb = M.pair_sb[bra];
            sc = M.pair_sa[ket]; sd = M.pair_sb[ket];
            const double deg = (sa != sb ? 2.0 : 1.0) * (sc != sd ? 2.0 : 1.0) * (bra != ket ? 2.0 : 1.0);
            const int oa = M.shell_ao[sa], ob = M.shell_ao[sb], oc = M.shell_ao[sc], od = M.shell_ao[sd];
            size_t rec[12];
            pair_records<LA, LB, LC, LD>(M.n_bf, oa, ob, oc, od, rec);
            for (int c = r; c < N; c += TEAM) {
                const int id = c % ND, ic = (c / ND) % NC, ib = (c / (ND * NC)) % NB, ia = c / (ND * NC * NB);
                double gf, gl;
                gamma_sym<LA, LB, LC, LD>(M, rec, ia, ib, ic, id, deg, gf, gl);
                myG[c] = F(gf);
                if constexpr (LR) myG[N + c] = F(gl);
            }
        }
        wave_sync();
        double acc[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        int atA = 0, atB = 0, atC = 0, atD = 0;
        if (valid) {
            atA = M.shell_atom[sa]; atB = M.shell_atom[sb]; atC = M.shell_atom[sc]; atD = M.shell_atom[sd];
            double A[3], AB[3], Cc[3], CD[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                A[d] = M.coords[3 * atA + d];
                AB[d] = A[d] - M.coords[3 * atB + d];
                Cc[d] = M.coords[3 * atC + d];
                CD[d] = Cc[d] - M.coords[3 * atD + d];
            }
            const int pb0 = M.pair_ppoff[bra], nbp = M.pair_npp[bra];
            const int pk0 = M.pair_ppoff[ket], nkp = M.pair_npp[ket];
            const int gbase = (lane_ok ? team : 0) * K::GSTRIDE + set * N;
            const double2 *rb = M.pp_rec + 4 * (size_t)pb0, *rk = M.pp_rec + 4 * (size_t)pk0;
            for (int ib = 0; ib < nbp; ++ib) {
                const double2 b0 = rb[4 * ib], b1 = rb[4 * ib + 1], b2 = rb[4 * ib + 2], b3 = rb[4 * ib + 3];
                const double p = b0.x, ip = b0.y, zab = b1.y, zb2 = 2.0 * b2.x;
                // 2 pi^(5/2) times the bra contraction factor over p
                const double cab = 34.98683665524972 * b1.x * ip;
                const double P[3] = {b2.y, b3.x, b3.y};
                // ket record of the current primitive; the next one is loaded ahead: at the
                // start of the current primitive's work in the small classes (the latency of
                // the load is then hidden behind the whole primitive), else at its end
                double2 n0 = rk[0], n1 = rk[1], n2 = rk[2], n3 = rk[3];
                for (int ik = 0; ik < nkp; ++ik) {
                    // Gamma is re-read from LDS for every primitive quartet: an opaque offset
                    // keeps the compiler from hoisting all N values into registers
                    int goff = gbase;
                    if constexpr (N > 8) asm volatile("" : "+v"(goff));
                    const F *gam = s_gam + goff;
                    const double2 k0 = n0, k1 = n1, k2 = n2, k3 = n3;
                    const int kn = ik + 1 < nkp ? ik + 1 : ik;
                    if constexpr (K::EARLY_PREFETCH) {
                        n0 = rk[4 * kn]; n1 = rk[4 * kn + 1]; n2 = rk[4 * kn + 2]; n3 = rk[4 * kn + 3];
                    }
                    const double q = k0.x, iq = k0.y, ccd = k1.x;
                    const double zc2 = 2.0 * k1.y, zd2 = 2.0 * k2.x;
                    const double Q[3] = {k2.y, k3.x, k3.y};
                    const double sipq = rsq64(p + q), ipq = sipq * sipq;
                    const double rho = p * q * ipq;
                    double PQ[3], pq2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        PQ[d] = P[d] - Q[d];
                        pq2 += PQ[d] * PQ[d];
                    }
                    double Tr = rho * pq2, eta = 1.0, seta = 1.0;
                    if (LR && set) {
                        seta = rsq64(1.0 + rho * iom2); // sqrt(omega^2 / (omega^2 + rho))
                        eta = seta * seta;
                        Tr *= eta;
                    }
#pragma unroll K::ROOT_UNROLL
                    for (int rr = 0; rr < RPL; ++rr) {
                    const int ir = RPL == 1 ? ir0 : rr;
                    double u, w;
                    if constexpr (K::TAB_LDS) rys_root_lds<NR>(s_rys, Tr, ir, u, w);
                    else rys_root<NR>(Tr, ir, u, w);
                    if (LR && set) {
                        u *= eta;
                        w *= seta;
                    }
                    // 2 pi^(5/2) / (p q sqrt(p+q)) times contraction and pair factors
                    const double pref = cab * (ccd * iq) * sipq * w;
                    const double B00 = 0.5 * u * ipq;
                    const double B10 = 0.5 * ip * (1.0 - q * ipq * u);
                    const double B01 = 0.5 * iq * (1.0 - p * ipq * u);
                    const double cq = q * ipq * u, cp = p * ipq * u;
                    F pacc[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) pacc[k] = F(0);
                    if constexpr (MODE == 0) {
                        Rys2D<LA + LB + 1, LC + LD + 1, LA, LB + 1, LD + 1, F> g[3];
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double PA = P[d] - A[d], QC = Q[d] - Cc[d];
                            g[d].build(F(d == 2 ? pref : 1.0), F(PA - cq * PQ[d]), F(QC + cp * PQ[d]), F(B10), F(B01),
                                       F(B00), F(AB[d]), F(CD[d]));
                        }
                        const F fzb2 = F(zb2), fzc2 = F(zc2), fzd2 = F(zd2);
#pragma unroll
                        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                            for (int ib2 = 0; ib2 < NB; ++ib2)
#pragma unroll
                                for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                                    for (int id = 0; id < ND; ++id) {
                                        const int c = ((ia * NB + ib2) * NC + ic) * ND + id;
                                        const F gm = gam[c];
                                        F v[3], dB[3], dC[3], dD[3];
#pragma unroll
                                        for (int d = 0; d < 3; ++d) {
                                            const int i = kCart.v[LA][ia][d], j = kCart.v[LB][ib2][d];
                                            const int k = kCart.v[LC][ic][d], l = kCart.v[LD][id][d];
                                            const auto &X = g[d].X;
                                            v[d] = X[i][j][k][l];
                                            dB[d] = fzb2 * X[i][j + 1][k][l] - (j ? F(j) * X[i][j ? j - 1 : 0][k][l] : F(0));
                                            dC[d] = fzc2 * X[i][j][k + 1][l] - (k ? F(k) * X[i][j][k ? k - 1 : 0][l] : F(0));
                                            dD[d] = fzd2 * X[i][j][k][l + 1] - (l ? F(l) * X[i][j][k][l ? l - 1 : 0] : F(0));
                                        }
                                        const F gz = gm * v[2];
                                        const F tyz = gz * v[1], txz = gz * v[0], txy = gm * v[0] * v[1];
                                        pacc[0] += tyz * dB[0]; pacc[1] += txz * dB[1]; pacc[2] += txy * dB[2];
                                        pacc[3] += tyz * dC[0]; pacc[4] += txz * dC[1]; pacc[5] += txy * dC[2];
                                        pacc[6] += tyz * dD[0]; pacc[7] += txz * dD[1]; pacc[8] += txy * dD[2];
                                    }
                    } else if constexpr (MODE == 1) {
                        constexpr int NBASE = (LA + 1) * (LB + 1) * (LC + 1) * (LD + 1);
                        const double za = zab;
                        const DirectCoef dc = direct_coef(za, 0.5 * zb2, 0.5 * zc2, 0.5 * zd2, p, q, ip, iq, u, ipq, B10, B01, B00);
                        F T[3][4 * NBASE];
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double CA = (P[d] - A[d]) - cq * PQ[d], CB = CA + AB[d];
                            const double CCx = (Q[d] - Cc[d]) + cp * PQ[d], CDx = CCx + CD[d];
                            direct_tables<LA, LB, LC, LD, F>(T[d], F(d == 2 ? pref : 1.0), F(CA), F(CB), F(CCx), F(CDx),
                                                             F(B10), F(B01), F(B00), F(zb2 * CB), F(dc.e2), F(dc.e3),
                                                             F(dc.e4), F(zc2 * CCx), F(dc.f2), F(dc.f3), F(dc.f4),
                                                             F(zd2 * CDx), F(dc.g2), F(dc.g3), F(dc.g4));
                        }
#pragma unroll
                        for (int ia = 0; ia < NA; ++ia) {
#pragma unroll
                            for (int ib2 = 0; ib2 < NB; ++ib2) {
#pragma unroll
                                for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                                    for (int id = 0; id < ND; ++id) {
                                        const int c = ((ia * NB + ib2) * NC + ic) * ND + id;
                                        const F gm = gam[c];
                                        int e[3];
#pragma unroll
                                        for (int d = 0; d < 3; ++d)
                                            e[d] = ((kCart.v[LA][ia][d] * (LB + 1) + kCart.v[LB][ib2][d]) * (LC + 1) +
                                                    kCart.v[LC][ic][d]) * (LD + 1) + kCart.v[LD][id][d];
                                        const F vx = T[0][e[0]], vy = T[1][e[1]], vz = T[2][e[2]];
                                        const F gz = gm * vz;
                                        const F tyz = gz * vy, txz = gz * vx, txy = gm * vx * vy;
                                        pacc[0] += tyz * T[0][NBASE + e[0]]; pacc[3] += tyz * T[0][2 * NBASE + e[0]];
                                        pacc[6] += tyz * T[0][3 * NBASE + e[0]];
                                        pacc[1] += txz * T[1][NBASE + e[1]]; pacc[4] += txz * T[1][2 * NBASE + e[1]];
                                        pacc[7] += txz * T[1][3 * NBASE + e[1]];
                                        pacc[2] += txy * T[2][NBASE + e[2]]; pacc[5] += txy * T[2][2 * NBASE + e[2]];
                                        pacc[8] += txy * T[2][3 * NBASE + e[2]];
                                    }
                                // FP32 partial sums span at most a few dozen components
                                if constexpr (FLUSH == 2) flush(acc, pacc);
                            }
                            if constexpr (FLUSH == 1) flush(acc, pacc);
                        }
                    } else {
                        constexpr int NBASE = (LA + 1) * (LB + 1) * (LC + 1) * (LD + 1);
                        const double za = zab;
                        const DirectCoef dc = direct_coef(za, 0.5 * zb2, 0.5 * zc2, 0.5 * zd2, p, q, ip, iq, u, ipq, B10, B01, B00);
                        F I[3][NBASE], H[3][NBASE];
                        double CB[3], CCx[3], CDx[3];
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double CA = (P[d] - A[d]) - cq * PQ[d];
                            CB[d] = CA + AB[d];
                            CCx[d] = (Q[d] - Cc[d]) + cp * PQ[d];
                            CDx[d] = CCx[d] + CD[d];
                            direct_base<LA, LB, LC, LD, F>(I[d], F(d == 2 ? pref : 1.0), F(CA), F(CB[d]), F(CCx[d]),
                                                           F(CDx[d]), F(B10), F(B01), F(B00));
#pragma unroll
                            for (int e = 0; e < NBASE; ++e) H[d][e] = F(0);
                        }
#pragma unroll
                        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                            for (int ib2 = 0; ib2 < NB; ++ib2)
#pragma unroll
                                for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                                    for (int id = 0; id < ND; ++id) {
                                        const int c = ((ia * NB + ib2) * NC + ic) * ND + id;
                                        const F gm = gam[c];
                                        int e[3];
#pragma unroll
                                        for (int d = 0; d < 3; ++d)
                                            e[d] = ((kCart.v[LA][ia][d] * (LB + 1) + kCart.v[LB][ib2][d]) * (LC + 1) +
                                                    kCart.v[LC][ic][d]) * (LD + 1) + kCart.v[LD][id][d];
                                        const F vx = I[0][e[0]], vy = I[1][e[1]], vz = I[2][e[2]];
                                        const F gz = gm * vz;
                                        H[0][e[0]] += gz * vy;
                                        H[1][e[1]] += gz * vx;
                                        H[2][e[2]] += (gm * vx) * vy;
                                    }
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            double S[5];
                            collapse_sums<LA, LB, LC, LD, F>(H[d], I[d], S);
                            const double sij = S[1] + S[2], skl = S[3] + S[4];
                            acc[d] += zb2 * CB[d] * S[0] + dc.e2 * S[1] + dc.e3 * S[2] + dc.e4 * skl;
                            acc[3 + d] += zc2 * CCx[d] * S[0] + dc.f2 * S[3] + dc.f3 * S[4] + dc.f4 * sij;
                            acc[6 + d] += zd2 * CDx[d] * S[0] + dc.g2 * S[3] + dc.g3 * S[4] + dc.g4 * sij;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 9; ++k) acc[k] += double(pacc[k]);
                    } // roots of this lane
                    if constexpr (!K::EARLY_PREFETCH) {
                        // requested only after this primitive's contraction, so that the
                        // record does not hold registers across the contraction
                        asm volatile("" ::: "memory");
                        n0 = rk[4 * kn]; n1 = rk[4 * kn + 1]; n2 = rk[4 * kn + 2]; n3 = rk[4 * kn + 3];
                    }
                }
            }
        }
        double out[12];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            out[3 + d] = acc[d];
            out[6 + d] = acc[3 + d];
            out[9 + d] = acc[6 + d];
            out[d] = -(acc[d] + acc[3 + d] + acc[6 + d]); // translational invariance (eq ti)
        }
        if (a.task_out) {
            // per-quartet output: the team's lanes are summed in lane order (the same
            // order on every run), and the first lane of the team stores the twelve values
            const int lead = tw * TEAM;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                double v = __shfl(out[k], lead);
#pragma unroll
                for (int q = 1; q < TEAM; ++q) v += __shfl(out[k], lead + q);
                out[k] = v;
            }
            if (valid && r == 0) {
#pragma unroll
                for (int k = 0; k < 12; ++k) a.task_out[12 * t + k] = out[k];
            }
        } else if (valid) {
            {
                const int at[4] = {atA, atB, atC, atD};
#pragma unroll
                for (int X = 0; X < 4; ++X)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (a.lds_atoms) atomicAdd(&s_atoms[3 * at[X] + d], out[3 * X + d]);
                        else atomic_add_global(&M.grad[3 * at[X] + d], out[3 * X + d]);
                    }
            }
        }
        wave_sync();
    }
    if (a.lds_atoms) {
        // every wavefront's LDS additions (issued without return) land before the array is
        // read: the barrier alone does not order LDS operations of different wavefronts
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __syncthreads();
        for (int i = tid; i < 3 * a.n_atoms; i += blockDim.x) {
            const double v = s_atoms[i];
            if (v != 0.0) atomic_add_global(&a.grad[i], v);
        }
    }
}

} // namespace tdg
