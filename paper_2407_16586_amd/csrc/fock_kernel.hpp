// Two-electron part of the Fock-type matrix (section II.B, eqs G_2e and zfock):
// shell-quartet integrals by Rys quadrature over the direct four-centre base tables
// (deriv_kernel.hpp, without derivatives), contracted on the fly with a symmetric
// matrix B into Coulomb- and exchange-type blocks.
#pragma once
#include "deriv_kernel.hpp"

namespace tdg {

struct FockArgs {
    const double *coords;   // [n_atoms][3]
    const int *shell_atom;  // [n_shells]
    const int *shell_ao;    // [n_shells]
    const int *pair_sa, *pair_sb, *pair_ppoff, *pair_npp; // sorted shell pairs
    const double2 *pp_rec;  // per primitive pair, 4 x double2 (layout of DerivArgs)
    const double *bmat;     // shell-blocked records of (B + B^T)/2 with the angular factors
                            // folded in, in the first slot of the density record layout
    int n_bf;
    const int2 *tasks;      // (bra pair, ket pair) of this class
    long long ntasks;
    double omega;           // long-range kernel erf(omega r)/r
    double cJ, cK, cKlr;    // F = cJ J + cK K + cKlr K_lr
    double *G;              // [n_bf][n_bf] accumulator; F = ang (G + G^T) ang afterwards
};

// Group layout: G lanes per shell quartet, QPW quartets per wavefront.  For each primitive
// quartet, lane (slot, direction) of the group builds the base table of one Rys root of one
// kernel (slot = set * NR + root; set 1 is the long-range kernel) and direction into the
// group's LDS; the lanes then sum, for the components they own, the products of the three
// directions over all slots into registers.  After the last primitive quartet the contracted
// integrals go to LDS (over the tables), the six B blocks beside them, and the lanes form the
// six output blocks, one element each at a time, with one global atomic add per element.
template <int LA, int LB, int LC, int LD, bool LR>
struct FockClass {
    static constexpr int L = LA + LB + LC + LD;
    static constexpr int NR = L / 2 + 1;          // Rys roots of total momentum L (no derivative)
    static constexpr int NSET = LR ? 2 : 1;
    static constexpr int NSLOT = NR * NSET;
    static constexpr int JOBS = 3 * NSLOT;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int N = NA * NB * NC * ND;
    static constexpr int NBASE = (LA + 1) * (LB + 1) * (LC + 1) * (LD + 1);
    static constexpr int pow2ceil(int x)
    {
        int p = 1;
        while (p < x) p *= 2;
        return p;
    }
    static constexpr int max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }
    static constexpr int GR = pow2ceil(max3(JOBS, (N + 7) / 8, 4));
    static constexpr int G = GR < kWave ? GR : kWave;
    static constexpr int QPW = kWave / G;
    static constexpr int CPL = (N + G - 1) / G;   // components per lane
    static constexpr int TABN = NSLOT * 3 * NBASE;
    static constexpr int VN = 2 * N;              // J-weighted and K-weighted contracted integrals
    static constexpr int UN = TABN > VN ? TABN : VN;
    // six B blocks, in the order the output blocks J_ab J_cd K_ac K_ad K_bc K_bd read them
    static constexpr int OB_CD = 0, OB_AB = NC * ND, OB_BD = OB_AB + NA * NB, OB_BC = OB_BD + NB * ND,
                         OB_AD = OB_BC + NB * NC, OB_AC = OB_AD + NA * ND, SB = OB_AC + NA * NC;
    static constexpr int GSTRIDE = UN + SB + 1;
    // Rys table of the class in LDS when it fits beside the groups (n <= 3 roots)
    static constexpr bool TAB_LDS = NR <= 3;
    static constexpr int TAB_N = TAB_LDS ? rys_table_size<NR>() : 1;
    static constexpr int WAVES = 2;
    static constexpr int QPB = QPW * WAVES;
    static constexpr int BLOCK = WAVES * kWave;
    static_assert(JOBS <= G, "one table job per lane");
};

template <int LA, int LB, int LC, int LD, bool LR>
__global__ void __launch_bounds__((FockClass<LA, LB, LC, LD, LR>::BLOCK)) k_fock(const FockArgs a)
{
    using K = FockClass<LA, LB, LC, LD, LR>;
    constexpr int NR = K::NR, G = K::G, QPW = K::QPW, QPB = K::QPB, CPL = K::CPL;
    constexpr int NA = K::NA, NB = K::NB, NC = K::NC, ND = K::ND, N = K::N, NBASE = K::NBASE;
    __shared__ double s_buf[QPB * K::GSTRIDE];
    __shared__ double s_rys[K::TAB_N];
    if constexpr (K::TAB_LDS) {
        rys_table_to_lds<NR>(s_rys);
        __syncthreads();
    }

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int grp = lane / G, t = lane % G;
    const int q = wave * QPW + grp;
    double *tab = s_buf + q * K::GSTRIDE; // tables, then the contracted integrals
    double *bs = tab + K::UN;             // B blocks
    // base-table indices (x, y, z packed by 8 bits) of the components this lane owns
    int epk[CPL];
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
        const int c = t + m * G;
        int e = 0;
        if (c < N) {
            const int id = c % ND, ic = (c / ND) % NC, ib = (c / (ND * NC)) % NB, ia = c / (ND * NC * NB);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int ex = ((kCart.v[LA][ia][d] * (LB + 1) + kCart.v[LB][ib][d]) * (LC + 1) + kCart.v[LC][ic][d]) *
                                   (LD + 1) + kCart.v[LD][id][d];
                e |= ex << (8 * d);
            }
        }
        epk[m] = e;
    }
    // table job of this lane
    const bool job = t < K::JOBS;
    const int jslot = job ? t / 3 : 0, jdir = t % 3;
    const int jset = jslot / NR, jroot = jslot % NR;
    const double iom2 = LR ? 1.0 / (a.omega * a.omega) : 0.0;
    const bool doJ = a.cJ != 0.0, doK = a.cK != 0.0 || (LR && a.cKlr != 0.0);

    const long long stride = (long long)gridDim.x * QPB;
    for (long long base = (long long)blockIdx.x * QPB; base < a.ntasks; base += stride) {
        const long long ti = base + q;
        const bool valid = (grp < QPW) && ti < a.ntasks; // uniform within the group
        double acc[2][CPL];
#pragma unroll
        for (int m = 0; m < CPL; ++m) acc[0][m] = acc[1][m] = 0.0;
        int sa = 0, sb = 0, sc = 0, sd = 0, bra = 0, ket = 0;
        if (valid) {
            const int2 tk = a.tasks[ti];
            bra = tk.x;
            ket = tk.y;
            sa = a.pair_sa[bra]; sb = a.pair_sb[bra];
            sc = a.pair_sa[ket]; sd = a.pair_sb[ket];
            const int atA = a.shell_atom[sa], atB = a.shell_atom[sb], atC = a.shell_atom[sc], atD = a.shell_atom[sd];
            const double Ad = a.coords[3 * atA + jdir], ABd = Ad - a.coords[3 * atB + jdir];
            const double Cd = a.coords[3 * atC + jdir], CDd = Cd - a.coords[3 * atD + jdir];
            const int pb0 = a.pair_ppoff[bra], nbp = a.pair_npp[bra];
            const int pk0 = a.pair_ppoff[ket], nkp = a.pair_npp[ket];
            const double2 *rb = a.pp_rec + 4 * (size_t)pb0, *rk = a.pp_rec + 4 * (size_t)pk0;
            for (int ib = 0; ib < nbp; ++ib) {
                const double2 b0 = rb[4 * ib], b1 = rb[4 * ib + 1], b2 = rb[4 * ib + 2], b3 = rb[4 * ib + 3];
                const double p = b0.x, ip = b0.y;
                const double cab = 34.98683665524972 * b1.x * ip; // 2 pi^(5/2) c_ab / p
                const double P[3] = {b2.y, b3.x, b3.y};
                // next ket record requested one primitive ahead
                double2 n0 = rk[0], n1 = rk[1], n2 = rk[2], n3 = rk[3];
                for (int ik = 0; ik < nkp; ++ik) {
                    const double2 k0 = n0, k1 = n1, k2 = n2, k3 = n3;
                    const int kn = ik + 1 < nkp ? ik + 1 : ik;
                    n0 = rk[4 * kn]; n1 = rk[4 * kn + 1]; n2 = rk[4 * kn + 2]; n3 = rk[4 * kn + 3];
                    if (job) {
                        const double qq = k0.x, iq = k0.y, ccd = k1.x;
                        const double Q[3] = {k2.y, k3.x, k3.y};
                        const double sipq = rsq64(p + qq), ipq = sipq * sipq;
                        const double rho = p * qq * ipq;
                        double pq2 = 0.0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) pq2 += (P[d] - Q[d]) * (P[d] - Q[d]);
                        double Tr = rho * pq2, eta = 1.0, seta = 1.0;
                        if (LR && jset) {
                            seta = rsq64(1.0 + rho * iom2); // sqrt(omega^2 / (omega^2 + rho))
                            eta = seta * seta;
                            Tr *= eta;
                        }
                        double u, w;
                        if constexpr (K::TAB_LDS) rys_root_lds<NR>(s_rys, Tr, jroot, u, w);
                        else rys_root<NR>(Tr, jroot, u, w);
                        if (LR && jset) {
                            u *= eta;
                            w *= seta;
                        }
                        const double B00 = 0.5 * u * ipq;
                        const double B10 = 0.5 * ip * (1.0 - qq * ipq * u);
                        const double B01 = 0.5 * iq * (1.0 - p * ipq * u);
                        const double cq = qq * ipq * u, cp = p * ipq * u;
                        const double PQd = P[jdir] - Q[jdir];
                        const double CA = (P[jdir] - Ad) - cq * PQd, CB = CA + ABd;
                        const double CC = (Q[jdir] - Cd) + cp * PQd, CDx = CC + CDd;
                        const double I0 = jdir == 2 ? cab * (ccd * iq) * sipq * w : 1.0;
                        // built in place in LDS (a register copy of the largest tables would
                        // spill beside the accumulators)
                        direct_base<LA, LB, LC, LD, double>(tab + (jslot * 3 + jdir) * NBASE, I0, CA, CB, CC, CDx,
                                                            B10, B01, B00);
                    }
                    wave_sync();
                    // the roots of each kernel in a rolled loop (unrolled, the largest classes
                    // spill the accumulators)
#pragma unroll
                    for (int set = 0; set < K::NSET; ++set) {
#pragma unroll 1
                        for (int s = set * NR; s < set * NR + NR; ++s) {
                            const double *tx = tab + s * 3 * NBASE, *ty = tx + NBASE, *tz = ty + NBASE;
#pragma unroll
                            for (int m = 0; m < CPL; ++m) {
                                if (m < CPL - 1 || t + m * G < N) {
                                    const int e = epk[m];
                                    acc[set][m] += tx[e & 255] * ty[(e >> 8) & 255] * tz[e >> 16];
                                }
                            }
                        }
                    }
                    wave_sync();
                }
            }
        }
        const double deg = (sa != sb ? 2.0 : 1.0) * (sc != sd ? 2.0 : 1.0) * (bra != ket ? 2.0 : 1.0);
        const double wJ = 0.25 * deg * a.cJ, wK = 0.125 * deg;
        const int oa = valid ? a.shell_ao[sa] : 0, ob = valid ? a.shell_ao[sb] : 0;
        const int oc = valid ? a.shell_ao[sc] : 0, od = valid ? a.shell_ao[sd] : 0;
        if (valid) {
#pragma unroll
            for (int m = 0; m < CPL; ++m) {
                const int c = t + m * G;
                if (c < N) {
                    tab[c] = wJ * acc[0][m];
                    tab[N + c] = wK * (a.cK * acc[0][m] + (LR ? a.cKlr * acc[1][m] : 0.0));
                }
            }
            const int n = a.n_bf;
            for (int x = t; x < K::SB; x += G) {
                int o1, n1, o2, el; // element el of the record of the ordered pair (o1, o2), n1 rows
                if (x < K::OB_AB) { o1 = oc; n1 = NC; o2 = od; el = x - K::OB_CD; }
                else if (x < K::OB_BD) { o1 = oa; n1 = NA; o2 = ob; el = x - K::OB_AB; }
                else if (x < K::OB_BC) { o1 = ob; n1 = NB; o2 = od; el = x - K::OB_BD; }
                else if (x < K::OB_AD) { o1 = ob; n1 = NB; o2 = oc; el = x - K::OB_BC; }
                else if (x < K::OB_AC) { o1 = oa; n1 = NA; o2 = od; el = x - K::OB_AD; }
                else { o1 = oa; n1 = NA; o2 = oc; el = x - K::OB_AC; }
                bs[x] = a.bmat[dens_rec(n, o1, n1, o2) + el];
            }
        }
        wave_sync();
        if (valid) {
            const int n = a.n_bf;
            const double *vJ = tab, *vK = tab + N;
#define V_(i, j, k, l) ((((i) * NB + (j)) * NC + (k)) * ND + (l))
            for (int o = t; o < K::SB; o += G) {
                double s = 0.0;
                size_t dst;
                if (o < NA * NB) { // J_ab[i][j] = sum_kl v B_cd[k][l]
                    if (!doJ) continue;
                    const int i = o / NB, j = o % NB;
                    for (int k = 0; k < NC; ++k)
                        for (int l = 0; l < ND; ++l) s += vJ[V_(i, j, k, l)] * bs[K::OB_CD + k * ND + l];
                    dst = (size_t)(oa + i) * n + ob + j;
                } else if (o < NA * NB + NC * ND) { // J_cd[k][l] = sum_ij v B_ab[i][j]
                    if (!doJ) continue;
                    const int x = o - NA * NB, k = x / ND, l = x % ND;
                    for (int i = 0; i < NA; ++i)
                        for (int j = 0; j < NB; ++j) s += vJ[V_(i, j, k, l)] * bs[K::OB_AB + i * NB + j];
                    dst = (size_t)(oc + k) * n + od + l;
                } else if (o < NA * NB + NC * ND + NA * NC) { // K_ac[i][k] = sum_jl v B_bd[j][l]
                    if (!doK) continue;
                    const int x = o - NA * NB - NC * ND, i = x / NC, k = x % NC;
                    for (int j = 0; j < NB; ++j)
                        for (int l = 0; l < ND; ++l) s += vK[V_(i, j, k, l)] * bs[K::OB_BD + j * ND + l];
                    dst = (size_t)(oa + i) * n + oc + k;
                } else if (o < NA * NB + NC * ND + NA * NC + NA * ND) { // K_ad[i][l] = sum_jk v B_bc[j][k]
                    if (!doK) continue;
                    const int x = o - NA * NB - NC * ND - NA * NC, i = x / ND, l = x % ND;
                    for (int j = 0; j < NB; ++j)
                        for (int k = 0; k < NC; ++k) s += vK[V_(i, j, k, l)] * bs[K::OB_BC + j * NC + k];
                    dst = (size_t)(oa + i) * n + od + l;
                } else if (o < NA * NB + NC * ND + NA * NC + NA * ND + NB * NC) { // K_bc[j][k] = sum_il v B_ad[i][l]
                    if (!doK) continue;
                    const int x = o - NA * NB - NC * ND - NA * NC - NA * ND, j = x / NC, k = x % NC;
                    for (int i = 0; i < NA; ++i)
                        for (int l = 0; l < ND; ++l) s += vK[V_(i, j, k, l)] * bs[K::OB_AD + i * ND + l];
                    dst = (size_t)(ob + j) * n + oc + k;
                } else { // K_bd[j][l] = sum_ik v B_ac[i][k]
                    if (!doK) continue;
                    const int x = o - NA * NB - NC * ND - NA * NC - NA * ND - NB * NC, j = x / ND, l = x % ND;
                    for (int i = 0; i < NA; ++i)
                        for (int k = 0; k < NC; ++k) s += vK[V_(i, j, k, l)] * bs[K::OB_AC + i * NC + k];
                    dst = (size_t)(ob + j) * n + od + l;
                }
                if (s != 0.0) atomic_add_global(a.G + dst, s);
            }
#undef V_
        }
        wave_sync(); // the next quartet's tables overwrite this one's integrals
    }
}

// Lane layout for the classes with few components: one lane per shell quartet (N <= 27)
// evaluates every root of both kernels with its base tables in registers, keeps the N
// contracted integrals of each kernel in registers, and forms the six output blocks
// itself (compile-time indices throughout); the Rys table of the class sits in LDS.  No
// wavefront synchronisation inside the task loop.  PAIR (long-range classes with
// 27 < N <= 54): two neighbouring lanes per quartet, one per kernel (full range, long
// range), so that each holds N integrals; they exchange them once, and the first forms the
// Coulomb blocks, the second the exchange blocks.
template <int LA, int LB, int LC, int LD, bool LR, bool PAIR = false>
struct FockLane {
    static constexpr int L = LA + LB + LC + LD;
    static constexpr int NR = L / 2 + 1;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int N = NA * NB * NC * ND;
    static constexpr int NBASE = (LA + 1) * (LB + 1) * (LC + 1) * (LD + 1);
    static constexpr bool TAB_LDS = NR <= 3;
    static constexpr int TAB_N = TAB_LDS ? rys_table_size<NR>() : 1;
    static constexpr int BLOCK = 128;
    static constexpr int LPQ = PAIR ? 2 : 1;          // lanes per quartet
    static constexpr int QPB = BLOCK / LPQ;           // quartets per block and round
    static constexpr int NV = (LR && !PAIR) ? 2 : 1;  // kernels a lane accumulates
    static_assert(!PAIR || LR, "the paired layout splits the two kernels");
};

template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ constexpr int fock_e(int c, int d)
{
    constexpr int NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    const int id = c % ND, ic = (c / ND) % NC, ib = (c / (ND * NC)) % NB, ia = c / (ND * NC * NB);
    return ((kCart.v[LA][ia][d] * (LB + 1) + kCart.v[LB][ib][d]) * (LC + 1) + kCart.v[LC][ic][d]) * (LD + 1) +
           kCart.v[LD][id][d];
}

// The six output blocks of one quartet from its contracted integrals v0 (full range) and v1
// (long range; read only when LR) into G with FP64 atomics.  Every lane of the wavefront
// calls it; wave_j (uniform) enables the Coulomb part, cj says whether this lane forms the
// Coulomb blocks, ck the exchange blocks.  J_ab is first summed over the wavefront when its
// lanes share the bra pair (the tasks of a class are ordered by bra pair, so one atomic
// replaces up to 64 on one address).
template <int LA, int LB, int LC, int LD, bool LR>
__device__ __forceinline__ void fock_lane_out(const FockArgs &a, bool valid, int bra, int ket, int sa, int sb, int sc,
                                              int sd, bool cj, bool ck, bool wave_j, const double *v0,
                                              const double *v1)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    const double deg = (sa != sb ? 2.0 : 1.0) * (sc != sd ? 2.0 : 1.0) * (bra != ket ? 2.0 : 1.0);
    const double wJ = 0.25 * deg * a.cJ, wK = 0.125 * deg;
    const int n = a.n_bf;
    const int oa = a.shell_ao[sa], ob = a.shell_ao[sb], oc = a.shell_ao[sc], od = a.shell_ao[sd];
    const double *Bcd = a.bmat + dens_rec(n, oc, NC, od), *Bab = a.bmat + dens_rec(n, oa, NA, ob);
    const double *Bbd = a.bmat + dens_rec(n, ob, NB, od), *Bbc = a.bmat + dens_rec(n, ob, NB, oc);
    const double *Bad = a.bmat + dens_rec(n, oa, NA, od), *Bac = a.bmat + dens_rec(n, oa, NA, oc);
    const bool jl = valid && cj;
#define V_(i, j, k, l) ((((i) * NB + (j)) * NC + (k)) * ND + (l))
#define KV_(x) (a.cK * v0[x] + (LR ? a.cKlr * v1[x] : 0.0))
    if (wave_j) {
        const int bra0 = __shfl(bra, 0);
        const bool same_bra = __all(!jl || bra == bra0);
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int l = 0; l < ND; ++l) s += v0[V_(i, j, k, l)] * Bcd[k * ND + l];
                s = jl ? wJ * s : 0.0;
                if (same_bra) {
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
                    if ((threadIdx.x & (kWave - 1)) == 0 && s != 0.0)
                        atomic_add_global(a.G + (size_t)(oa + i) * n + ob + j, s);
                } else if (s != 0.0) {
                    atomic_add_global(a.G + (size_t)(oa + i) * n + ob + j, s);
                }
            }
        if (jl) {
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int j = 0; j < NB; ++j) s += v0[V_(i, j, k, l)] * Bab[i * NB + j];
                    if (s != 0.0) atomic_add_global(a.G + (size_t)(oc + k) * n + od + l, wJ * s);
                }
        }
    }
    if (ck && valid) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int k = 0; k < NC; ++k) { // K_ac
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int l = 0; l < ND; ++l) s += KV_(V_(i, j, k, l)) * Bbd[j * ND + l];
                if (s != 0.0) atomic_add_global(a.G + (size_t)(oa + i) * n + oc + k, wK * s);
            }
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int l = 0; l < ND; ++l) { // K_ad
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int k = 0; k < NC; ++k) s += KV_(V_(i, j, k, l)) * Bbc[j * NC + k];
                if (s != 0.0) atomic_add_global(a.G + (size_t)(oa + i) * n + od + l, wK * s);
            }
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int k = 0; k < NC; ++k) { // K_bc
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int l = 0; l < ND; ++l) s += KV_(V_(i, j, k, l)) * Bad[i * ND + l];
                if (s != 0.0) atomic_add_global(a.G + (size_t)(ob + j) * n + oc + k, wK * s);
            }
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int l = 0; l < ND; ++l) { // K_bd
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int k = 0; k < NC; ++k) s += KV_(V_(i, j, k, l)) * Bac[i * NC + k];
                if (s != 0.0) atomic_add_global(a.G + (size_t)(ob + j) * n + od + l, wK * s);
            }
    }
#undef KV_
#undef V_
}

template <int LA, int LB, int LC, int LD, bool LR, bool PAIR = false>
__global__ void __launch_bounds__(128) k_fock_lane(const FockArgs a)
{
    using K = FockLane<LA, LB, LC, LD, LR, PAIR>;
    constexpr int NR = K::NR, N = K::N, NBASE = K::NBASE, NV = K::NV;
    constexpr int NA = K::NA, NB = K::NB, NC = K::NC, ND = K::ND;
    __shared__ double s_rys[K::TAB_N];
    if constexpr (K::TAB_LDS) {
        rys_table_to_lds<NR>(s_rys);
        __syncthreads();
    }
    const double iom2 = LR ? 1.0 / (a.omega * a.omega) : 0.0;
    const bool doJ = a.cJ != 0.0, doK = a.cK != 0.0 || (LR && a.cKlr != 0.0);
    // PAIR: the odd lane of a pair evaluates the long-range kernel and forms the exchange blocks
    const int half = PAIR ? (int)(threadIdx.x & 1) : 0;
    const bool jrole = !PAIR || half == 0, krole = !PAIR || half == 1;
    const long long stride = (long long)gridDim.x * K::QPB;
    // every lane of a block takes the same number of rounds (the J_ab reduction below is a
    // wavefront operation); lanes past the end carry no task
    for (long long t0 = (long long)blockIdx.x * K::QPB; t0 < a.ntasks; t0 += stride) {
        const long long ti = t0 + threadIdx.x / K::LPQ;
        const bool valid = ti < a.ntasks;
        const int2 tk = a.tasks[valid ? ti : a.ntasks - 1];
        const int bra = tk.x, ket = tk.y;
        const int sa = a.pair_sa[bra], sb = a.pair_sb[bra], sc = a.pair_sa[ket], sd = a.pair_sb[ket];
        const int atA = a.shell_atom[sa], atB = a.shell_atom[sb], atC = a.shell_atom[sc], atD = a.shell_atom[sd];
        double A[3], AB[3], Cc[3], CD[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[d] = a.coords[3 * atA + d];
            AB[d] = A[d] - a.coords[3 * atB + d];
            Cc[d] = a.coords[3 * atC + d];
            CD[d] = Cc[d] - a.coords[3 * atD + d];
        }
        double v[NV][N];
#pragma unroll
        for (int x = 0; x < NV; ++x)
#pragma unroll
            for (int c = 0; c < N; ++c) v[x][c] = 0.0;
        const int pb0 = a.pair_ppoff[bra], nbp = valid ? a.pair_npp[bra] : 0;
        const int pk0 = a.pair_ppoff[ket], nkp = a.pair_npp[ket];
        const double2 *rb = a.pp_rec + 4 * (size_t)pb0, *rk = a.pp_rec + 4 * (size_t)pk0;
        for (int ib = 0; ib < nbp; ++ib) {
            const double2 b0 = rb[4 * ib], b1 = rb[4 * ib + 1], b2 = rb[4 * ib + 2], b3 = rb[4 * ib + 3];
            const double p = b0.x, ip = b0.y;
            const double cab = 34.98683665524972 * b1.x * ip; // 2 pi^(5/2) c_ab / p
            const double P[3] = {b2.y, b3.x, b3.y};
            // ket record of the current primitive; the next one is requested before the
            // current one's work so that its latency is hidden behind it
            double2 n0 = rk[0], n1 = rk[1], n2 = rk[2], n3 = rk[3];
            for (int ik = 0; ik < nkp; ++ik) {
                const double2 k0 = n0, k1 = n1, k2 = n2, k3 = n3;
                const int kn = ik + 1 < nkp ? ik + 1 : ik;
                n0 = rk[4 * kn]; n1 = rk[4 * kn + 1]; n2 = rk[4 * kn + 2]; n3 = rk[4 * kn + 3];
                const double qq = k0.x, iq = k0.y, ccd = k1.x;
                const double Q[3] = {k2.y, k3.x, k3.y};
                const double sipq = rsq64(p + qq), ipq = sipq * sipq;
                const double rho = p * qq * ipq;
                double PQ[3], pq2 = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    PQ[d] = P[d] - Q[d];
                    pq2 += PQ[d] * PQ[d];
                }
                const double base_pref = cab * (ccd * iq) * sipq;
#pragma unroll
                for (int x = 0; x < NV; ++x) {
                    const bool lr_set = PAIR ? half == 1 : (LR && x == 1);
                    double Tr = rho * pq2, eta = 1.0, seta = 1.0;
                    if (lr_set) {
                        seta = rsq64(1.0 + rho * iom2); // sqrt(omega^2 / (omega^2 + rho))
                        eta = seta * seta;
                        Tr *= eta;
                    }
#pragma unroll 1
                    for (int r = 0; r < NR; ++r) {
                        double u, w;
                        if constexpr (K::TAB_LDS) rys_root_lds<NR>(s_rys, Tr, r, u, w);
                        else rys_root<NR>(Tr, r, u, w);
                        if (lr_set) {
                            u *= eta;
                            w *= seta;
                        }
                        const double B00 = 0.5 * u * ipq;
                        const double B10 = 0.5 * ip * (1.0 - qq * ipq * u);
                        const double B01 = 0.5 * iq * (1.0 - p * ipq * u);
                        const double cq = qq * ipq * u, cp = p * ipq * u;
                        double I[3][NBASE];
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double CA = (P[d] - A[d]) - cq * PQ[d], CB = CA + AB[d];
                            const double CCx = (Q[d] - Cc[d]) + cp * PQ[d], CDx = CCx + CD[d];
                            direct_base<LA, LB, LC, LD, double>(I[d], d == 2 ? base_pref * w : 1.0, CA, CB, CCx, CDx,
                                                                B10, B01, B00);
                        }
#pragma unroll
                        for (int c = 0; c < N; ++c)
                            v[x][c] += I[0][fock_e<LA, LB, LC, LD>(c, 0)] * I[1][fock_e<LA, LB, LC, LD>(c, 1)] *
                                       I[2][fock_e<LA, LB, LC, LD>(c, 2)];
                    }
                }
            }
        }
        if constexpr (PAIR) {
            // the pair's lanes swap their integrals: afterwards v[0] holds the full-range and
            // v1 the long-range ones on the exchange lane (the Coulomb lane needs v[0] only)
            double o[N];
#pragma unroll
            for (int c = 0; c < N; ++c) o[c] = __shfl_xor(v[0][c], 1);
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const double mine = v[0][c];
                v[0][c] = half ? o[c] : mine;
                o[c] = half ? mine : 0.0;
            }
            fock_lane_out<LA, LB, LC, LD, LR>(a, valid, bra, ket, sa, sb, sc, sd, jrole, krole && doK, doJ, v[0], o);
        } else {
            fock_lane_out<LA, LB, LC, LD, LR>(a, valid, bra, ket, sa, sb, sc, sd, true, doK, doJ, v[0], v[NV - 1]);
        }
    }
}

} // namespace tdg
