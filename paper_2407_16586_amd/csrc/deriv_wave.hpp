// Wavefront-per-quartet ERI-derivative kernels for the high angular-momentum
// classes (section II.C, eqs deriv, deri, ti, eriupdate).
//
// One wavefront evaluates one shell quartet.  For each primitive quartet the
// Rys root slots (n full-range + n long-range) are processed in chunks:
//   stage 1: lane (slot, direction) evaluates the root and the direct
//            four-centre recurrence and writes derivative-ready 2D tables to
//            LDS: for every index quadruple (i<=la, j<=lb, k<=lc, l<=ld) the
//            integral G and its B, C, D derivatives;
//   stage 2: lanes split the Cartesian components; each lane reads the
//            symmetrised Gamma of its components (written to LDS once per
//            quartet) and 12 table values per component and root.
// The A derivative follows from translational invariance.
#pragma once
#include "deriv_kernel.hpp"

namespace tdg {

template <int LA, int LB, int LC, int LD, bool LR, typename F = double>
struct WaveClass {
    static constexpr int L = LA + LB + LC + LD;
    static constexpr int NR = nroots_deriv(L);
    static constexpr int NSET = LR ? 2 : 1;
    static constexpr int NSLOT = NR * NSET;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int N = NA * NB * NC * ND;
    static constexpr int NBASE = (LA + 1) * (LB + 1) * (LC + 1) * (LD + 1);
    static constexpr int TAB = 12 * NBASE;               // doubles per slot (3 dirs x 4 kinds)
    static constexpr int FB = (int)sizeof(F);
    // LDS for the root-slot tables of one wavefront: 14 KB, or 40 KB for the classes with
    // large tables (at least 36 base entries: d on three centres), where 14 KB holds only one
    // or two slots and leaves stage 1 with a handful of active lanes per chunk
    static constexpr int TAB_BUDGET = NBASE >= 36 ? 40 * 1024 : 14 * 1024;
    static constexpr int CH_LDS = TAB_BUDGET / (TAB * FB) > 0 ? TAB_BUDGET / (TAB * FB) : 1;
    static constexpr int CH0 = CH_LDS < NSLOT ? CH_LDS : NSLOT;
    static constexpr int CH = CH0 * 3 <= kWave ? CH0 : kWave / 3;
    static constexpr int NCHUNK = (NSLOT + CH - 1) / CH;
    static constexpr int GN = LR ? 2 * N : N;            // symmetrised Gamma (and Gamma^lr) of the quartet
    static constexpr int WAVE_LDS = CH * TAB + GN;       // elements per wave
    static constexpr int WAVES = WAVE_LDS * FB * 4 <= 64 * 1024 ? 4 : (WAVE_LDS * FB * 2 <= 64 * 1024 ? 2 : 1);
    static constexpr int BLOCK = WAVES * kWave;
    static constexpr int CPL = (N + kWave - 1) / kWave;  // components per lane
    static constexpr bool EARLY_PREFETCH = N <= 27;      // next ket record loaded ahead
};

template <int LA, int LB, int LC, int LD, bool LR, typename F>
__global__ void __launch_bounds__((WaveClass<LA, LB, LC, LD, LR, F>::BLOCK))
k_deriv_wave(const DerivArgs a)
{
    using K = WaveClass<LA, LB, LC, LD, LR, F>;
    constexpr int NR = K::NR, NSLOT = K::NSLOT, CH = K::CH, NCHUNK = K::NCHUNK, CPL = K::CPL;
    constexpr int NB = K::NB, NC = K::NC, ND = K::ND, N = K::N, NBASE = K::NBASE, TAB = K::TAB;
    extern __shared__ double s_atoms[];
    __shared__ F s_tab[K::WAVES * K::WAVE_LDS];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    F *tab = s_tab + wave * K::WAVE_LDS;
    F *sg = tab + CH * TAB; // Gamma of the wavefront's quartet, Gamma^lr behind it
    // block-level accumulation in LDS
    const bool use_lds = a.lds_atoms;
    if (use_lds) {
        for (int i = tid; i < 3 * a.n_atoms; i += blockDim.x) s_atoms[i] = 0.0;
        __syncthreads();
    }
    // this lane's components: table offsets per direction
    int eoff[CPL][3];
    bool cok[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int c = lane + q * kWave;
        cok[q] = c < N;
        const int cc = cok[q] ? c : 0;
        const int id = cc % ND, ic = (cc / ND) % NC, ib = (cc / (ND * NC)) % NB, ia = cc / (ND * NC * NB);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int i = kCart.v[LA][ia][d], j = kCart.v[LB][ib][d], k = kCart.v[LC][ic][d], l = kCart.v[LD][id][d];
            eoff[q][d] = d * 4 * NBASE + ((i * (LB + 1) + j) * (LC + 1) + k) * (LD + 1) + l;
        }
    }
    const double iom2 = LR ? 1.0 / (a.omega * a.omega) : 0.0;
    const long long wstride = (long long)gridDim.x * K::WAVES;
    for (long long t = (long long)blockIdx.x * K::WAVES + wave; t < a.ntasks; t += wstride) {
        const DerivArgs &M = a;
        const int2 tk = a.tasks[t];
        const int bra = tk.x, ket = tk.y;
        const int sa = M.pair_sa[bra], sb = M.pair_sb[bra], sc = M.pair_sa[ket], sd = M.pair_sb[ket];
        const double deg = (sa != sb ? 2.0 : 1.0) * (sc != sd ? 2.0 : 1.0) * (bra != ket ? 2.0 : 1.0);
        const int oa = M.shell_ao[sa], ob = M.shell_ao[sb], oc = M.shell_ao[sc], od = M.shell_ao[sd];
        // the quartet's symmetrised Gamma goes to LDS (in registers it would hold two values
        // per component for the whole task beside the tables' addresses; the largest
        // classes then spill)
        size_t rec[12];
        pair_records<LA, LB, LC, LD>(M.n_bf, oa, ob, oc, od, rec);
#pragma unroll 1
        for (int c = lane; c < N; c += kWave) {
            const int id = c % ND, ic = (c / ND) % NC, ib = (c / (ND * NC)) % NB, ia = c / (ND * NC * NB);
            double gf, gl;
            gamma_sym<LA, LB, LC, LD>(M, rec, ia, ib, ic, id, deg, gf, gl);
            sg[c] = F(gf);
            if constexpr (LR) sg[N + c] = F(gl);
        }
        const int atA = M.shell_atom[sa], atB = M.shell_atom[sb], atC = M.shell_atom[sc], atD = M.shell_atom[sd];
        // stage-1 lane role
        const int s1 = lane / 3, d1 = lane % 3;
        double Ad = 0.0, ABd = 0.0, Cd = 0.0, CDd = 0.0;
        if (s1 < CH) {
            Ad = M.coords[3 * atA + d1];
            ABd = Ad - M.coords[3 * atB + d1];
            Cd = M.coords[3 * atC + d1];
            CDd = Cd - M.coords[3 * atD + d1];
        }
        double acc[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        const int pb0 = M.pair_ppoff[bra], nbp = M.pair_npp[bra];
        const int pk0 = M.pair_ppoff[ket], nkp = M.pair_npp[ket];
        // primitive-pair records (p, 1/p) (c, za) (zb, P); in the classes with few
        // components the ket record of the next primitive quartet is requested while the
        // current one is evaluated (elsewhere the extra live registers cost occupancy)
        const double2 *rb = M.pp_rec + 4 * (size_t)pb0, *rk = M.pp_rec + 4 * (size_t)pk0;
        double2 n0, n1, n2, n3, c0, c1, c2, c3;
        if constexpr (K::EARLY_PREFETCH) {
            n0 = rk[0]; n1 = rk[1]; n2 = rk[2]; n3 = rk[3];
        }
        for (int ib = 0; ib < nbp; ++ib) {
            for (int ik = 0; ik < nkp; ++ik) {
                if constexpr (K::EARLY_PREFETCH) {
                    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
                    const int kn = ik + 1 < nkp ? ik + 1 : 0;
                    n0 = rk[4 * kn]; n1 = rk[4 * kn + 1]; n2 = rk[4 * kn + 2]; n3 = rk[4 * kn + 3];
                }
                for (int ch = 0; ch < NCHUNK; ++ch) {
                    const int slot = ch * CH + s1;
                    if (s1 < CH && slot < NSLOT) {
                        const double2 b0 = rb[4 * ib], b1 = rb[4 * ib + 1], b2 = rb[4 * ib + 2], b3 = rb[4 * ib + 3];
                        double2 k0, k1, k2, k3;
                        if constexpr (K::EARLY_PREFETCH) {
                            k0 = c0; k1 = c1; k2 = c2; k3 = c3;
                        } else {
                            k0 = rk[4 * ik]; k1 = rk[4 * ik + 1]; k2 = rk[4 * ik + 2]; k3 = rk[4 * ik + 3];
                        }
                        const double p = b0.x, ip = b0.y, cab = b1.x;
                        const double zb2 = 2.0 * b2.x;
                        const double q = k0.x, iq = k0.y, ccd = k1.x;
                        const double zc2 = 2.0 * k1.y, zd2 = 2.0 * k2.x;
                        const double P[3] = {b2.y, b3.x, b3.y};
                        const double Q[3] = {k2.y, k3.x, k3.y};
                        const double sipq = rsq64(p + q), ipq = sipq * sipq, rho = p * q * ipq;
                        const double PQ0 = P[0] - Q[0], PQ1 = P[1] - Q[1], PQ2 = P[2] - Q[2];
                        const double pq2 = PQ0 * PQ0 + PQ1 * PQ1 + PQ2 * PQ2;
                        const int set = slot / NR, ir = slot % NR;
                        double Tr = rho * pq2, eta = 1.0, seta = 1.0;
                        if (LR && set) {
                            seta = rsq64(1.0 + rho * iom2); // sqrt(omega^2 / (omega^2 + rho))
                            eta = seta * seta;
                            Tr *= eta;
                        }
                        double u, w;
                        rys_root<NR>(Tr, ir, u, w);
                        if (LR && set) {
                            u *= eta;
                            w *= seta;
                        }
                        const double pref = 34.98683665524972 * (cab * ip) * (ccd * iq) * sipq * w;
                        const double B00 = 0.5 * u * ipq;
                        const double B10 = 0.5 * ip * (1.0 - q * ipq * u);
                        const double B01 = 0.5 * iq * (1.0 - p * ipq * u);
                        const double PQd = d1 == 0 ? PQ0 : (d1 == 1 ? PQ1 : PQ2);
                        const double Pd = P[d1 == 0 ? 0 : (d1 == 1 ? 1 : 2)], Qd = Q[d1 == 0 ? 0 : (d1 == 1 ? 1 : 2)];
                        const double za = b1.y;
                        const DirectCoef dc =
                            direct_coef(za, 0.5 * zb2, 0.5 * zc2, 0.5 * zd2, p, q, ip, iq, u, ipq, B10, B01, B00);
                        const double CA = (Pd - Ad) - q * ipq * u * PQd, CB = CA + ABd;
                        const double CCx = (Qd - Cd) + p * ipq * u * PQd, CDx = CCx + CDd;
                        F *o = tab + s1 * TAB + d1 * 4 * NBASE;
                        direct_tables<LA, LB, LC, LD, F>(o, F(d1 == 2 ? pref : 1.0), F(CA), F(CB), F(CCx), F(CDx),
                                                         F(B10), F(B01), F(B00), F(zb2 * CB), F(dc.e2), F(dc.e3),
                                                         F(dc.e4), F(zc2 * CCx), F(dc.f2), F(dc.f3), F(dc.f4),
                                                         F(zd2 * CDx), F(dc.g2), F(dc.g3), F(dc.g4));
                    }
                    wave_sync();
#pragma unroll 1
                    for (int s = 0; s < CH; ++s) {
                        const int slot2 = ch * CH + s;
                        if (slot2 >= NSLOT) break;
                        const F *T = tab + s * TAB;
                        const F *G = sg + ((LR && slot2 >= NR) ? N : 0);
                        F pacc[9];
#pragma unroll
                        for (int k = 0; k < 9; ++k) pacc[k] = F(0);
#pragma unroll
                        for (int q = 0; q < CPL; ++q) {
                            if (!cok[q]) continue;
                            const F gm = G[lane + q * kWave];
                            const int ex = eoff[q][0], ey = eoff[q][1], ez = eoff[q][2];
                            const F vx = T[ex], vy = T[ey], vz = T[ez];
                            const F gz = gm * vz;
                            const F tyz = gz * vy, txz = gz * vx, txy = gm * vx * vy;
                            pacc[0] += tyz * T[ex + NBASE];
                            pacc[3] += tyz * T[ex + 2 * NBASE];
                            pacc[6] += tyz * T[ex + 3 * NBASE];
                            pacc[1] += txz * T[ey + NBASE];
                            pacc[4] += txz * T[ey + 2 * NBASE];
                            pacc[7] += txz * T[ey + 3 * NBASE];
                            pacc[2] += txy * T[ez + NBASE];
                            pacc[5] += txy * T[ez + 2 * NBASE];
                            pacc[8] += txy * T[ez + 3 * NBASE];
                        }
#pragma unroll
                        for (int k = 0; k < 9; ++k) acc[k] += double(pacc[k]);
                    }
                    wave_sync();
                }
            }
        }
        // wavefront reduction of the nine sums
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double v = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            acc[k] = v;
        }
        if (lane < 12) {
            const int X = lane / 3, d = lane % 3;
            const double v = X == 0 ? -(acc[d] + acc[3 + d] + acc[6 + d]) : acc[3 * (X - 1) + d];
            const int at = X == 0 ? atA : (X == 1 ? atB : (X == 2 ? atC : atD));
            if (a.task_out) atomic_add_global(&a.task_out[12 * t + lane], v);
            else if (use_lds) atomicAdd(&s_atoms[3 * at + d], v);
            else atomic_add_global(&M.grad[3 * at + d], v);
        }
    }
    if (use_lds) {
        // every wavefront's LDS additions land before the array is read (the barrier alone
        // does not order LDS operations of different wavefronts)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __syncthreads();
        for (int i = tid; i < 3 * a.n_atoms; i += blockDim.x) {
            const double v = s_atoms[i];
            if (v != 0.0) atomic_add_global(&a.grad[i], v);
        }
    }
}

} // namespace tdg
