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
    const double *pp_p, *pp_Px, *pp_Py, *pp_Pz, *pp_c, *pp_za, *pp_zb; // primitive pairs
    const double *Pn, *Dn, *Rn; // densities with the angular normalisation folded in
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
template <int NM, int MM, int IE, int JE, int LE>
struct Rys2D {
    double X[IE + 1][JE + 1][MM + 1][LE + 1];

    __device__ __forceinline__ void build(double I0, double C00, double D00, double B10, double B01,
                                          double B00, double AB, double CD)
    {
        double V[NM + 1][MM + 1];
        V[0][0] = I0;
        if constexpr (NM >= 1) V[1][0] = C00 * I0;
#pragma unroll
        for (int n = 1; n < NM; ++n) V[n + 1][0] = C00 * V[n][0] + (n * B10) * V[n - 1][0];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
#pragma unroll
            for (int n = 0; n <= NM; ++n) {
                double v = D00 * V[n][m];
                if (m > 0) v += (m * B01) * V[n][m > 0 ? m - 1 : 0];
                if (n > 0) v += (n * B00) * V[n > 0 ? n - 1 : 0][m];
                V[n][m + 1] = v;
            }
        }
        double W[NM + 1][JE + 1][MM + 1];
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

template <int LA, int LB, int LC, int LD, bool LR>
struct DerivClass {
    static constexpr int L = LA + LB + LC + LD;
    static constexpr int NR = nroots_deriv(L);
    static constexpr int NSET = LR ? 2 : 1;
    static constexpr int TEAM = NR * NSET;
    static constexpr int TPW = kWave / TEAM;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int N = NA * NB * NC * ND;
    static constexpr int GSTRIDE = NSET * N + 1;  // odd stride: teams start in different banks
    static constexpr int LDS_G_BYTES = 40 * 1024;
    static constexpr int TPB_LDS = LDS_G_BYTES / (GSTRIDE * 8) > 0 ? LDS_G_BYTES / (GSTRIDE * 8) : 1;
    static constexpr int TPB = TPW * 4 < TPB_LDS ? TPW * 4 : TPB_LDS;
    static constexpr int WAVES = (TPB + TPW - 1) / TPW;
    static constexpr int BLOCK = WAVES * kWave;
};

__device__ __forceinline__ void gamma_sym(const DerivArgs &a, int mu, int nu, int lam, int sig, double deg,
                                          double &gf, double &gl)
{
    const size_t n = a.n_bf;
    const double *P = a.Pn, *D = a.Dn, *R = a.Rn;
#define E_(M, i, j) M[(size_t)(i) * n + (j)]
    const double rs_mn = 0.5 * (E_(R, mu, nu) + E_(R, nu, mu));
    const double rs_ls = 0.5 * (E_(R, lam, sig) + E_(R, sig, lam));
    const double J = 2.0 * rs_mn * rs_ls + 0.25 * (E_(D, mu, nu) * E_(P, lam, sig) + E_(P, mu, nu) * E_(D, lam, sig));
    const double KD = E_(D, mu, sig) * E_(P, nu, lam) + E_(D, nu, sig) * E_(P, mu, lam) +
                      E_(D, mu, lam) * E_(P, nu, sig) + E_(D, nu, lam) * E_(P, mu, sig);
    const double KR = E_(R, sig, mu) * E_(R, lam, nu) + E_(R, sig, nu) * E_(R, lam, mu) +
                      E_(R, mu, sig) * E_(R, nu, lam) + E_(R, mu, lam) * E_(R, nu, sig);
#undef E_
    const double K = 0.0625 * KD + 0.25 * KR;
    gf = deg * (((a.terms & 1) ? J : 0.0) - ((a.terms & 2) ? a.alpha * K : 0.0));
    gl = deg * ((a.terms & 4) ? -a.beta * K : 0.0);
}

template <int LA, int LB, int LC, int LD, bool LR>
__global__ void __launch_bounds__((DerivClass<LA, LB, LC, LD, LR>::BLOCK))
k_deriv(const DerivArgs a)
{
    using K = DerivClass<LA, LB, LC, LD, LR>;
    constexpr int NR = K::NR, TEAM = K::TEAM, TPW = K::TPW, TPB = K::TPB;
    constexpr int NA = K::NA, NB = K::NB, NC = K::NC, ND = K::ND, N = K::N;
    extern __shared__ double s_atoms[];
    __shared__ double s_gam[TPB * K::GSTRIDE];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int tw = lane / TEAM, r = lane % TEAM;
    const int team = wave * TPW + tw;
    const bool lane_ok = (tw < TPW) && (team < TPB);
    const int set = r / NR, ir = r % NR;
    double *myG = s_gam + (lane_ok ? team : 0) * K::GSTRIDE;

    if (a.lds_atoms) {
        for (int i = tid; i < 3 * a.n_atoms; i += blockDim.x) s_atoms[i] = 0.0;
        __syncthreads();
    }
    const double om2 = a.omega * a.omega;
    const long long stride = (long long)gridDim.x * TPB;
    for (long long base = (long long)blockIdx.x * TPB; base < a.ntasks; base += stride) {
        const long long t = base + team;
        const bool valid = lane_ok && t < a.ntasks;
        int bra = 0, ket = 0, sa = 0, sb = 0, sc = 0, sd = 0;
        if (valid) {
            const int2 tk = a.tasks[t];
            bra = tk.x;
            ket = tk.y;
            sa = a.pair_sa[bra]; sb = a.pair_sb[bra];
            sc = a.pair_sa[ket]; sd = a.pair_sb[ket];
            const double deg = (sa != sb ? 2.0 : 1.0) * (sc != sd ? 2.0 : 1.0) * (bra != ket ? 2.0 : 1.0);
            const int oa = a.shell_ao[sa], ob = a.shell_ao[sb], oc = a.shell_ao[sc], od = a.shell_ao[sd];
            for (int c = r; c < N; c += TEAM) {
                const int id = c % ND, ic = (c / ND) % NC, ib = (c / (ND * NC)) % NB, ia = c / (ND * NC * NB);
                double gf, gl;
                gamma_sym(a, oa + ia, ob + ib, oc + ic, od + id, deg, gf, gl);
                myG[c] = gf;
                if constexpr (LR) myG[N + c] = gl;
            }
        }
        wave_sync();
        double acc[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        int atA = 0, atB = 0, atC = 0, atD = 0;
        if (valid) {
            atA = a.shell_atom[sa]; atB = a.shell_atom[sb]; atC = a.shell_atom[sc]; atD = a.shell_atom[sd];
            double A[3], AB[3], Cc[3], CD[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                A[d] = a.coords[3 * atA + d];
                AB[d] = A[d] - a.coords[3 * atB + d];
                Cc[d] = a.coords[3 * atC + d];
                CD[d] = Cc[d] - a.coords[3 * atD + d];
            }
            const int pb0 = a.pair_ppoff[bra], nbp = a.pair_npp[bra];
            const int pk0 = a.pair_ppoff[ket], nkp = a.pair_npp[ket];
            const double *gam = myG + set * N;
            for (int ib = 0; ib < nbp; ++ib) {
                const double p = a.pp_p[pb0 + ib], cab = a.pp_c[pb0 + ib], zb2 = 2.0 * a.pp_zb[pb0 + ib];
                const double P[3] = {a.pp_Px[pb0 + ib], a.pp_Py[pb0 + ib], a.pp_Pz[pb0 + ib]};
                for (int ik = 0; ik < nkp; ++ik) {
                    const double q = a.pp_p[pk0 + ik], ccd = a.pp_c[pk0 + ik];
                    const double zc2 = 2.0 * a.pp_za[pk0 + ik], zd2 = 2.0 * a.pp_zb[pk0 + ik];
                    const double Q[3] = {a.pp_Px[pk0 + ik], a.pp_Py[pk0 + ik], a.pp_Pz[pk0 + ik]};
                    const double ipq = 1.0 / (p + q);
                    const double rho = p * q * ipq;
                    double PQ[3], pq2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        PQ[d] = P[d] - Q[d];
                        pq2 += PQ[d] * PQ[d];
                    }
                    double Tr = rho * pq2, eta = 1.0;
                    if (LR && set) {
                        eta = om2 / (om2 + rho);
                        Tr *= eta;
                    }
                    double u, w;
                    rys_root<NR>(Tr, ir, u, w);
                    if (LR && set) {
                        u *= eta;
                        w *= sqrt(eta);
                    }
                    // 2 pi^(5/2) / (p q sqrt(p+q)) times contraction and pair factors
                    const double pref = 34.98683665524972 / (p * q) * sqrt(ipq) * cab * ccd * w;
                    const double B00 = 0.5 * u * ipq;
                    const double B10 = 0.5 / p * (1.0 - q * ipq * u);
                    const double B01 = 0.5 / q * (1.0 - p * ipq * u);
                    const double cq = q * ipq * u, cp = p * ipq * u;
                    Rys2D<LA + LB + 1, LC + LD + 1, LA, LB + 1, LD + 1> g[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double PA = P[d] - A[d], QC = Q[d] - Cc[d];
                        g[d].build(d == 2 ? pref : 1.0, PA - cq * PQ[d], QC + cp * PQ[d], B10, B01, B00, AB[d], CD[d]);
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
                                    const double gm = gam[c];
                                    double v[3], dB[3], dC[3], dD[3];
#pragma unroll
                                    for (int d = 0; d < 3; ++d) {
                                        const int i = kCart.v[LA][ia][d], j = kCart.v[LB][ib2][d];
                                        const int k = kCart.v[LC][ic][d], l = kCart.v[LD][id][d];
                                        const auto &X = g[d].X;
                                        v[d] = X[i][j][k][l];
                                        dB[d] = zb2 * X[i][j + 1][k][l] - (j ? j * X[i][j ? j - 1 : 0][k][l] : 0.0);
                                        dC[d] = zc2 * X[i][j][k + 1][l] - (k ? k * X[i][j][k ? k - 1 : 0][l] : 0.0);
                                        dD[d] = zd2 * X[i][j][k][l + 1] - (l ? l * X[i][j][k][l ? l - 1 : 0] : 0.0);
                                    }
                                    const double gz = gm * v[2];
                                    const double tyz = gz * v[1], txz = gz * v[0], txy = gm * v[0] * v[1];
                                    acc[0] += tyz * dB[0]; acc[1] += txz * dB[1]; acc[2] += txy * dB[2];
                                    acc[3] += tyz * dC[0]; acc[4] += txz * dC[1]; acc[5] += txy * dC[2];
                                    acc[6] += tyz * dD[0]; acc[7] += txz * dD[1]; acc[8] += txy * dD[2];
                                }
                }
            }
        }
        if (valid) {
            double out[12];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                out[3 + d] = acc[d];
                out[6 + d] = acc[3 + d];
                out[9 + d] = acc[6 + d];
                out[d] = -(acc[d] + acc[3 + d] + acc[6 + d]); // translational invariance (eq ti)
            }
            if (a.task_out) {
#pragma unroll
                for (int k = 0; k < 12; ++k) atomic_add_global(&a.task_out[12 * t + k], out[k]);
            } else {
                const int at[4] = {atA, atB, atC, atD};
#pragma unroll
                for (int X = 0; X < 4; ++X)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (a.lds_atoms) atomicAdd(&s_atoms[3 * at[X] + d], out[3 * X + d]);
                        else atomic_add_global(&a.grad[3 * at[X] + d], out[3 * X + d]);
                    }
            }
        }
        wave_sync();
    }
    if (a.lds_atoms) {
        __syncthreads();
        for (int i = tid; i < 3 * a.n_atoms; i += blockDim.x) {
            const double v = s_atoms[i];
            if (v != 0.0) atomic_add_global(&a.grad[i], v);
        }
    }
}

} // namespace tdg
