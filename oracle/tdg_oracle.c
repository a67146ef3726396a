/*
 * tdg_oracle.c -- CPU reference for the two-electron part of the TDA-TDDFT
 * nuclear gradient with range-separated hybrids.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * What it computes (paper section II.A, eq dE_ao, its fourth and fifth terms):
 *
 *   G[E][x] = sum_{mu nu lam sig} Gamma_{mu nu lam sig}   d(mu nu|lam sig)/dE_x
 *                               + Gamma^lr_{mu nu lam sig} d(mu nu|lam sig)_lr/dE_x
 *
 * with Gamma and Gamma^lr of eq gamma (P read as the ground-state density P0,
 * D = P0 + 2 PDelta), the full-range Coulomb ERI of eq eri_j and the
 * erf(omega r)/r ERI of eq lreri_k, over contracted Cartesian Gaussians
 * (eq cartG).  Units: hartree/bohr; the result is dE/dA (not the force).
 *
 * Method (deliberately different from the GPU's Rys quadrature):
 *   - Boys function by its power series with downward recursion (small T) and
 *     by erf with upward recursion (large T);
 *   - Obara-Saika vertical recursion to [e0|f0], Head-Gordon-Pople horizontal
 *     recursion to (ab|cd);
 *   - the long-range integral takes the same recursion with the auxiliary
 *     integrals eta^(m+1/2) F_m(eta T), eta = omega^2/(omega^2+rho);
 *   - derivatives of every one of the four centres are formed explicitly from
 *     eq deriv: d phi/dA_x = 2 zeta phi^(+x) - l_x phi^(-x) (centre derivative
 *     is minus the electron-coordinate derivative of eq deri), i.e. from a
 *     shell raised to l+1 with coefficients 2 zeta_k c_k and a shell lowered to
 *     l-1 with coefficients c_k.  Translational invariance (eq ti) is NOT used,
 *     so it stays an independent check.
 *   - fast mode: unique shell quartets, the 8-permutation average of Gamma and
 *     the shell-level degeneracy 2^([a!=b]+[c!=d]+[ab!=cd]);
 *   - brute mode: every ordered shell quartet with the literal Gamma.
 *
 * Also (section II.B, eqs G_2e and zfock): the two-electron part of the
 * Fock-type matrix of a matrix B, written out by its definition over every
 * ordered shell quartet (orc_fock_blocks).
 *
 * Normalisation: every Cartesian component is normalised to one: primitive
 * factor of the x^l component, contraction factor (cross overlaps included)
 * and the angular factor sqrt((2l-1)!!/((2lx-1)!!(2ly-1)!!(2lz-1)!!)).
 * Component order within a shell: lx descending, then ly descending.
 *
 * Screening (optional, tau > 0): a quartet is skipped when
 * Q_ab Q_cd M_abcd < tau with Q_ab = sqrt(max_{mu in a, nu in b}(mu nu|mu nu))
 * and M_abcd the largest of the products of shell-block maxima
 *   |D|ab|P|cd, |P|ab|D|cd, |R|ab|R|cd, |D|ac|P|bd, |D|bd|P|ac,
 *   |D|ad|P|bc, |D|bc|P|ad, |R|ac|R|bd, |R|ad|R|bc,
 * where |R|xy takes both orientations.  Quartets whose four shells sit on one
 * atom are skipped always (their derivative contribution is exactly zero).
 */
#include <tgmath.h> /* type-generic exp, sqrt, pow, erf, fabs, fmax */

/* Working precision of every integral, recursion and sum: x87 extended (64-bit
 * significand).  Inputs and outputs are FP64.  With contraction exponents up to
 * several thousand on d shells, the horizontal transfers and the 2 zeta phi^(+) -
 * l phi^(-) combinations of this algorithm cancel to the point where FP64 rounding
 * reaches ~1e-8 Eh/bohr in a gradient, the size of the FP64 tolerance the GPU path
 * is held to; the extra 11 bits keep the reference's own rounding far below it. */
typedef long double real;
#define ORC_PI 3.141592653589793238462643383279502884L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXL 2          /* basis shells up to d */
#define ORC_MAXLR 5         /* raised bra side: f + d */
#define ORC_NTRIP 56        /* Cartesian triples with l <= 5 */
#define ORC_MAXM 11
#define ORC_MAXPRIM 32

typedef struct {
    int32_t n_atoms;
    const double *coords;
    int32_t n_shells;
    const int32_t *shell_atom, *shell_l, *shell_nprim, *shell_prim_off, *shell_ao_off;
    int32_t n_prims;
    const double *exps, *coefs;
    int32_t n_bf;
} orc_basis_t;

typedef struct {
    double omega, alpha, beta, tau;
    int32_t terms;     /* bit 0: J, bit 1: full-range K (alpha), bit 2: long-range K (beta) */
    int32_t nthreads;  /* 0: OpenMP default */
} orc_params_t;

typedef struct {
    int64_t quartets;       /* unique shell quartets evaluated */
    int64_t prim_quartets;  /* primitive quartets of those */
    int64_t skipped;        /* quartets skipped by screening */
    int64_t one_center;     /* quartets skipped because all four shells share an atom */
} orc_stats_t;

/* ------------------------------------------------------------------------ */
/* Cartesian triples                                                         */

static int trip[ORC_NTRIP][3];
static int trip_ready = 0;

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int cart_off(int l) { return l * (l + 1) * (l + 2) / 6; }

/* position of (lx,ly,lz) among the components of l = lx+ly+lz */
static int cart_pos(int lx, int ly, int lz)
{
    int l = lx + ly + lz, s = l - lx;
    (void)lz;
    return s * (s + 1) / 2 + (s - ly);
}

static int idx3(const int t[3]) { return cart_off(t[0] + t[1] + t[2]) + cart_pos(t[0], t[1], t[2]); }

static void init_trip(void)
{
    if (trip_ready) return;
    int n = 0;
    for (int l = 0; l <= ORC_MAXLR; ++l)
        for (int lx = l; lx >= 0; --lx)
            for (int ly = l - lx; ly >= 0; --ly) {
                trip[n][0] = lx; trip[n][1] = ly; trip[n][2] = l - lx - ly; ++n;
            }
    trip_ready = 1;
}

static real dfact(int n) /* (n)!! with (-1)!! = 1 */
{
    real r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Boys function F_m(T), m = 0..mmax                                         */

static void boys(int mmax, real T, real *F)
{
    if (T < 30.0) {
        /* F_mmax(T) = exp(-T) sum_k (2T)^k / ((2mmax+1)(2mmax+3)...(2mmax+2k+1)) */
        real term = 1.0L / (2 * mmax + 1), sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= 2.0L * T / (2 * mmax + 2 * k + 1);
            sum += term;
            if (term < 1e-22L * sum) break;
        }
        real e = exp(-T);
        F[mmax] = e * sum;
        for (int m = mmax; m > 0; --m) F[m - 1] = (2.0L * T * F[m] + e) / (2 * m - 1);
    } else {
        real e = exp(-T);
        F[0] = 0.5L * sqrt(ORC_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0L * T);
    }
}

void orc_boys(int mmax, double T, double *F)
{
    real Fx[ORC_MAXM + 1];
    boys(mmax, T, Fx);
    for (int m = 0; m <= mmax; ++m) F[m] = (double)Fx[m];
}

/* ------------------------------------------------------------------------ */
/* A contracted Cartesian shell with all normalisation except the angular    */
/* factor folded into its coefficients.                                      */

typedef struct {
    int l, np;
    real A[3];
    real z[ORC_MAXPRIM];
    real c[ORC_MAXPRIM];
} oshell_t;

/* contraction coefficients for the x^l component, unit self-overlap */
static void normalise_shell(int l, int np, const real *z, const double *d, real *c)
{
    for (int k = 0; k < np; ++k) {
        real nk = pow(2.0 * z[k] / ORC_PI, 0.75) * pow(4.0 * z[k], 0.5 * l) / sqrt(dfact(2 * l - 1));
        c[k] = d[k] * nk;
    }
    real s = 0.0;
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            real zz = z[i] + z[j];
            s += c[i] * c[j] * dfact(2 * l - 1) / pow(2.0 * zz, l) * pow(ORC_PI / zz, 1.5);
        }
    real nc = 1.0 / sqrt(s);
    for (int k = 0; k < np; ++k) c[k] *= nc;
}

static real ang_norm(int lx, int ly, int lz)
{
    int l = lx + ly + lz;
    return sqrt(dfact(2 * l - 1) / (dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1)));
}

static void load_shell(const orc_basis_t *b, int s, oshell_t *out)
{
    int l = b->shell_l[s], np = b->shell_nprim[s], off = b->shell_prim_off[s];
    out->l = l;
    out->np = np;
    for (int k = 0; k < 3; ++k) out->A[k] = b->coords[3 * b->shell_atom[s] + k];
    for (int k = 0; k < np; ++k) out->z[k] = b->exps[off + k];
    normalise_shell(l, np, out->z, b->coefs + off, out->c);
}

/* ------------------------------------------------------------------------ */
/* Contracted ERI block over unnormalised Cartesian components               */
/* out[((ia*nb+ib)*nc+ic)*nd+id], op 0: 1/r, op 1: erf(omega r)/r            */

typedef struct {
    const real *Ic; /* contracted [e0|f0], e over triples |e|<=Emax, f over |f|<=Fmax */
    int nF;
    real AB[3], CD[3];
} hrr_ctx;

static real bra_hrr(const hrr_ctx *h, const int a[3], const int b[3], int f)
{
    if (b[0] + b[1] + b[2] == 0) return h->Ic[idx3(a) * h->nF + f];
    int i = b[0] ? 0 : (b[1] ? 1 : 2);
    int a1[3] = {a[0], a[1], a[2]}, b1[3] = {b[0], b[1], b[2]};
    a1[i] += 1;
    b1[i] -= 1;
    /* (a, b| = (a+1_i, b-1_i| + (A_i - B_i)(a, b-1_i| */
    return bra_hrr(h, a1, b1, f) + h->AB[i] * bra_hrr(h, a, b1, f);
}

static real full_hrr(const hrr_ctx *h, const int a[3], const int b[3], const int c[3], const int d[3])
{
    if (d[0] + d[1] + d[2] == 0) return bra_hrr(h, a, b, idx3(c));
    int i = d[0] ? 0 : (d[1] ? 1 : 2);
    int c1[3] = {c[0], c[1], c[2]}, d1[3] = {d[0], d[1], d[2]};
    c1[i] += 1;
    d1[i] -= 1;
    return full_hrr(h, a, b, c1, d1) + h->CD[i] * full_hrr(h, a, b, c, d1);
}

static void eri_block(const oshell_t *sa, const oshell_t *sb, const oshell_t *sc, const oshell_t *sd,
                      int op, real omega, real *out, int64_t *nprim)
{
    init_trip();
    const int la = sa->l, lb = sb->l, lc = sc->l, ld = sd->l;
    const int Emax = la + lb, Fmax = lc + ld, L = Emax + Fmax;
    const int nE = cart_off(Emax + 1), nF = cart_off(Fmax + 1), nM = L + 1;
    real *V = (real *)calloc((size_t)nE * nF * nM, sizeof(real));
    real *Ic = (real *)calloc((size_t)nE * nF, sizeof(real));
#define VV(e, f, m) V[((size_t)(e) * nF + (f)) * nM + (m)]
    real F[ORC_MAXM + 1];
    const real *A = sa->A, *B = sb->A, *C = sc->A, *D = sd->A;
    real AB2 = 0, CD2 = 0;
    for (int k = 0; k < 3; ++k) {
        AB2 += (A[k] - B[k]) * (A[k] - B[k]);
        CD2 += (C[k] - D[k]) * (C[k] - D[k]);
    }
    for (int i = 0; i < sa->np; ++i)
        for (int j = 0; j < sb->np; ++j) {
            real za = sa->z[i], zb = sb->z[j], p = za + zb;
            real P[3], PA[3];
            for (int k = 0; k < 3; ++k) {
                P[k] = (za * A[k] + zb * B[k]) / p;
                PA[k] = P[k] - A[k];
            }
            real Kab = exp(-za * zb / p * AB2);
            for (int k2 = 0; k2 < sc->np; ++k2)
                for (int l2 = 0; l2 < sd->np; ++l2) {
                    real zc = sc->z[k2], zd = sd->z[l2], q = zc + zd;
                    real Q[3], QC[3], W[3], WP[3], WQ[3];
                    for (int k = 0; k < 3; ++k) {
                        Q[k] = (zc * C[k] + zd * D[k]) / q;
                        QC[k] = Q[k] - C[k];
                    }
                    real Kcd = exp(-zc * zd / q * CD2);
                    real rho = p * q / (p + q), PQ2 = 0;
                    for (int k = 0; k < 3; ++k) {
                        W[k] = (p * P[k] + q * Q[k]) / (p + q);
                        WP[k] = W[k] - P[k];
                        WQ[k] = W[k] - Q[k];
                        PQ2 += (P[k] - Q[k]) * (P[k] - Q[k]);
                    }
                    real T = rho * PQ2;
                    real pref = 2.0 * pow(ORC_PI, 2.5) / (p * q * sqrt(p + q)) * Kab * Kcd *
                                  sa->c[i] * sb->c[j] * sc->c[k2] * sd->c[l2];
                    if (op == 0) {
                        boys(L, T, F);
                        for (int m = 0; m <= L; ++m) VV(0, 0, m) = pref * F[m];
                    } else {
                        real eta = omega * omega / (omega * omega + rho);
                        boys(L, eta * T, F);
                        real s = sqrt(eta);
                        for (int m = 0; m <= L; ++m) {
                            VV(0, 0, m) = pref * s * F[m];
                            s *= eta;
                        }
                    }
                    /* bra vertical recursion:
                     * [e+1_i 0|00]^m = PA_i [e|]^m + WP_i [e|]^(m+1)
                     *                  + e_i/(2p) ([e-1_i|]^m - rho/p [e-1_i|]^(m+1)) */
                    for (int e = 1; e < nE; ++e) {
                        const int *t = trip[e];
                        int n = t[0] + t[1] + t[2];
                        int i3 = t[0] ? 0 : (t[1] ? 1 : 2);
                        int em[3] = {t[0], t[1], t[2]};
                        em[i3] -= 1;
                        int e1 = idx3(em);
                        int ei = em[i3];
                        int e2 = -1;
                        if (ei > 0) {
                            int emm[3] = {em[0], em[1], em[2]};
                            emm[i3] -= 1;
                            e2 = idx3(emm);
                        }
                        for (int m = 0; m <= L - n; ++m) {
                            real v = PA[i3] * VV(e1, 0, m) + WP[i3] * VV(e1, 0, m + 1);
                            if (e2 >= 0) v += ei / (2.0 * p) * (VV(e2, 0, m) - rho / p * VV(e2, 0, m + 1));
                            VV(e, 0, m) = v;
                        }
                    }
                    /* ket vertical recursion:
                     * [e0|f+1_i 0]^m = QC_i [e|f]^m + WQ_i [e|f]^(m+1)
                     *   + f_i/(2q) ([e|f-1_i]^m - rho/q [e|f-1_i]^(m+1))
                     *   + e_i/(2(p+q)) [e-1_i|f]^(m+1) */
                    for (int f = 1; f < nF; ++f) {
                        const int *t = trip[f];
                        int nf = t[0] + t[1] + t[2];
                        int i3 = t[0] ? 0 : (t[1] ? 1 : 2);
                        int fm[3] = {t[0], t[1], t[2]};
                        fm[i3] -= 1;
                        int f1 = idx3(fm);
                        int fi = fm[i3];
                        int f2 = -1;
                        if (fi > 0) {
                            int fmm[3] = {fm[0], fm[1], fm[2]};
                            fmm[i3] -= 1;
                            f2 = idx3(fmm);
                        }
                        for (int e = 0; e < nE; ++e) {
                            const int *te = trip[e];
                            int ne = te[0] + te[1] + te[2];
                            int ei = te[i3];
                            int e1 = -1;
                            if (ei > 0) {
                                int em[3] = {te[0], te[1], te[2]};
                                em[i3] -= 1;
                                e1 = idx3(em);
                            }
                            for (int m = 0; m <= L - ne - nf; ++m) {
                                real v = QC[i3] * VV(e, f1, m) + WQ[i3] * VV(e, f1, m + 1);
                                if (f2 >= 0) v += fi / (2.0 * q) * (VV(e, f2, m) - rho / q * VV(e, f2, m + 1));
                                if (e1 >= 0) v += ei / (2.0 * (p + q)) * VV(e1, f1, m + 1);
                                VV(e, f, m) = v;
                            }
                        }
                    }
                    for (int e = 0; e < nE; ++e)
                        for (int f = 0; f < nF; ++f) Ic[(size_t)e * nF + f] += VV(e, f, 0);
                    if (nprim) ++*nprim;
                }
        }
#undef VV
    hrr_ctx h;
    h.Ic = Ic;
    h.nF = nF;
    for (int k = 0; k < 3; ++k) {
        h.AB[k] = A[k] - B[k];
        h.CD[k] = C[k] - D[k];
    }
    const int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
    const int oa = cart_off(la), ob = cart_off(lb), oc = cart_off(lc), od = cart_off(ld);
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib)
            for (int ic = 0; ic < nc; ++ic)
                for (int id = 0; id < nd; ++id)
                    out[((ia * nb + ib) * nc + ic) * nd + id] =
                        full_hrr(&h, trip[oa + ia], trip[ob + ib], trip[oc + ic], trip[od + id]);
    free(V);
    free(Ic);
}

/* ------------------------------------------------------------------------ */
/* Normalised blocks: value block and the 12 centre-derivative blocks        */

static void apply_ang(const oshell_t *s[4], real *blk)
{
    const int n[4] = {ncart(s[0]->l), ncart(s[1]->l), ncart(s[2]->l), ncart(s[3]->l)};
    for (int ia = 0; ia < n[0]; ++ia)
        for (int ib = 0; ib < n[1]; ++ib)
            for (int ic = 0; ic < n[2]; ++ic)
                for (int id = 0; id < n[3]; ++id) {
                    const int *ta = trip[cart_off(s[0]->l) + ia], *tb = trip[cart_off(s[1]->l) + ib];
                    const int *tc = trip[cart_off(s[2]->l) + ic], *td = trip[cart_off(s[3]->l) + id];
                    blk[((ia * n[1] + ib) * n[2] + ic) * n[3] + id] *=
                        ang_norm(ta[0], ta[1], ta[2]) * ang_norm(tb[0], tb[1], tb[2]) *
                        ang_norm(tc[0], tc[1], tc[2]) * ang_norm(td[0], td[1], td[2]);
                }
}

/* value block (normalised components) */
static void value_block(const oshell_t *s[4], int op, real omega, real *blk, int64_t *np)
{
    eri_block(s[0], s[1], s[2], s[3], op, omega, blk, np);
    apply_ang(s, blk);
}

/* der[(X*3+x)*N + comp]: d(ab|cd)/dX_x for the four centres X = a,b,c,d, explicitly */
static void deriv_blocks(const oshell_t *s[4], int op, real omega, real *der, int64_t *np)
{
    const int n[4] = {ncart(s[0]->l), ncart(s[1]->l), ncart(s[2]->l), ncart(s[3]->l)};
    const int N = n[0] * n[1] * n[2] * n[3];
    memset(der, 0, sizeof(real) * 12 * N);
    for (int X = 0; X < 4; ++X) {
        const oshell_t *base = s[X];
        oshell_t up = *base, dn = *base;
        up.l = base->l + 1;
        for (int k = 0; k < base->np; ++k) up.c[k] = 2.0 * base->z[k] * base->c[k];
        dn.l = base->l - 1;
        int nu[4] = {n[0], n[1], n[2], n[3]}, nd[4] = {n[0], n[1], n[2], n[3]};
        nu[X] = ncart(up.l);
        nd[X] = dn.l >= 0 ? ncart(dn.l) : 0;
        real *bu = (real *)malloc(sizeof(real) * nu[0] * nu[1] * nu[2] * nu[3]);
        real *bd = nd[X] ? (real *)malloc(sizeof(real) * nd[0] * nd[1] * nd[2] * nd[3]) : NULL;
        const oshell_t *su[4] = {s[0], s[1], s[2], s[3]}, *sd[4] = {s[0], s[1], s[2], s[3]};
        su[X] = &up;
        sd[X] = &dn;
        eri_block(su[0], su[1], su[2], su[3], op, omega, bu, X == 0 ? np : NULL); /* count once */
        if (bd) eri_block(sd[0], sd[1], sd[2], sd[3], op, omega, bd, NULL);
        for (int c0 = 0; c0 < n[0]; ++c0)
            for (int c1 = 0; c1 < n[1]; ++c1)
                for (int c2 = 0; c2 < n[2]; ++c2)
                    for (int c3 = 0; c3 < n[3]; ++c3) {
                        int cc[4] = {c0, c1, c2, c3};
                        const int *t = trip[cart_off(base->l) + cc[X]];
                        int comp = ((c0 * n[1] + c1) * n[2] + c2) * n[3] + c3;
                        for (int x = 0; x < 3; ++x) {
                            int tu[3] = {t[0], t[1], t[2]};
                            tu[x] += 1;
                            int cu[4] = {c0, c1, c2, c3};
                            cu[X] = cart_pos(tu[0], tu[1], tu[2]);
                            real v = bu[((cu[0] * nu[1] + cu[1]) * nu[2] + cu[2]) * nu[3] + cu[3]];
                            if (t[x] > 0) {
                                int td[3] = {t[0], t[1], t[2]};
                                td[x] -= 1;
                                int cd[4] = {c0, c1, c2, c3};
                                cd[X] = cart_pos(td[0], td[1], td[2]);
                                v -= t[x] * bd[((cd[0] * nd[1] + cd[1]) * nd[2] + cd[2]) * nd[3] + cd[3]];
                            }
                            der[(X * 3 + x) * N + comp] = v;
                        }
                    }
        free(bu);
        free(bd);
    }
    for (int k = 0; k < 12; ++k) apply_ang(s, der + (size_t)k * N);
}

/* ------------------------------------------------------------------------ */
/* Two-particle densities                                                    */

typedef struct {
    int n;
    const double *P, *PD, *R;
    real alpha, beta;
    int terms;
} dens_t;

#define M_(X, i, j) ((X)[(size_t)(i) * d->n + (j)])

static real Dm(const dens_t *d, int i, int j) { return M_(d->P, i, j) + 2.0 * M_(d->PD, i, j); }

/* literal Gamma and Gamma^lr of eq gamma (P -> P0, D = P0 + 2 PDelta) */
static void gamma_literal(const dens_t *d, int mu, int nu, int lam, int sig, real *gf, real *gl)
{
    real J = 2.0 * M_(d->R, nu, mu) * M_(d->R, lam, sig) + 0.5 * Dm(d, mu, nu) * M_(d->P, lam, sig);
    real K = M_(d->R, sig, mu) * M_(d->R, lam, nu) + 0.25 * Dm(d, mu, sig) * M_(d->P, lam, nu);
    *gf = ((d->terms & 1) ? J : 0.0) - ((d->terms & 2) ? d->alpha * K : 0.0);
    *gl = (d->terms & 4) ? -d->beta * K : 0.0;
}

/* average of the literal Gamma over the eight index permutations that leave
 * (mu nu|lam sig) unchanged */
static void gamma_sym(const dens_t *d, int mu, int nu, int lam, int sig, real *gf, real *gl)
{
    real Rs_mn = 0.5 * (M_(d->R, mu, nu) + M_(d->R, nu, mu));
    real Rs_ls = 0.5 * (M_(d->R, lam, sig) + M_(d->R, sig, lam));
    real J = 2.0 * Rs_mn * Rs_ls +
               0.25 * (Dm(d, mu, nu) * M_(d->P, lam, sig) + M_(d->P, mu, nu) * Dm(d, lam, sig));
    real KD = 0.25 * (Dm(d, mu, sig) * M_(d->P, nu, lam) + Dm(d, nu, sig) * M_(d->P, mu, lam) +
                        Dm(d, mu, lam) * M_(d->P, nu, sig) + Dm(d, nu, lam) * M_(d->P, mu, sig));
    real KR = 0.25 * (M_(d->R, sig, mu) * M_(d->R, lam, nu) + M_(d->R, sig, nu) * M_(d->R, lam, mu) +
                        M_(d->R, mu, sig) * M_(d->R, nu, lam) + M_(d->R, mu, lam) * M_(d->R, nu, sig));
    real K = 0.25 * KD + KR;
    *gf = ((d->terms & 1) ? J : 0.0) - ((d->terms & 2) ? d->alpha * K : 0.0);
    *gl = (d->terms & 4) ? -d->beta * K : 0.0;
}
#undef M_

/* ------------------------------------------------------------------------ */
/* Screening                                                                 */

typedef struct {
    real *Q;      /* [npair] Schwarz factors, unique pairs a>=b, index a(a+1)/2+b */
    real *mP, *mD, *mR; /* [ns*ns] shell-block maxima of |P0|, |D|, |R| (both orientations) */
} screen_t;

static int64_t pidx(int a, int b) { return a >= b ? (int64_t)a * (a + 1) / 2 + b : (int64_t)b * (b + 1) / 2 + a; }

static void screen_build(const orc_basis_t *b, const oshell_t *sh, const dens_t *d, int nthreads, screen_t *s)
{
    const int ns = b->n_shells;
    const int64_t np = (int64_t)ns * (ns + 1) / 2;
    s->Q = (real *)calloc(np, sizeof(real));
    s->mP = (real *)calloc((size_t)ns * ns, sizeof(real));
    s->mD = (real *)calloc((size_t)ns * ns, sizeof(real));
    s->mR = (real *)calloc((size_t)ns * ns, sizeof(real));
#pragma omp parallel for schedule(dynamic) num_threads(nthreads)
    for (int a = 0; a < ns; ++a) {
        for (int c = 0; c <= a; ++c) {
            const oshell_t *q4[4] = {&sh[a], &sh[c], &sh[a], &sh[c]};
            int na = ncart(sh[a].l), nc = ncart(sh[c].l);
            real *blk = (real *)malloc(sizeof(real) * na * nc * na * nc);
            value_block(q4, 0, 0.0, blk, NULL);
            real mx = 0.0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nc; ++j) {
                    real v = blk[((i * nc + j) * na + i) * nc + j];
                    if (v > mx) mx = v;
                }
            free(blk);
            s->Q[pidx(a, c)] = sqrt(mx);
        }
        for (int c = 0; c < ns; ++c) {
            real mp = 0, md = 0, mr = 0;
            int oa = b->shell_ao_off[a], oc = b->shell_ao_off[c];
            for (int i = 0; i < ncart(sh[a].l); ++i)
                for (int j = 0; j < ncart(sh[c].l); ++j) {
                    size_t ij = (size_t)(oa + i) * d->n + (oc + j), ji = (size_t)(oc + j) * d->n + (oa + i);
                    real vp = fabs(d->P[ij]), vd = fabs(d->P[ij] + 2.0 * d->PD[ij]);
                    real vr = fmax(fabs(d->R[ij]), fabs(d->R[ji]));
                    if (vp > mp) mp = vp;
                    if (vd > md) md = vd;
                    if (vr > mr) mr = vr;
                }
            s->mP[(size_t)a * ns + c] = mp;
            s->mD[(size_t)a * ns + c] = md;
            s->mR[(size_t)a * ns + c] = mr;
        }
    }
}

static void screen_free(screen_t *s)
{
    free(s->Q); free(s->mP); free(s->mD); free(s->mR);
}

static real quartet_bound(const screen_t *s, int ns, int a, int b, int c, int d)
{
#define PR(X, i, j) (s->X[(size_t)(i) * ns + (j)])
    real m = PR(mD, a, b) * PR(mP, c, d);
    m = fmax(m, PR(mP, a, b) * PR(mD, c, d));
    m = fmax(m, PR(mR, a, b) * PR(mR, c, d));
    m = fmax(m, PR(mD, a, c) * PR(mP, b, d));
    m = fmax(m, PR(mD, b, d) * PR(mP, a, c));
    m = fmax(m, PR(mD, a, d) * PR(mP, b, c));
    m = fmax(m, PR(mD, b, c) * PR(mP, a, d));
    m = fmax(m, PR(mR, a, c) * PR(mR, b, d));
    m = fmax(m, PR(mR, a, d) * PR(mR, b, c));
#undef PR
    return s->Q[pidx(a, b)] * s->Q[pidx(c, d)] * m;
}

/* ------------------------------------------------------------------------ */
/* Per-quartet gradient contribution: out12[X*3+x] for centres a,b,c,d        */

static void quartet_contrib(const orc_basis_t *b, const oshell_t *sh, const dens_t *d, real omega,
                            int sa, int sb, int sc, int sd, int literal, real weight,
                            real *out12, int64_t *np, real *scratch)
{
    const oshell_t *q4[4] = {&sh[sa], &sh[sb], &sh[sc], &sh[sd]};
    const int n[4] = {ncart(q4[0]->l), ncart(q4[1]->l), ncart(q4[2]->l), ncart(q4[3]->l)};
    const int N = n[0] * n[1] * n[2] * n[3];
    real *df = scratch, *dl = scratch + 12 * N;
    int need_f = (d->terms & 3) != 0, need_l = (d->terms & 4) != 0;
    if (need_f) deriv_blocks(q4, 0, omega, df, np);
    else memset(df, 0, sizeof(real) * 12 * N);
    if (need_l) deriv_blocks(q4, 1, omega, dl, need_f ? NULL : np);
    else memset(dl, 0, sizeof(real) * 12 * N);
    const int o[4] = {b->shell_ao_off[sa], b->shell_ao_off[sb], b->shell_ao_off[sc], b->shell_ao_off[sd]};
    for (int k = 0; k < 12; ++k) out12[k] = 0.0;
    for (int i = 0; i < n[0]; ++i)
        for (int j = 0; j < n[1]; ++j)
            for (int k = 0; k < n[2]; ++k)
                for (int l = 0; l < n[3]; ++l) {
                    int comp = ((i * n[1] + j) * n[2] + k) * n[3] + l;
                    real gf, gl;
                    if (literal) gamma_literal(d, o[0] + i, o[1] + j, o[2] + k, o[3] + l, &gf, &gl);
                    else gamma_sym(d, o[0] + i, o[1] + j, o[2] + k, o[3] + l, &gf, &gl);
                    for (int x = 0; x < 12; ++x) out12[x] += gf * df[x * N + comp] + gl * dl[x * N + comp];
                }
    for (int x = 0; x < 12; ++x) out12[x] *= weight;
}

static int max_nprim(const orc_basis_t *b)
{
    int m = 0;
    for (int s = 0; s < b->n_shells; ++s)
        if (b->shell_nprim[s] > m) m = b->shell_nprim[s];
    return m;
}

static int check_basis(const orc_basis_t *b)
{
    if (!b || b->n_shells <= 0 || b->n_atoms <= 0) return -1;
    for (int s = 0; s < b->n_shells; ++s) {
        if (b->shell_l[s] < 0 || b->shell_l[s] > ORC_MAXL) return -2;
        if (b->shell_nprim[s] < 1 || b->shell_nprim[s] > ORC_MAXPRIM) return -2;
        if (b->shell_atom[s] < 0 || b->shell_atom[s] >= b->n_atoms) return -1;
    }
    (void)max_nprim;
    return 0;
}

static oshell_t *load_all(const orc_basis_t *b)
{
    oshell_t *sh = (oshell_t *)malloc(sizeof(oshell_t) * b->n_shells);
    for (int s = 0; s < b->n_shells; ++s) load_shell(b, s, &sh[s]);
    return sh;
}

#define SCRATCH_N (2 * 12 * 1296)

/* ------------------------------------------------------------------------ */
/* Public entry points (ctypes)                                              */

/* fast mode: unique shell quartets, symmetrised Gamma, degeneracy weights */
int orc_grad(const orc_basis_t *b, const double *P0, const double *PD, const double *R,
             const orc_params_t *prm, double *grad, orc_stats_t *st)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    const int ns = b->n_shells, na = b->n_atoms;
    int nth = prm->nthreads > 0 ? prm->nthreads : 1;
#ifdef _OPENMP
    if (prm->nthreads <= 0) nth = omp_get_max_threads();
#endif
    oshell_t *sh = load_all(b);
    dens_t d = {b->n_bf, P0, PD, R, prm->alpha, prm->beta, prm->terms};
    screen_t scr;
    memset(&scr, 0, sizeof scr);
    if (prm->tau > 0) screen_build(b, sh, &d, nth, &scr);
    const int64_t npair = (int64_t)ns * (ns + 1) / 2;
    int *pa = (int *)malloc(sizeof(int) * npair), *pb = (int *)malloc(sizeof(int) * npair);
    for (int a = 0, k = 0; a < ns; ++a)
        for (int c = 0; c <= a; ++c, ++k) { pa[k] = a; pb[k] = c; }
    real *gsum = (real *)calloc((size_t)na * 3, sizeof(real));
    int64_t q = 0, pq = 0, sk = 0, oc = 0;
#pragma omp parallel num_threads(nth) reduction(+ : q, pq, sk, oc)
    {
        real *gl = (real *)calloc((size_t)na * 3, sizeof(real));
        real *scratch = (real *)malloc(sizeof(real) * SCRATCH_N);
        real c12[12];
#pragma omp for schedule(dynamic, 1)
        for (int64_t ab = 0; ab < npair; ++ab) {
            int a = pa[ab], bb = pb[ab];
            for (int64_t cd = 0; cd <= ab; ++cd) {
                int c = pa[cd], dd = pb[cd];
                int at = b->shell_atom[a];
                if (b->shell_atom[bb] == at && b->shell_atom[c] == at && b->shell_atom[dd] == at) { ++oc; continue; }
                if (prm->tau > 0 && quartet_bound(&scr, ns, a, bb, c, dd) < prm->tau) { ++sk; continue; }
                real deg = (a != bb ? 2.0 : 1.0) * (c != dd ? 2.0 : 1.0) * (ab != cd ? 2.0 : 1.0);
                int64_t np = 0;
                quartet_contrib(b, sh, &d, prm->omega, a, bb, c, dd, 0, deg, c12, &np, scratch);
                const int s4[4] = {a, bb, c, dd};
                for (int X = 0; X < 4; ++X)
                    for (int x = 0; x < 3; ++x) gl[3 * b->shell_atom[s4[X]] + x] += c12[3 * X + x];
                ++q;
                pq += np;
            }
        }
#pragma omp critical
        for (int k = 0; k < 3 * na; ++k) gsum[k] += gl[k];
        free(gl);
        free(scratch);
    }
    for (int k = 0; k < 3 * na; ++k) grad[k] = (double)gsum[k];
    if (st) { st->quartets = q; st->prim_quartets = pq; st->skipped = sk; st->one_center = oc; }
    free(gsum); free(pa); free(pb); free(sh);
    if (prm->tau > 0) screen_free(&scr);
    return 0;
}

/* brute mode: every ordered shell quartet, literal Gamma, no screening */
int orc_grad_brute(const orc_basis_t *b, const double *P0, const double *PD, const double *R,
                   const orc_params_t *prm, double *grad)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    const int ns = b->n_shells, na = b->n_atoms;
    int nth = 1;
#ifdef _OPENMP
    nth = prm->nthreads > 0 ? prm->nthreads : omp_get_max_threads();
#endif
    oshell_t *sh = load_all(b);
    dens_t d = {b->n_bf, P0, PD, R, prm->alpha, prm->beta, prm->terms};
    real *gsum = (real *)calloc((size_t)na * 3, sizeof(real));
#pragma omp parallel num_threads(nth)
    {
        real *gl = (real *)calloc((size_t)na * 3, sizeof(real));
        real *scratch = (real *)malloc(sizeof(real) * SCRATCH_N);
        real c12[12];
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int a = 0; a < ns; ++a)
            for (int bb = 0; bb < ns; ++bb)
                for (int c = 0; c < ns; ++c)
                    for (int dd = 0; dd < ns; ++dd) {
                        quartet_contrib(b, sh, &d, prm->omega, a, bb, c, dd, 1, 1.0, c12, NULL, scratch);
                        const int s4[4] = {a, bb, c, dd};
                        for (int X = 0; X < 4; ++X)
                            for (int x = 0; x < 3; ++x) gl[3 * b->shell_atom[s4[X]] + x] += c12[3 * X + x];
                    }
#pragma omp critical
        for (int k = 0; k < 3 * na; ++k) gsum[k] += gl[k];
        free(gl);
        free(scratch);
    }
    for (int k = 0; k < 3 * na; ++k) grad[k] = (double)gsum[k];
    free(gsum); free(sh);
    return 0;
}

/* pseudo-energy E2 = sum Gamma (mu nu|lam sig) + Gamma^lr (mu nu|lam sig)_lr with the
 * densities held fixed (the quantity whose nuclear derivative orc_grad returns) */
int orc_energy(const orc_basis_t *b, const double *P0, const double *PD, const double *R,
               const orc_params_t *prm, double *energy)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    const int ns = b->n_shells;
    int nth = 1;
#ifdef _OPENMP
    nth = prm->nthreads > 0 ? prm->nthreads : omp_get_max_threads();
#endif
    oshell_t *sh = load_all(b);
    dens_t d = {b->n_bf, P0, PD, R, prm->alpha, prm->beta, prm->terms};
    const int64_t npair = (int64_t)ns * (ns + 1) / 2;
    int *pa = (int *)malloc(sizeof(int) * npair), *pb = (int *)malloc(sizeof(int) * npair);
    for (int a = 0, k = 0; a < ns; ++a)
        for (int c = 0; c <= a; ++c, ++k) { pa[k] = a; pb[k] = c; }
    real e = 0.0;
#pragma omp parallel num_threads(nth) reduction(+ : e)
    {
        real *bf = (real *)malloc(sizeof(real) * 1296), *bl = (real *)malloc(sizeof(real) * 1296);
#pragma omp for schedule(dynamic, 1)
        for (int64_t ab = 0; ab < npair; ++ab)
            for (int64_t cd = 0; cd <= ab; ++cd) {
                int a = pa[ab], bb = pb[ab], c = pa[cd], dd = pb[cd];
                const oshell_t *q4[4] = {&sh[a], &sh[bb], &sh[c], &sh[dd]};
                const int n[4] = {ncart(q4[0]->l), ncart(q4[1]->l), ncart(q4[2]->l), ncart(q4[3]->l)};
                const int N = n[0] * n[1] * n[2] * n[3];
                if (d.terms & 3) value_block(q4, 0, prm->omega, bf, NULL); else memset(bf, 0, sizeof(real) * N);
                if (d.terms & 4) value_block(q4, 1, prm->omega, bl, NULL); else memset(bl, 0, sizeof(real) * N);
                real deg = (a != bb ? 2.0 : 1.0) * (c != dd ? 2.0 : 1.0) * (ab != cd ? 2.0 : 1.0);
                const int o[4] = {b->shell_ao_off[a], b->shell_ao_off[bb], b->shell_ao_off[c], b->shell_ao_off[dd]};
                real s = 0.0;
                for (int i = 0; i < n[0]; ++i)
                    for (int j = 0; j < n[1]; ++j)
                        for (int k = 0; k < n[2]; ++k)
                            for (int l = 0; l < n[3]; ++l) {
                                int comp = ((i * n[1] + j) * n[2] + k) * n[3] + l;
                                real gf, gl;
                                gamma_sym(&d, o[0] + i, o[1] + j, o[2] + k, o[3] + l, &gf, &gl);
                                s += gf * bf[comp] + gl * bl[comp];
                            }
                e += deg * s;
            }
        free(bf);
        free(bl);
    }
    *energy = e;
    free(pa); free(pb); free(sh);
    return 0;
}

/* contributions of listed shell quartets: out[q*12 + X*3 + x] for centres (a,b,c,d) as given,
 * weighted by the degeneracy of the unordered quartet; symmetrised Gamma, no screening */
int orc_quartet_contribs(const orc_basis_t *b, const double *P0, const double *PD, const double *R,
                         const orc_params_t *prm, int64_t nq, const int32_t *quartets, double *out)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    int nth = 1;
#ifdef _OPENMP
    nth = prm->nthreads > 0 ? prm->nthreads : omp_get_max_threads();
#endif
    oshell_t *sh = load_all(b);
    dens_t d = {b->n_bf, P0, PD, R, prm->alpha, prm->beta, prm->terms};
#pragma omp parallel num_threads(nth)
    {
        real *scratch = (real *)malloc(sizeof(real) * SCRATCH_N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < nq; ++k) {
            int a = quartets[4 * k], bb = quartets[4 * k + 1], c = quartets[4 * k + 2], dd = quartets[4 * k + 3];
            int64_t ab = pidx(a, bb), cd = pidx(c, dd);
            real deg = (a != bb ? 2.0 : 1.0) * (c != dd ? 2.0 : 1.0) * (ab != cd ? 2.0 : 1.0);
            real c12[12];
            quartet_contrib(b, sh, &d, prm->omega, a, bb, c, dd, 0, deg, c12, NULL, scratch);
            for (int x = 0; x < 12; ++x) out[12 * k + x] = (double)c12[x];
        }
        free(scratch);
    }
    free(sh);
    return 0;
}

/* screening data as the oracle defines it: Q[npair] and per-quartet bound for listed quartets */
int orc_schwarz(const orc_basis_t *b, double *Q)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    const int ns = b->n_shells;
    oshell_t *sh = load_all(b);
    for (int a = 0; a < ns; ++a)
        for (int c = 0; c <= a; ++c) {
            const oshell_t *q4[4] = {&sh[a], &sh[c], &sh[a], &sh[c]};
            int na = ncart(sh[a].l), nc = ncart(sh[c].l);
            real *blk = (real *)malloc(sizeof(real) * na * nc * na * nc);
            value_block(q4, 0, 0.0, blk, NULL);
            real mx = 0.0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nc; ++j) {
                    real v = blk[((i * nc + j) * na + i) * nc + j];
                    if (v > mx) mx = v;
                }
            free(blk);
            Q[pidx(a, c)] = sqrt(mx);
        }
    free(sh);
    return 0;
}

int orc_quartet_bounds(const orc_basis_t *b, const double *P0, const double *PD, const double *R,
                       int64_t nq, const int32_t *quartets, double *bound)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    oshell_t *sh = load_all(b);
    dens_t d = {b->n_bf, P0, PD, R, 0.0, 0.0, 7};
    screen_t scr;
    screen_build(b, sh, &d, 1, &scr);
    for (int64_t k = 0; k < nq; ++k)
        bound[k] = quartet_bound(&scr, b->n_shells, quartets[4 * k], quartets[4 * k + 1], quartets[4 * k + 2],
                                 quartets[4 * k + 3]);
    screen_free(&scr);
    free(sh);
    return 0;
}

/* The screening decision itself: every unique quartet (a>=b, c>=d, pair(ab)>=pair(cd), not
 * all four shells on one atom) whose bound Q_ab Q_cd M_abcd is >= tau (keep = 1) or < tau
 * (keep = 0), in that enumeration order; up to cap quartets [k][4] and their bounds are
 * written, *n_out receives the full count. */
int orc_screen_select(const orc_basis_t *b, const double *P0, const double *PD, const double *R, double tau,
                      int keep, int nthreads, int64_t cap, int32_t *quartets, double *bound, int64_t *n_out)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    const int ns = b->n_shells;
    oshell_t *sh = load_all(b);
    dens_t d = {b->n_bf, P0, PD, R, 0.0, 0.0, 7};
    screen_t scr;
    screen_build(b, sh, &d, nth, &scr);
    const int64_t npair = (int64_t)ns * (ns + 1) / 2;
    int *pa = (int *)malloc(sizeof(int) * npair), *pb = (int *)malloc(sizeof(int) * npair);
    for (int a = 0, k = 0; a < ns; ++a)
        for (int c = 0; c <= a; ++c, ++k) { pa[k] = a; pb[k] = c; }
    int64_t *cnt = (int64_t *)calloc(npair + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
        for (int64_t ab = 0; ab < npair; ++ab) {
            const int a = pa[ab], bb = pb[ab];
            const int at = b->shell_atom[a];
            int64_t k = pass ? cnt[ab] : 0;
            for (int64_t cd = 0; cd <= ab; ++cd) {
                const int c = pa[cd], dd = pb[cd];
                if (b->shell_atom[bb] == at && b->shell_atom[c] == at && b->shell_atom[dd] == at) continue;
                const real q = quartet_bound(&scr, ns, a, bb, c, dd);
                if ((q >= tau) != (keep != 0)) continue;
                if (pass && k < cap) {
                    quartets[4 * k] = a; quartets[4 * k + 1] = bb;
                    quartets[4 * k + 2] = c; quartets[4 * k + 3] = dd;
                    bound[k] = (double)q;
                }
                ++k;
            }
            if (!pass) cnt[ab] = k;
        }
        if (!pass) { /* exclusive prefix sums: first output slot of every bra pair */
            int64_t acc = 0;
            for (int64_t ab = 0; ab <= npair; ++ab) {
                const int64_t v = ab < npair ? cnt[ab] : 0;
                cnt[ab] = acc;
                acc += v;
            }
        }
    }
    *n_out = cnt[npair];
    free(cnt); free(pa); free(pb); free(sh);
    screen_free(&scr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fock-type matrix of section II.B (eq G_2e, eq zfock), two-electron part:  */
/*   F_mu nu = sum_{lam sig} Bs_{lam sig} [ cJ (mu nu|lam sig)                */
/*             + cK (mu lam|nu sig) + cKlr (mu lam|nu sig)_lr ],              */
/* Bs = (B + B^T)/2.  Written out by its definition: the block of F for the   */
/* shells (a, b) sums over every ordered pair of shells (c, d), with the      */
/* integral blocks (ab|cd) for the Coulomb term and (ac|bd) for the exchange  */
/* terms.  out receives, for each requested pair (a, b), its na x nb block    */
/* (row-major) one after another.                                            */
int orc_fock_blocks(const orc_basis_t *b, const double *B, double cJ, double cK, double cKlr, double omega,
                    int nthreads, int64_t npairs, const int32_t *pairs, double *out)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    const int ns = b->n_shells, n = b->n_bf;
    oshell_t *sh = load_all(b);
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (npairs + 1));
    off[0] = 0;
    for (int64_t k = 0; k < npairs; ++k)
        off[k + 1] = off[k] + (int64_t)ncart(sh[pairs[2 * k]].l) * ncart(sh[pairs[2 * k + 1]].l);
#pragma omp parallel num_threads(nth)
    {
        real *blk = (real *)malloc(sizeof(real) * 1296);
        real *acc = (real *)malloc(sizeof(real) * 36);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < npairs; ++k) {
            const int a = pairs[2 * k], bb = pairs[2 * k + 1];
            const int na = ncart(sh[a].l), nb = ncart(sh[bb].l);
            const int oa = b->shell_ao_off[a], ob = b->shell_ao_off[bb];
            for (int x = 0; x < na * nb; ++x) acc[x] = 0.0;
            for (int c = 0; c < ns; ++c)
                for (int d = 0; d < ns; ++d) {
                    const int nc = ncart(sh[c].l), nd = ncart(sh[d].l);
                    const int oc = b->shell_ao_off[c], od = b->shell_ao_off[d];
#define BS(i, j) (0.5L * ((real)B[(size_t)(i) * n + (j)] + (real)B[(size_t)(j) * n + (i)]))
                    if (cJ != 0.0) { /* (ab|cd) Bs_cd */
                        const oshell_t *q4[4] = {&sh[a], &sh[bb], &sh[c], &sh[d]};
                        value_block(q4, 0, 0.0, blk, NULL);
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nb; ++j) {
                                real v = 0.0;
                                for (int kk = 0; kk < nc; ++kk)
                                    for (int l = 0; l < nd; ++l)
                                        v += blk[((i * nb + j) * nc + kk) * nd + l] * BS(oc + kk, od + l);
                                acc[i * nb + j] += cJ * v;
                            }
                    }
                    for (int op = 0; op < 2; ++op) { /* (a c|b d) Bs_cd: mu in a, lam in c, nu in b, sig in d */
                        const double cx = op ? cKlr : cK;
                        if (cx == 0.0) continue;
                        const oshell_t *q4[4] = {&sh[a], &sh[c], &sh[bb], &sh[d]};
                        value_block(q4, op, omega, blk, NULL);
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nb; ++j) {
                                real v = 0.0;
                                for (int kk = 0; kk < nc; ++kk)
                                    for (int l = 0; l < nd; ++l)
                                        v += blk[((i * nc + kk) * nb + j) * nd + l] * BS(oc + kk, od + l);
                                acc[i * nb + j] += cx * v;
                            }
                    }
#undef BS
                }
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) out[off[k] + i * nb + j] = (double)acc[i * nb + j];
            (void)oa; (void)ob;
        }
        free(blk);
        free(acc);
    }
    free(off);
    free(sh);
    return 0;
}

/* full AO integral tensor (normalised), tiny bases only: out[((mu*n+nu)*n+lam)*n+sig] */
int orc_eri_tensor(const orc_basis_t *b, int op, double omega, double *out)
{
    init_trip();
    int rc = check_basis(b);
    if (rc) return rc;
    const int ns = b->n_shells, n = b->n_bf;
    oshell_t *sh = load_all(b);
    real *blk = (real *)malloc(sizeof(real) * 1296);
    for (int a = 0; a < ns; ++a)
        for (int bb = 0; bb < ns; ++bb)
            for (int c = 0; c < ns; ++c)
                for (int dd = 0; dd < ns; ++dd) {
                    const oshell_t *q4[4] = {&sh[a], &sh[bb], &sh[c], &sh[dd]};
                    const int nn[4] = {ncart(q4[0]->l), ncart(q4[1]->l), ncart(q4[2]->l), ncart(q4[3]->l)};
                    value_block(q4, op, omega, blk, NULL);
                    const int o[4] = {b->shell_ao_off[a], b->shell_ao_off[bb], b->shell_ao_off[c], b->shell_ao_off[dd]};
                    for (int i = 0; i < nn[0]; ++i)
                        for (int j = 0; j < nn[1]; ++j)
                            for (int k = 0; k < nn[2]; ++k)
                                for (int l = 0; l < nn[3]; ++l)
                                    out[(((size_t)(o[0] + i) * n + o[1] + j) * n + o[2] + k) * n + o[3] + l] =
                                        blk[((i * nn[1] + j) * nn[2] + k) * nn[3] + l];
                }
    free(blk);
    free(sh);
    return 0;
}

/* normalised contraction coefficients (x^l component) for every primitive */
int orc_norm_coefs(const orc_basis_t *b, double *c_out)
{
    for (int s = 0; s < b->n_shells; ++s) {
        const int off = b->shell_prim_off[s], np = b->shell_nprim[s];
        if (np > ORC_MAXPRIM) return -2;
        real z[ORC_MAXPRIM], c[ORC_MAXPRIM];
        for (int k = 0; k < np; ++k) z[k] = b->exps[off + k];
        normalise_shell(b->shell_l[s], np, z, b->coefs + off, c);
        for (int k = 0; k < np; ++k) c_out[off + k] = (double)c[k];
    }
    return 0;
}

/* one primitive Cartesian integral over unnormalised Gaussians
 * (x-A_x)^ax (y-A_y)^ay (z-A_z)^az exp(-za |r-A|^2) ... ; op 0: 1/r, 1: erf(omega r)/r */
double orc_prim_eri(const int32_t *lxyz /* [4][3] */, const double *zeta /* [4] */,
                    const double *centers /* [4][3] */, int op, double omega)
{
    init_trip();
    oshell_t s[4];
    int l[4];
    for (int k = 0; k < 4; ++k) {
        l[k] = lxyz[3 * k] + lxyz[3 * k + 1] + lxyz[3 * k + 2];
        s[k].l = l[k];
        s[k].np = 1;
        s[k].z[0] = zeta[k];
        s[k].c[0] = 1.0;
        for (int x = 0; x < 3; ++x) s[k].A[x] = centers[3 * k + x];
    }
    if (l[0] + l[1] > ORC_MAXLR || l[2] + l[3] > ORC_MAXLR) return NAN;
    const int n[4] = {ncart(l[0]), ncart(l[1]), ncart(l[2]), ncart(l[3])};
    real *blk = (real *)malloc(sizeof(real) * n[0] * n[1] * n[2] * n[3]);
    eri_block(&s[0], &s[1], &s[2], &s[3], op, omega, blk, NULL);
    int p[4];
    for (int k = 0; k < 4; ++k) p[k] = cart_pos(lxyz[3 * k], lxyz[3 * k + 1], lxyz[3 * k + 2]);
    real v = blk[((p[0] * n[1] + p[1]) * n[2] + p[2]) * n[3] + p[3]];
    free(blk);
    return v;
}
