// tdgrad.hip -- host runtime, set-up kernels and C ABI of libtdgrad.so.
//
// Pipeline of one gradient call (all on the caller's stream):
//   density preparation: angular normalisation folded into P0, D = P0 + 2 PDelta
//      and R; shell-block maxima of |P0|, |D|, |R| for the screening bound;
//   task generation: for each of the 21 angular classes and each bra pair, the
//      ket pairs whose density-multiplied Schwarz bound passes (section II.E),
//      found as a Q-sorted prefix per contraction group, then tested exactly;
//   class kernels: one per class (deriv_kernel.hpp, deriv_wave.hpp), accumulating
//      into the per-atom FP64 gradient.
// The plan (tdg_plan_create) holds the normalisation, shell pairs, primitive
// pairs and Schwarz factors, sorted by class, contraction degree and Q (D1 of
// section II.C: presorted shell-pair lists).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tdgrad.h"
#include "class_launch.hpp"
#include "deriv_kernel.hpp"
#include "fock_kernel.hpp"
#include "fock_launch.hpp"
#include "mlp.hpp"

using namespace tdg;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" int tdg_set_error_(int code, const char *msg) { return fail(code, "%s", msg); }
struct tdg_plan;
int tdg_plan_device_(const tdg_plan *pl); // the plan's HIP device (for zvector.hip)

namespace tdg {
void mlp_device_ptrs(const tdg_mlp *m, const float **w, const uint16_t **w1b, const uint16_t **w2b);
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(TDG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------- constants
static constexpr int kPairL[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
static int pair_class(int la, int lb) // la >= lb
{
    static const int tab[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
    return tab[la][lb];
}
static constexpr int kNumClasses = 21;
// class index c <-> (bra pair class PB, ket pair class PK), PB >= PK
static void class_pk(int c, int &pb, int &pk)
{
    int k = 0;
    for (int b = 0; b < 6; ++b)
        for (int q = 0; q <= b; ++q, ++k)
            if (k == c) { pb = b; pk = q; return; }
}

template <class T> struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    int alloc(size_t count)
    {
        if (count <= n && p) return 0;
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
        if (count == 0) return 0;
        if (hipMalloc((void **)&p, count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            return fail(TDG_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
        }
        n = count;
        return 0;
    }
    int upload(const std::vector<T> &h)
    {
        int rc = alloc(h.size());
        if (rc) return rc;
        if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return fail(TDG_EDEVICE, "hipMemcpy upload failed");
        return 0;
    }
    void release()
    {
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// Largest |P0|, |D| and |R| (both orientations) of one ordered shell-pair block, one
// 32-byte record per pair so that a screening bound reads 5 records.
struct __align__(32) BlkMax {
    double p, d, r, pad;
};

struct tdg_plan {
    int device = 0;
    int n_atoms = 0, n_shells = 0, n_prims = 0, n_bf = 0;
    tdg_params_t prm{};
    std::vector<int> shell_atom, shell_l, shell_ao;
    // sorted pairs
    int npair = 0;
    int pc_start[7] = {0};                 // pair-class segments of the sorted list
    std::vector<int> grp_start;            // contraction groups (equal Ka*Kb) inside a class
    std::vector<int> pc_grp_start;         // [7] index into grp_start per pair class
    std::vector<int> pair_sa, pair_sb, pair_K;
    std::vector<double> pair_Q;
    std::vector<int> user_pair_to_sorted;  // by a*(a+1)/2+b with a>=b in caller's shell order
    // device
    DevBuf<double> d_coords;
    DevBuf<int> d_shell_atom, d_shell_ao, d_shell_l;
    DevBuf<int> d_pair_sa, d_pair_sb, d_pair_ppoff, d_pair_npp, d_pair_K;
    DevBuf<double> d_pair_Q;
    DevBuf<double> d_pp_p, d_pp_Px, d_pp_Py, d_pp_Pz, d_pp_c; // per-field copy for the Schwarz kernel
    DevBuf<double> d_pp_rec; // the same eight values per primitive pair as one 64-byte record
    DevBuf<double> d_ang;                  // angular normalisation per AO
    DevBuf<int> d_grp_start;
    // work buffers
    DevBuf<double> d_in;                   // staging of host densities (3 n_bf^2)
    DevBuf<double> d_dens;                 // shell-blocked scaled densities (3 n_bf^2)
    DevBuf<BlkMax> d_bmax;                 // [n_shells^2] shell-block maxima
    DevBuf<double> d_grad;
    DevBuf<unsigned long long> d_mx;       // max of block maxima (bit pattern of a double >= 0)
    DevBuf<int> d_item_cnt;                // per (class, bra pair) survivor counts
    DevBuf<long long> d_item_off;
    DevBuf<unsigned long long> d_prim_cnt; // per class primitive quartets
    DevBuf<unsigned long long> d_cand_cnt; // per class candidates tested by the exact bound
    DevBuf<int2> d_tasks;
    std::vector<int> item_class_off;       // [22] offset of each class's items
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_cls[kNumClasses + 1] = {};   // class start events (and the autotuner's timing)
    std::vector<hipEvent_t> ev_item;           // start and end of every class-kernel item of a call
    // class kernels spread over nstreams streams: the caller's and nstreams - 1 of the plan's
    static constexpr int kMaxAux = 3;
    int nstreams = 1;
    hipStream_t aux[kMaxAux] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kMaxAux] = {};
    int variant[2][kNumClasses];           // kernel variant per (precision, class), numbered as kernel_variant
    bool tf_ok[2][2][kNumClasses];         // transfer-form variants (0, 3) offered: no p/d on B or D and
                                           // the kernel keeps its tables in registers; else 2 (4) runs
    int gpc[2][kNumClasses];               // launch shape per (precision, class): blocks per compute unit
    int bgpc[2][kNumClasses];              // the same for batched calls
    int split[kNumClasses];                // 1: the FP32-routed quartets of the class run in FP32; 0: the
                                           // whole class runs in FP64 (measured faster by the autotuner)
    std::vector<double> pair_pmax;         // largest primitive exponent sum of each sorted pair
    DevBuf<double> d_pair_pmax;
    std::vector<double> pair_famp;         // FP32 error-amplification proxy of each sorted pair
    DevBuf<double> d_pair_famp;
    DevBuf<int> d_item_cnt32;              // per (class, bra pair) FP32-routed survivor counts
    DevBuf<long long> d_item_off32;
    bool tuned[kNumClasses] = {};          // variants of the class measured (on the first chunk holding it)
    DevBuf<double> d_grad_tune;            // scratch gradient for the tuning launches
    DevBuf<int2> d_tune_tasks;             // strided sample of a class's tasks for the autotuner
    DevBuf<int> d_tune_mol;
    // kernel variants of batched calls led by this plan (the first plan of tdg_grad_jk_batch)
    int bvariant[2][kNumClasses];
    int bsplit[kNumClasses];
    bool btuned[kNumClasses] = {};
    // learned screening: estimator and thresholds (log10 of the contribution)
    const tdg_mlp *ml = nullptr;
    double ml_log10 = -1e30, ml_tau_hi = 0.0;
    std::vector<double> pair_pmin;
    DevBuf<double> d_pair_pmin;
    DevBuf<unsigned char> d_keep;
    DevBuf<int2> d_tasks2;
    DevBuf<long long> d_blkcnt, d_segcnt;
    // fused screening: regions per (class, bra contraction group, list), flat index
    // 2 (fgrp_off[class] + group) + list; capacities learned from the previous call
    std::vector<int> pair_grp;             // contraction group of each sorted pair within its pair class
    std::vector<int> fgrp_off;             // [22]
    bool fused_ready = false;
    std::vector<long long> fcap, freg, hcnt;
    DevBuf<unsigned long long> d_ccnt;
    DevBuf<long long> d_fcap, d_freg, d_moves;
    DevBuf<int2> d_ftasks;
    int ncu = 0;                           // compute units of the plan's device
    // copy of the caller's basis (tdg_plan_update_coords rebuilds the plan from it)
    std::vector<double> b_coords, b_exps, b_coefs;
    std::vector<int> b_nprim, b_primoff;
    // deterministic reduction: per-task values and per-block partial gradients
    DevBuf<double> d_tout, d_part;
    // Fock-type matrix calls: the screening keeps one-centre quartets and has one (FP64) list;
    // the accumulator G of F = ang (G + G^T) ang
    int screen_fock = 0;
    DevBuf<double> d_fockG;
    // the caller's functions: Cartesian (sph = 0: the internal layout itself) or with d shells
    // as real solid harmonics (sph = 1: internal Cartesian offsets are cumulative in shell order)
    int sph = 0, n_user = 0;
    std::vector<int> shell_ao_user;
    DevBuf<int> d_shell_ao_user, d_ao_shell_user; // caller's AO offset per shell, shell per caller AO
    // host-side state of the current call
    std::vector<int> h_cnt, h_cnt32;
    std::vector<unsigned long long> h_prim, h_cand;
};

// ======================================================================= normalisation
static double dfact(int n)
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

// normalised contraction coefficients of the x^l component (unit self-overlap)
static void normalise(int l, int np, const double *z, const double *d, double *c)
{
    for (int k = 0; k < np; ++k)
        c[k] = d[k] * std::pow(2.0 * z[k] / M_PI, 0.75) * std::pow(4.0 * z[k], 0.5 * l) / std::sqrt(dfact(2 * l - 1));
    double s = 0.0;
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            const double zz = z[i] + z[j];
            s += c[i] * c[j] * dfact(2 * l - 1) / std::pow(2.0 * zz, l) * std::pow(M_PI / zz, 1.5);
        }
    const double nc = 1.0 / std::sqrt(s);
    for (int k = 0; k < np; ++k) c[k] *= nc;
}

static double ang_factor(int lx, int ly, int lz)
{
    const int l = lx + ly + lz;
    return std::sqrt(dfact(2 * l - 1) / (dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1)));
}

// ======================================================================= shell pairs and Schwarz factors
// Q_ab = sqrt(max over components (mu nu|mu nu)), (ab|ab) by Rys quadrature with
// LA+LB+1 roots, one thread per pair.
template <int LA, int LB>
__global__ void k_schwarz(int npair, const int *pair_sa, const int *pair_sb, const int *ppoff, const int *npp,
                          const int *shell_atom, const double *coords, const double *pp_p, const double *pp_Px,
                          const double *pp_Py, const double *pp_Pz, const double *pp_c, const double *ang_ab,
                          double *Q)
{
    constexpr int NR = LA + LB + 1, NA = ncart(LA), NB = ncart(LB);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npair) return;
    const int sa = pair_sa[i], sb = pair_sb[i];
    double A[3], AB[3];
    for (int d = 0; d < 3; ++d) {
        A[d] = coords[3 * shell_atom[sa] + d];
        AB[d] = A[d] - coords[3 * shell_atom[sb] + d];
    }
    double acc[NA * NB];
#pragma unroll
    for (int k = 0; k < NA * NB; ++k) acc[k] = 0.0;
    const int p0 = ppoff[i], n = npp[i];
    for (int x = 0; x < n; ++x) {
        const double p = pp_p[p0 + x], cx = pp_c[p0 + x];
        const double P[3] = {pp_Px[p0 + x], pp_Py[p0 + x], pp_Pz[p0 + x]};
        for (int y = 0; y < n; ++y) {
            const double q = pp_p[p0 + y], cy = pp_c[p0 + y];
            const double Qc[3] = {pp_Px[p0 + y], pp_Py[p0 + y], pp_Pz[p0 + y]};
            const double ipq = 1.0 / (p + q), rho = p * q * ipq;
            double PQ[3], pq2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                PQ[d] = P[d] - Qc[d];
                pq2 += PQ[d] * PQ[d];
            }
            const double pref = 34.98683665524972 / (p * q) * sqrt(ipq) * cx * cy;
            for (int r = 0; r < NR; ++r) {
                double u, w;
                rys_root<NR>(rho * pq2, r, u, w);
                const double B00 = 0.5 * u * ipq, B10 = 0.5 / p * (1.0 - q * ipq * u), B01 = 0.5 / q * (1.0 - p * ipq * u);
                Rys2D<LA + LB, LA + LB, LA, LB, LB> g[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double PA = P[d] - A[d], QC = Qc[d] - A[d];
                    g[d].build(d == 2 ? pref * w : 1.0, PA - q * ipq * u * PQ[d], QC + p * ipq * u * PQ[d], B10, B01,
                               B00, AB[d], AB[d]);
                }
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int ib = 0; ib < NB; ++ib) {
                        double v = 1.0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const int ii = kCart.v[LA][ia][d], jj = kCart.v[LB][ib][d];
                            v *= g[d].X[ii][jj][ii][jj];
                        }
                        acc[ia * NB + ib] += v;
                    }
            }
        }
    }
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < NA * NB; ++k) mx = fmax(mx, acc[k] * ang_ab[k]);
    Q[i] = sqrt(mx);
}

// ======================================================================= density preparation
// scaled densities and shell-block maxima; one thread per shell block (a, c)
// max over the block products that Gamma contains (reading R10), times Q_ab Q_cd;
// ab is the bra pair's record (uniform across a wavefront)
__device__ __forceinline__ double block_bound(const BlkMax &ab, const BlkMax *bm, size_t n, int a, int b, int c,
                                              int d)
{
    const BlkMax cd = bm[(size_t)c * n + d], ac = bm[(size_t)a * n + c], bd = bm[(size_t)b * n + d];
    const BlkMax ad = bm[(size_t)a * n + d], bc = bm[(size_t)b * n + c];
    double m = ab.d * cd.p;
    m = fmax(m, ab.p * cd.d);
    m = fmax(m, ab.r * cd.r);
    m = fmax(m, ac.d * bd.p);
    m = fmax(m, bd.d * ac.p);
    m = fmax(m, ad.d * bc.p);
    m = fmax(m, bc.d * ad.p);
    m = fmax(m, ac.r * bd.r);
    m = fmax(m, ad.r * bc.r);
    return m;
}

// Real solid-harmonic d functions in terms of the unit-normalised Cartesian d components
// (xx, xy, xz, yy, yz, zz): xy, yz, (2 zz - xx - yy)/2, xz, (sqrt 3 / 2)(xx - yy), each of
// unit norm (the Cartesian components overlap as <xx|yy> = 1/3, <xx|xx> = 1).
// sph_coef(l, sph, p, i): coefficient of Cartesian component i in function p of a shell of
// momentum l (identity for s, p and for Cartesian d).
__device__ __forceinline__ double sph_coef(int l, int sph, int p, int i)
{
    if (l != 2 || !sph) return p == i ? 1.0 : 0.0;
    constexpr double h = 0.5, r3h = 0.86602540378443864676; // 1/2, sqrt(3)/2
    switch (p) {
    case 0: return i == 1 ? 1.0 : 0.0;                                   // xy
    case 1: return i == 4 ? 1.0 : 0.0;                                   // yz
    case 2: return i == 5 ? 1.0 : ((i == 0 || i == 3) ? -h : 0.0);       // z^2
    case 3: return i == 2 ? 1.0 : 0.0;                                   // xz
    default: return i == 0 ? r3h : (i == 3 ? -r3h : 0.0);                // x^2 - y^2
    }
}
__device__ __forceinline__ int nfun(int l, int sph) { return (l == 2 && sph) ? 5 : ncart(l); }

// Cartesian element (i, j) of the block (a, c) of a caller matrix X (dimension n_in, caller
// offsets ua, uc): X_cart = T_a^T X T_c for solid-harmonic shells, X itself otherwise.
__device__ __forceinline__ double cart_elem(const double *X, int n_in, int la, int ua, int lc, int uc, int sph, int i,
                                            int j)
{
    if (!sph || (la != 2 && lc != 2)) return X[(size_t)(ua + i) * n_in + uc + j];
    double v = 0.0;
    const int fa = nfun(la, sph), fc = nfun(lc, sph);
    for (int p = 0; p < fa; ++p) {
        const double tp = sph_coef(la, sph, p, i);
        if (tp == 0.0) continue;
        for (int q = 0; q < fc; ++q) {
            const double tq = sph_coef(lc, sph, q, j);
            if (tq != 0.0) v += tp * X[(size_t)(ua + p) * n_in + uc + q] * tq;
        }
    }
    return v;
}

// One thread per ordered shell pair (a, c): the pair's record of the shell-blocked
// densities (P, D = P0 + 2 PDelta and R blocks, angular factors folded in; layout in
// deriv_kernel.hpp) and the block maxima used by the screening bound.
__global__ void k_density_prep(int n_shells, int n_bf, const int *shell_l, const int *shell_ao, const double *ang,
                               const double *P0, const double *PD, const double *R, double *dens, BlkMax *bmax,
                               unsigned long long *mx, int sph, int n_in, const int *shell_ao_in)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n_shells * n_shells) return;
    const int a = (int)(idx / n_shells), c = (int)(idx % n_shells);
    const int la = shell_l[a], lc = shell_l[c];
    const int oa = shell_ao[a], oc = shell_ao[c], na = ncart(la), nc = ncart(lc);
    // caller layout: the same offsets for Cartesian functions, else the caller's
    const int ua = sph ? shell_ao_in[a] : oa, uc = sph ? shell_ao_in[c] : oc;
    double *rec = dens + dens_rec(n_bf, oa, na, oc);
    double vp = 0.0, vd = 0.0, vr = 0.0;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nc; ++j) {
            const double p = cart_elem(P0, n_in, la, ua, lc, uc, sph, i, j);
            const double d = p + 2.0 * cart_elem(PD, n_in, la, ua, lc, uc, sph, i, j);
            const double rr = cart_elem(R, n_in, la, ua, lc, uc, sph, i, j);
            const double rt = cart_elem(R, n_in, lc, uc, la, ua, sph, j, i);
            const double s = ang[oa + i] * ang[oc + j];
            rec[i * nc + j] = s * p;
            rec[na * nc + i * nc + j] = s * d;
            rec[2 * na * nc + i * nc + j] = s * rr;
            vp = fmax(vp, fabs(p));
            vd = fmax(vd, fabs(d));
            vr = fmax(vr, fmax(fabs(rr), fabs(rt)));
        }
    BlkMax bm;
    bm.p = vp; bm.d = vd; bm.r = vr; bm.pad = 0.0;
    bmax[idx] = bm;
    const double m = fmax(vp, fmax(vd, vr));
    atomicMax(mx, (unsigned long long)__double_as_longlong(m)); // non-negative doubles order as integers
}

// Fock-type matrix input: one thread per ordered shell pair (a, c); the pair's record holds
// Bs = (B + B^T)/2 with the angular factors folded in (first slot of the record layout of
// deriv_kernel.hpp).  The block maxima take the screening bound's P slot (|Bs|) with the D
// slot at one and R at zero, so that the gradient's bound becomes Q_ab Q_cd times the
// largest |Bs| of the six blocks a quartet reads; mx receives the square root of the
// largest |Bs| (its square scales the prefix cut).
__global__ void k_fock_prep(int n_shells, int n_bf, const int *shell_l, const int *shell_ao, const double *ang,
                            const double *B, double *dens, BlkMax *bmax, unsigned long long *mx, int sph, int n_in,
                            const int *shell_ao_in)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n_shells * n_shells) return;
    const int a = (int)(idx / n_shells), c = (int)(idx % n_shells);
    const int la = shell_l[a], lc = shell_l[c];
    const int oa = shell_ao[a], oc = shell_ao[c], na = ncart(la), nc = ncart(lc);
    const int ua = sph ? shell_ao_in[a] : oa, uc = sph ? shell_ao_in[c] : oc;
    double *rec = dens + dens_rec(n_bf, oa, na, oc);
    double vb = 0.0;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nc; ++j) {
            const double b = 0.5 * (cart_elem(B, n_in, la, ua, lc, uc, sph, i, j) +
                                    cart_elem(B, n_in, lc, uc, la, ua, sph, j, i));
            rec[i * nc + j] = ang[oa + i] * ang[oc + j] * b;
            vb = fmax(vb, fabs(b));
        }
    BlkMax bm;
    bm.p = vb; bm.d = 1.0; bm.r = 0.0; bm.pad = 0.0;
    bmax[idx] = bm;
    atomicMax(mx, (unsigned long long)__double_as_longlong(sqrt(vb)));
}

// F = ang (G + G^T) ang, one thread per element; with solid-harmonic d shells the element
// (mu, nu) of the caller's matrix is T_a F_cart T_c^T over the Cartesian components of the
// two shells (mu in shell a, nu in shell c)
__global__ void k_fock_finish(int n_bf, const double *ang, const double *G, double *F, int sph, int n_out,
                              const int *ao_shell_out, const int *shell_ao_out, const int *shell_ao,
                              const int *shell_l)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n_out * n_out) return;
    const int mu = (int)(idx / n_out), nu = (int)(idx % n_out);
    if (!sph) {
        F[idx] = ang[mu] * ang[nu] * (G[idx] + G[(size_t)nu * n_bf + mu]);
        return;
    }
    const int a = ao_shell_out[mu], c = ao_shell_out[nu];
    const int la = shell_l[a], lc = shell_l[c], oa = shell_ao[a], oc = shell_ao[c];
    const int p = mu - shell_ao_out[a], q = nu - shell_ao_out[c];
    double v = 0.0;
    for (int i = 0; i < ncart(la); ++i) {
        const double tp = sph_coef(la, sph, p, i);
        if (tp == 0.0) continue;
        for (int j = 0; j < ncart(lc); ++j) {
            const double tq = sph_coef(lc, sph, q, j);
            if (tq == 0.0) continue;
            const size_t ij = (size_t)(oa + i) * n_bf + oc + j, ji = (size_t)(oc + j) * n_bf + oa + i;
            v += tp * tq * ang[oa + i] * ang[oc + j] * (G[ij] + G[ji]);
        }
    }
    F[idx] = v;
}

// ======================================================================= screening and task generation
struct ScreenArgs {
    int cls, pb, pk;
    int bra0, nbra;               // bra pairs of this class: sorted indices [bra0, bra0+nbra)
    int grp0, grp1;               // contraction groups of the ket pair class
    const int *grp_start;         // [ngroups+1]
    const int *pair_sa, *pair_sb, *pair_K, *shell_atom;
    const double *pair_Q;
    const BlkMax *bmax;
    int n_shells;
    double tau;
    const unsigned long long *mx;
    int *item_cnt;                // count pass output, per bra (FP64-routed tasks)
    const long long *item_off;    // fill pass input (absolute task index of each bra's first task)
    int *item_cnt32;              // mixed precision: FP32-routed counts / offsets
    const long long *item_off32;
    const double *pair_pmax, *pair_famp;
    int tau_rel;                  // 1: the threshold is tau times the largest density factor (the
                                  // screening of a matrix scaled to unit largest element)
    int keep_one_center;          // 1: one-centre quartets are kept (Fock-type matrix; the gradient
                                  // skips them: their derivative sum vanishes, eq ti)
    int mixed;                    // 1: route to FP32 unless bound >= tau64 or an exponent sum >= p64
    double tau64, p64;
    int2 *tasks;
    unsigned long long *prim_cnt; // per class
    unsigned long long *cand_cnt; // per class
    // fused pass: per contraction group gb of the bra pair class, task counters, regions of the
    // task buffer and their capacities, [2 gb + list] (list 0 FP64, 1 FP32)
    int bgrp0, bgrp1;             // contraction groups of the bra pair class
    unsigned long long *ccnt;
    const long long *freg, *fcap;
};

// One wavefront per bra pair.  MODE 0 counts the survivors per bra (item_cnt), MODE 1
// writes them at the offsets item_off computed from those counts, MODE 2 does both in
// one launch: the survivors are counted while the chunks' ballot masks are kept in LDS,
// one atomic per bra claims space in the region of its (class, bra contraction group,
// list) -- so that bras of one contraction degree stay together -- (tasks beyond a
// region's capacity are counted but not written), and the tasks are written from the
// stored masks.  In the mixed-precision mode a survivor goes to the FP32 list
// when its bound times the two pairs' proxies is < tau64 and no primitive exponent
// sum reaches p64; otherwise to the FP64 list.
//
// All classes (of one molecule) are screened by one launch: the per-class fields travel in
// a table in the kernel arguments, wavefronts [wave_start[k], wave_start[k+1]) serve item k.
struct ScreenItem {
    int cls, pb, pk, bra0, nbra, grp0, grp1, item_base, bgrp0, bgrp1, fgrp_base;
};
struct ScreenTable {
    int n;
    int wave_start[kNumClasses + 1];
    ScreenItem it[kNumClasses];
};

template <int MODE>
__global__ void __launch_bounds__(256) k_screen(ScreenArgs s, const ScreenTable t)
{
    constexpr int MAXCH = 96; // chunks whose masks a wavefront keeps in LDS (MODE 2)
    constexpr int MAXG = 32;  // ket contraction groups whose prefix ends it keeps (MODE 2)
    __shared__ unsigned long long s_mask[MODE == 2 ? 4 : 1][MODE == 2 ? MAXCH : 1][2];
    __shared__ int s_gend[MODE == 2 ? 4 : 1][MODE == 2 ? MAXG : 1];
    // wavefront index in 64-bit arithmetic: a large system has more than 2^26 (class, bra) items
    const int gw = __builtin_amdgcn_readfirstlane(
        (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave));
    const int lane = threadIdx.x % kWave;
    const int wv = (threadIdx.x / kWave) & 3;
    if (gw >= t.wave_start[t.n]) return;
    int ci = 0;
    while (ci + 1 < t.n && t.wave_start[ci + 1] <= gw) ++ci;
    {
        const ScreenItem &it = t.it[ci];
        s.cls = it.cls; s.pb = it.pb; s.pk = it.pk; s.bra0 = it.bra0; s.nbra = it.nbra;
        s.grp0 = it.grp0; s.grp1 = it.grp1; s.bgrp0 = it.bgrp0; s.bgrp1 = it.bgrp1;
        if constexpr (MODE == 2) {
            s.ccnt += 2 * it.fgrp_base; s.freg += 2 * it.fgrp_base; s.fcap += 2 * it.fgrp_base;
        } else {
            s.item_cnt += it.item_base; s.item_off += it.item_base;
            s.item_cnt32 += it.item_base; s.item_off32 += it.item_base;
        }
    }
    const int wid = gw - t.wave_start[ci];
    const int i = s.bra0 + wid;
    const int a = s.pair_sa[i], b = s.pair_sb[i];
    const double Qi = s.pair_Q[i];
    const double mxv = __longlong_as_double((long long)*s.mx);
    const double tau = s.tau_rel ? s.tau * mxv * mxv : s.tau;
    const double cut = tau > 0.0 ? tau / (Qi * mxv * mxv) : -1.0;
    const int ata = s.shell_atom[a], atb = s.shell_atom[b];
    const BlkMax bm_ab = s.bmax[(size_t)a * s.n_shells + b];
    const int Ki = s.pair_K[i];
    const bool hot_i = s.mixed && s.pair_pmax[i] >= s.p64;
    const double famp_i = s.mixed ? s.pair_famp[i] : 0.0;
    // survivor flags of ket j for this bra (j must be a valid index; valid = false gives
    // no survivor).  Branch-free, so that the loads of several calls can be in flight
    // together.
    auto test = [&](int j, bool valid, bool &keep, bool &to32) {
        const int c = s.pair_sa[j], d = s.pair_sb[j];
        const bool one_center = !s.keep_one_center && (s.shell_atom[c] == ata) && (s.shell_atom[d] == ata) &&
                                (atb == ata);
        const double bnd = Qi * s.pair_Q[j] * block_bound(bm_ab, s.bmax, s.n_shells, a, b, c, d);
        keep = valid && !one_center && (tau <= 0.0 || bnd >= tau);
        to32 = keep && s.mixed && !hot_i && bnd * famp_i * s.pair_famp[j] < s.tau64 && s.pair_pmax[j] < s.p64;
    };
    // end of the Q-sorted prefix of group g that can pass the bound: the first ket with
    // Q < cut (Q sorted descending), found by the wavefront together -- each step probes
    // 64 evenly spaced kets and keeps the interval between the last one at or above the
    // cut and the first one below, so a group of n kets takes about log64(n) + 1
    // dependent loads instead of log2(n)
    auto group_end = [&](int g) {
        const int g0 = s.grp_start[g], g1 = s.grp_start[g + 1];
        int hi = g1;
        if (cut > 0.0) {
            int lo = g0; // invariant: Q >= cut below lo, Q < cut from hi on
            while (hi - lo > kWave) {
                const long long span = hi - lo;
                const int p = lo + (int)(span * lane / kWave);
                const int t = __popcll(__ballot(s.pair_Q[p] >= cut));
                const int nlo = t > 0 ? lo + (int)(span * (t - 1) / kWave) + 1 : lo;
                const int nhi = t < kWave ? lo + (int)(span * t / kWave) : hi;
                lo = nlo;
                hi = nhi;
            }
            const int p = lo + lane;
            hi = lo + __popcll(__ballot(p < hi && s.pair_Q[p] >= cut));
        }
        if (s.pb == s.pk && hi > i + 1) hi = i + 1; // canonical: ket index <= bra index
        return hi;
    };
    const unsigned long long below = (1ull << lane) - 1ull;
    long long out = MODE == 1 ? s.item_off[wid] : 0, out32 = (MODE == 1 && s.mixed) ? s.item_off32[wid] : 0;
    int cnt = 0, cnt32 = 0, k = 0;
    unsigned long long prim = 0, cand = 0;
    constexpr int UNR = 4; // chunks of 64 kets tested together
    for (int g = s.grp0; g < s.grp1; ++g) {
        const int g0 = s.grp_start[g], hi = group_end(g);
        if (MODE == 2 && g - s.grp0 < MAXG && lane == 0) s_gend[wv][g - s.grp0] = hi;
        if (hi > g0) cand += hi - g0;
        for (int jb = g0; jb < hi; jb += UNR * kWave) {
            bool kp[UNR], t3[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int j = jb + u * kWave + lane;
                test(j < hi ? j : hi - 1, j < hi, kp[u], t3[u]);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u, ++k) {
                const int j0 = jb + u * kWave;
                if (j0 >= hi) break; // wavefront-uniform
                const int j = j0 + lane;
                const bool keep = kp[u], to32 = t3[u];
                if (keep) prim += (unsigned long long)Ki * s.pair_K[j];
                const unsigned long long m64 = __ballot(keep && !to32), m32 = __ballot(to32);
                if (MODE == 1 && keep) {
                    const long long pos = to32 ? out32 + __popcll(m32 & below) : out + __popcll(m64 & below);
                    s.tasks[pos] = make_int2(i, j);
                }
                if (MODE == 2 && k < MAXCH && lane == 0) {
                    s_mask[wv][k][0] = m64;
                    s_mask[wv][k][1] = m32;
                }
                out += __popcll(m64);
                out32 += __popcll(m32);
                cnt += __popcll(m64);
                cnt32 += __popcll(m32);
            }
        }
    }
    if (MODE != 1) {
        for (int off = 32; off > 0; off >>= 1) prim += __shfl_xor(prim, off);
        if (lane == 0) {
            if (MODE == 0) {
                s.item_cnt[wid] = cnt;
                if (s.mixed) s.item_cnt32[wid] = cnt32;
            }
            atomicAdd(s.prim_cnt + s.cls, prim);
            atomicAdd(s.cand_cnt + s.cls, cand);
        }
    }
    if constexpr (MODE == 2) {
        if (cnt + cnt32 == 0) return;
        int gb = 0; // contraction group of the bra within its pair class
        while (s.bgrp0 + gb + 1 < s.bgrp1 && s.grp_start[s.bgrp0 + gb + 1] <= i) ++gb;
        const long long reg64 = s.freg[2 * gb], cap64 = s.fcap[2 * gb];
        const long long reg32 = s.freg[2 * gb + 1], cap32 = s.fcap[2 * gb + 1];
        unsigned long long b64 = 0, b32 = 0;
        if (lane == 0) {
            if (cnt) b64 = atomicAdd(s.ccnt + 2 * gb, (unsigned long long)cnt);
            if (cnt32) b32 = atomicAdd(s.ccnt + 2 * gb + 1, (unsigned long long)cnt32);
        }
        b64 = __shfl(b64, 0);
        b32 = __shfl(b32, 0);
        wave_sync(); // the masks lane 0 stored
        long long o64 = (long long)b64, o32 = (long long)b32;
        k = 0;
        for (int g = s.grp0; g < s.grp1; ++g) {
            const int g0 = s.grp_start[g], hi = g - s.grp0 < MAXG ? s_gend[wv][g - s.grp0] : group_end(g);
            for (int j0 = g0; j0 < hi; j0 += kWave, ++k) {
                const int j = j0 + lane;
                unsigned long long m64, m32;
                if (k < MAXCH) {
                    m64 = s_mask[wv][k][0];
                    m32 = s_mask[wv][k][1];
                } else {
                    bool keep, to32;
                    test(j < hi ? j : hi - 1, j < hi, keep, to32);
                    m64 = __ballot(keep && !to32);
                    m32 = __ballot(to32);
                }
                if ((m64 >> lane) & 1ull) {
                    const long long pos = o64 + __popcll(m64 & below);
                    if (pos < cap64) s.tasks[reg64 + pos] = make_int2(i, j);
                } else if ((m32 >> lane) & 1ull) {
                    const long long pos = o32 + __popcll(m32 & below);
                    if (pos < cap32) s.tasks[reg32 + pos] = make_int2(i, j);
                }
                o64 += __popcll(m64);
                o32 += __popcll(m32);
            }
        }
    }
}

// autotuner sample of a task range: every stride-th task (and its molecule index)
__global__ void k_sample_tasks(const int2 *src, const int *src_mol, long long b, long long stride, long long n,
                               int2 *dst, int *dst_mol)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = src[b + i * stride];
    if (src_mol) dst_mol[i] = src_mol[b + i * stride];
}

__global__ void k_zero(double *p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// fused screening: copy the used part of every region to its place in the packed list;
// one block per piece of a region, moves[3 r] = (source, destination, count)
constexpr long long kPackPiece = 4096; // tasks per piece
constexpr long long kTuneTasks = 1LL << 21; // tasks per class the autotuner times at most
// blocks per compute unit of a class launch (the blocks stride over the class's tasks);
// measured on the 60-atom chain: 2, 4, 8, 16, 32 give 14.0, 12.6, 11.7, 11.4, 11.3 ms of
// mixed-path class kernels
constexpr int kGridPerCU = 16;

__global__ void k_pack_regions(const int2 *src, int2 *dst, const long long *moves)
{
    const long long from = moves[3 * blockIdx.x], to = moves[3 * blockIdx.x + 1], n = moves[3 * blockIdx.x + 2];
    for (long long k = threadIdx.x; k < n; k += blockDim.x) dst[to + k] = src[from + k];
}

// ======================================================================= deterministic reduction
// Per-atom sums of per-quartet values vals[t][12] (centres A, B, C, D of task t) in a
// fixed order: block b sums the tasks [b per_block, (b+1) per_block) in task order into
// partial[b][3 n_atoms], then k_det_final adds the blocks in block order.  Inside a
// block (one wavefront) gradient entry g belongs to lane g % 64 alone, which adds its
// values one task after another, so no two additions to an entry race and the result
// does not depend on timing.
constexpr int kDetBlocks = 1024;            // partial gradients per reduction at most
constexpr long long kDetChunk = 1LL << 23;  // tasks per chunk in deterministic mode (768 MiB of values)

__global__ void __launch_bounds__(64) k_det_reduce(const int2 *tasks, long long n, long long per_block,
                                                   const double *vals, const int *pair_sa, const int *pair_sb,
                                                   const int *shell_atom, int n_atoms, int use_lds, double *partial)
{
    extern __shared__ double s_acc[];
    const int lane = threadIdx.x;
    const int n3 = 3 * n_atoms;
    double *acc = use_lds ? s_acc : partial + (size_t)blockIdx.x * n3;
    for (int g = lane; g < n3; g += kWave) acc[g] = 0.0;
    const long long t0 = (long long)blockIdx.x * per_block;
    const long long t1 = t0 + per_block < n ? t0 + per_block : n;
    for (long long t = t0; t < t1; ++t) {
        const int2 tk = tasks[t];
        const int at[4] = {shell_atom[pair_sa[tk.x]], shell_atom[pair_sb[tk.x]], shell_atom[pair_sa[tk.y]],
                           shell_atom[pair_sb[tk.y]]};
        const double *v = vals + 12 * t;
#pragma unroll
        for (int X = 0; X < 4; ++X)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int g = 3 * at[X] + d;
                if (g % kWave == lane) acc[g] += v[3 * X + d];
            }
    }
    if (use_lds)
        for (int g = lane; g < n3; g += kWave) partial[(size_t)blockIdx.x * n3 + g] = acc[g];
}

// grad[g] += sum over blocks b of partial[b][g]: one wavefront per entry, lanes take the
// blocks lane, lane + 64, ... in order, then a fixed butterfly over the lanes
__global__ void __launch_bounds__(256) k_det_final(const double *partial, int nblk, int n3, double *grad)
{
    const int g = blockIdx.x * 4 + threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (g >= n3) return;
    double v = 0.0;
    for (int b = lane; b < nblk; b += kWave) v += partial[(size_t)b * n3 + g];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) grad[g] += v;
}

// ======================================================================= dispatch
// ======================================================================= learned screening
// Features of a shell quartet for the contribution estimator (10 used of 16):
//   log10 Q_ab, log10 Q_cd, log10 of the largest density-block product (all /10),
//   log10 of the smallest and largest primitive exponent sums of both pairs (/4),
//   distance between the pairs' bond midpoints (/10), total angular momentum (/8),
//   |AB| + |CD| (/10).
struct FeatArgs {
    const int *pair_sa, *pair_sb, *shell_atom, *shell_l;
    const double *pair_Q, *pair_pmin, *pair_pmax, *coords;
    const BlkMax *bmax;
    int n_shells;
};

__device__ inline void quartet_features(const FeatArgs &f, int bra, int ket, float *x)
{
    const int a = f.pair_sa[bra], b = f.pair_sb[bra], c = f.pair_sa[ket], d = f.pair_sb[ket];
    const size_t n = f.n_shells;
    const double m = block_bound(f.bmax[(size_t)a * n + b], f.bmax, n, a, b, c, d);
    const double *A = f.coords + 3 * f.shell_atom[a], *B = f.coords + 3 * f.shell_atom[b];
    const double *C = f.coords + 3 * f.shell_atom[c], *D = f.coords + 3 * f.shell_atom[d];
    double ab2 = 0.0, cd2 = 0.0, r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        ab2 += (A[k] - B[k]) * (A[k] - B[k]);
        cd2 += (C[k] - D[k]) * (C[k] - D[k]);
        const double dm = 0.5 * (A[k] + B[k]) - 0.5 * (C[k] + D[k]);
        r2 += dm * dm;
    }
    x[0] = (float)(log10(fmax(f.pair_Q[bra], 1e-300)) * 0.1);
    x[1] = (float)(log10(fmax(f.pair_Q[ket], 1e-300)) * 0.1);
    x[2] = (float)(log10(fmax(m, 1e-300)) * 0.1);
    x[3] = (float)(log10(f.pair_pmin[bra]) * 0.25);
    x[4] = (float)(log10(f.pair_pmin[ket]) * 0.25);
    x[5] = (float)(log10(f.pair_pmax[bra]) * 0.25);
    x[6] = (float)(log10(f.pair_pmax[ket]) * 0.25);
    x[7] = (float)(sqrt(r2) * 0.1);
    x[8] = (float)((f.shell_l[a] + f.shell_l[b] + f.shell_l[c] + f.shell_l[d]) * 0.125);
    x[9] = (float)((sqrt(ab2) + sqrt(cd2)) * 0.1);
    for (int k = 10; k < MLP_IN; ++k) x[k] = 0.f;
}

// veto of the estimator: keep[t] = 0 when the predicted log10 contribution (target
// scaled by 1/10) is below the threshold and the screening bound is below tau_hi
__global__ void __launch_bounds__(256) k_ml_filter(const int2 *tasks, long long n, FeatArgs f, const float *w,
                                                   const uint16_t *w1b, const uint16_t *w2b, float thr, double tau_hi,
                                                   unsigned char *keep)
{
    __shared__ MlpShared S;
    __shared__ MlpWave W[4];
    mlp_load_shared(S, w1b, w2b, w);
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const long long stride = (long long)gridDim.x * 256;
    for (long long base = (long long)blockIdx.x * 256 + wave * 64; base < n; base += stride) {
        const long long t = base + lane;
        float x[MLP_IN];
        double bound = 0.0;
        if (t < n) {
            const int2 tk = tasks[t];
            quartet_features(f, tk.x, tk.y, x);
            bound = pow(10.0, 10.0 * ((double)x[0] + (double)x[1] + (double)x[2]));
        } else {
            for (int k = 0; k < MLP_IN; ++k) x[k] = 0.f;
        }
        const float pred = mlp_forward_wave(S, W[wave], x, lane);
        if (t < n) keep[t] = (pred >= thr || bound >= tau_hi) ? 1 : 0;
    }
}

// order-preserving compaction: per-block counts, one-block exclusive scan, scatter
__global__ void __launch_bounds__(1024) k_count_keep(const unsigned char *keep, long long n, long long *blk)
{
    __shared__ int s[16];
    const long long i = (long long)blockIdx.x * 1024 + threadIdx.x;
    const unsigned long long m = __ballot(i < n && keep[i]);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        long long c = 0;
        for (int k = 0; k < 16; ++k) c += s[k];
        blk[blockIdx.x] = c;
    }
}

__global__ void __launch_bounds__(1024) k_scan_blocks(long long *blk, long long nb, long long *total)
{
    __shared__ long long part[1024];
    // each thread scans a contiguous chunk, then the chunk sums are scanned
    const long long chunk = (nb + 1023) / 1024;
    const long long b0 = threadIdx.x * chunk, b1 = b0 + chunk < nb ? b0 + chunk : nb;
    long long sum = 0;
    for (long long b = b0; b < b1; ++b) sum += blk[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int k = 0; k < 1024; ++k) {
            const long long v = part[k];
            part[k] = acc;
            acc += v;
        }
        *total = acc;
    }
    __syncthreads();
    long long acc = part[threadIdx.x];
    for (long long b = b0; b < b1; ++b) {
        const long long v = blk[b];
        blk[b] = acc;
        acc += v;
    }
}

__global__ void __launch_bounds__(1024) k_scatter_keep(const int2 *in, const unsigned char *keep, long long n,
                                                       const long long *blk, int2 *out)
{
    __shared__ int s[16];
    const long long i = (long long)blockIdx.x * 1024 + threadIdx.x;
    const bool k = i < n && keep[i];
    const unsigned long long m = __ballot(k);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s[w] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int q = 0; q < w; ++q) before += s[q];
    if (k) out[blk[blockIdx.x] + before + __popcll(m & ((1ull << lane) - 1ull))] = in[i];
}

// training data: features of sampled tasks and the log10 (scaled by 1/10) of the largest
// of each task's twelve gradient contributions
__global__ void k_collect(const int2 *tasks, long long n, long long stride, FeatArgs f, const double *contrib,
                          float *feat, float *target, long long cap, long long out0)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long t = s * stride;
    if (t >= n || out0 + s >= cap) return;
    const int2 tk = tasks[t];
    float x[MLP_IN];
    quartet_features(f, tk.x, tk.y, x);
    for (int k = 0; k < MLP_IN; ++k) feat[(out0 + s) * MLP_IN + k] = x[k];
    double mx = 0.0;
    for (int k = 0; k < 12; ++k) mx = fmax(mx, fabs(contrib[12 * t + k]));
    target[out0 + s] = (float)(log10(fmax(mx, 1e-30)) * 0.1);
}

static const LaunchFn kLaunch[kNumClasses] = {
    tdg_launch_class_0,  tdg_launch_class_1,  tdg_launch_class_2,  tdg_launch_class_3,  tdg_launch_class_4,
    tdg_launch_class_5,  tdg_launch_class_6,  tdg_launch_class_7,  tdg_launch_class_8,  tdg_launch_class_9,
    tdg_launch_class_10, tdg_launch_class_11, tdg_launch_class_12, tdg_launch_class_13, tdg_launch_class_14,
    tdg_launch_class_15, tdg_launch_class_16, tdg_launch_class_17, tdg_launch_class_18, tdg_launch_class_19,
    tdg_launch_class_20};
static const FockFn kFock[kNumClasses] = {
    tdg_fock_class_0,  tdg_fock_class_1,  tdg_fock_class_2,  tdg_fock_class_3,  tdg_fock_class_4,
    tdg_fock_class_5,  tdg_fock_class_6,  tdg_fock_class_7,  tdg_fock_class_8,  tdg_fock_class_9,
    tdg_fock_class_10, tdg_fock_class_11, tdg_fock_class_12, tdg_fock_class_13, tdg_fock_class_14,
    tdg_fock_class_15, tdg_fock_class_16, tdg_fock_class_17, tdg_fock_class_18, tdg_fock_class_19,
    tdg_fock_class_20};
static const ScratchFn kScratch[kNumClasses] = {
    tdg_class_scratch_0,  tdg_class_scratch_1,  tdg_class_scratch_2,  tdg_class_scratch_3,  tdg_class_scratch_4,
    tdg_class_scratch_5,  tdg_class_scratch_6,  tdg_class_scratch_7,  tdg_class_scratch_8,  tdg_class_scratch_9,
    tdg_class_scratch_10, tdg_class_scratch_11, tdg_class_scratch_12, tdg_class_scratch_13, tdg_class_scratch_14,
    tdg_class_scratch_15, tdg_class_scratch_16, tdg_class_scratch_17, tdg_class_scratch_18, tdg_class_scratch_19,
    tdg_class_scratch_20};

static int class_ncomp(int c)
{
    int pb, pk;
    class_pk(c, pb, pk);
    return ncart(kPairL[pb][0]) * ncart(kPairL[pb][1]) * ncart(kPairL[pk][0]) * ncart(kPairL[pk][1]);
}

// default variant before measurement: the wave-per-quartet kernel for classes whose
// per-lane register tables would not fit (N >= 81 Cartesian components)
// variant of a class when nothing is tuned (the autotuner's usual choice on the chain and
// droplet workloads): per-range layouts for the smallest classes, the collapsed team
// kernel in between, one wavefront per quartet for (dd|dd)
static int default_variant(int c)
{
    const int n = class_ncomp(c);
    if (n <= 3) return 3;
    if (n <= 9) return 4;
    return n >= 1296 ? 1 : 2;
}
static constexpr int kNumVariants = 5;

template <int LA, int LB>
static void launch_schwarz(tdg_plan *pl, int i0, int n, const double *ang_ab, double *Q)
{
    const int bs = 64;
    hipLaunchKernelGGL((k_schwarz<LA, LB>), dim3((n + bs - 1) / bs), dim3(bs), 0, 0, n, pl->d_pair_sa.p + i0,
                       pl->d_pair_sb.p + i0, pl->d_pair_ppoff.p + i0, pl->d_pair_npp.p + i0, pl->d_shell_atom.p,
                       pl->d_coords.p, pl->d_pp_p.p, pl->d_pp_Px.p, pl->d_pp_Py.p, pl->d_pp_Pz.p, pl->d_pp_c.p,
                       ang_ab, Q + i0);
}

// ======================================================================= plan
static int build_plan(tdg_plan *pl, const tdg_basis_t *b)
{
    const int ns = b->n_shells;
    pl->n_atoms = b->n_atoms;
    pl->n_shells = ns;
    pl->n_prims = b->n_prims;
    pl->shell_atom.assign(b->shell_atom, b->shell_atom + ns);
    pl->shell_l.assign(b->shell_l, b->shell_l + ns);
    pl->sph = b->spherical ? 1 : 0;
    pl->shell_ao_user.assign(b->shell_ao_off, b->shell_ao_off + ns);
    if (pl->sph) { // internal Cartesian functions, cumulative in shell order
        pl->shell_ao.resize(ns);
        int o = 0;
        for (int s = 0; s < ns; ++s) {
            pl->shell_ao[s] = o;
            o += ncart(b->shell_l[s]);
        }
    } else {
        pl->shell_ao = pl->shell_ao_user;
    }
    pl->b_coords.assign(b->coords, b->coords + 3 * b->n_atoms);
    pl->b_exps.assign(b->exps, b->exps + b->n_prims);
    pl->b_coefs.assign(b->coefs, b->coefs + b->n_prims);
    pl->b_nprim.assign(b->shell_nprim, b->shell_nprim + ns);
    pl->b_primoff.assign(b->shell_prim_off, b->shell_prim_off + ns);
    int nbf = 0, nuser = 0;
    for (int s = 0; s < ns; ++s) {
        nbf = std::max(nbf, pl->shell_ao[s] + ncart(b->shell_l[s]));
        nuser = std::max(nuser, b->shell_ao_off[s] + ((pl->sph && b->shell_l[s] == 2) ? 5 : ncart(b->shell_l[s])));
    }
    pl->n_bf = nbf;
    pl->n_user = nuser;

    // normalised coefficients and per-AO angular factors
    std::vector<double> coef(b->n_prims);
    for (int s = 0; s < ns; ++s)
        normalise(b->shell_l[s], b->shell_nprim[s], b->exps + b->shell_prim_off[s], b->coefs + b->shell_prim_off[s],
                  coef.data() + b->shell_prim_off[s]);
    std::vector<double> ang(nbf, 1.0);
    for (int s = 0; s < ns; ++s)
        for (int k = 0; k < ncart(b->shell_l[s]); ++k) {
            const int *t = kCart.v[b->shell_l[s]][k];
            ang[pl->shell_ao[s] + k] = ang_factor(t[0], t[1], t[2]);
        }

    // canonical pairs (first shell has the higher l; equal l: higher index first)
    struct PairRec { int sa, sb, cls, K; long long user; };
    std::vector<PairRec> pr;
    pr.reserve((size_t)ns * (ns + 1) / 2);
    for (int x = 0; x < ns; ++x)
        for (int y = 0; y <= x; ++y) {
            int sa = x, sb = y;
            if (b->shell_l[sb] > b->shell_l[sa]) std::swap(sa, sb);
            pr.push_back({sa, sb, pair_class(b->shell_l[sa], b->shell_l[sb]), b->shell_nprim[sa] * b->shell_nprim[sb],
                          (long long)x * (x + 1) / 2 + y});
        }
    const int np = (int)pr.size();
    // primitive pairs in the unsorted order first (for the Schwarz pass)
    auto build_pp = [&](const std::vector<PairRec> &v, std::vector<int> &off, std::vector<int> &cnt,
                        std::vector<double> *pp) {
        off.resize(v.size());
        cnt.resize(v.size());
        for (int k = 0; k < 8; ++k) pp[k].clear();
        for (size_t i = 0; i < v.size(); ++i) {
            const int sa = v[i].sa, sb = v[i].sb;
            const double *A = b->coords + 3 * b->shell_atom[sa], *B = b->coords + 3 * b->shell_atom[sb];
            const double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
            off[i] = (int)pp[0].size();
            for (int ka = 0; ka < b->shell_nprim[sa]; ++ka)
                for (int kb = 0; kb < b->shell_nprim[sb]; ++kb) {
                    const double za = b->exps[b->shell_prim_off[sa] + ka], zb = b->exps[b->shell_prim_off[sb] + kb];
                    const double p = za + zb;
                    const double c = coef[b->shell_prim_off[sa] + ka] * coef[b->shell_prim_off[sb] + kb] *
                                     std::exp(-za * zb / p * ab2);
                    pp[0].push_back(p);
                    for (int d = 0; d < 3; ++d) pp[1 + d].push_back((za * A[d] + zb * B[d]) / p);
                    pp[4].push_back(c);
                    pp[5].push_back(za);
                    pp[6].push_back(zb);
                    pp[7].push_back(1.0 / p);
                }
            cnt[i] = (int)pp[0].size() - off[i];
        }
    };
    std::vector<int> off, cnt;
    std::vector<double> pp[8];
    build_pp(pr, off, cnt, pp);
    if (pp[0].size() > (size_t)0x7fffffff) return fail(TDG_EUNSUPPORTED, "too many primitive pairs");
    for (const auto &v : pp)
        if (v.size() != pp[0].size()) return fail(TDG_EINVAL, "internal: primitive-pair tables of unequal length");

    int rc;
    std::vector<int> sa(np), sb(np);
    for (int i = 0; i < np; ++i) { sa[i] = pr[i].sa; sb[i] = pr[i].sb; }
    std::vector<double> coords(b->coords, b->coords + 3 * b->n_atoms);
    if ((rc = pl->d_coords.upload(coords)) || (rc = pl->d_shell_atom.upload(pl->shell_atom)) ||
        (rc = pl->d_shell_ao.upload(pl->shell_ao)) || (rc = pl->d_shell_l.upload(pl->shell_l)) ||
        (rc = pl->d_pair_sa.upload(sa)) || (rc = pl->d_pair_sb.upload(sb)) || (rc = pl->d_pair_ppoff.upload(off)) ||
        (rc = pl->d_pair_npp.upload(cnt)) || (rc = pl->d_pp_p.upload(pp[0])) || (rc = pl->d_pp_Px.upload(pp[1])) ||
        (rc = pl->d_pp_Py.upload(pp[2])) || (rc = pl->d_pp_Pz.upload(pp[3])) || (rc = pl->d_pp_c.upload(pp[4])) ||
        (rc = pl->d_ang.upload(ang)))
        return rc;
    if (pl->sph) {
        std::vector<int> ao_shell(nuser, 0);
        for (int s = 0; s < ns; ++s)
            for (int k = 0; k < (b->shell_l[s] == 2 ? 5 : ncart(b->shell_l[s])); ++k) ao_shell[b->shell_ao_off[s] + k] = s;
        if ((rc = pl->d_shell_ao_user.upload(pl->shell_ao_user)) || (rc = pl->d_ao_shell_user.upload(ao_shell)))
            return rc;
    }

    // Schwarz per pair class: pairs grouped by class for the templated kernel
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pr[x].cls < pr[y].cls; });
    {
        std::vector<PairRec> pr2(np);
        for (int i = 0; i < np; ++i) pr2[i] = pr[order[i]];
        pr.swap(pr2);
        for (int i = 0; i < np; ++i) { sa[i] = pr[i].sa; sb[i] = pr[i].sb; }
        build_pp(pr, off, cnt, pp);
        if ((rc = pl->d_pair_sa.upload(sa)) || (rc = pl->d_pair_sb.upload(sb)) || (rc = pl->d_pair_ppoff.upload(off)) ||
            (rc = pl->d_pair_npp.upload(cnt)) || (rc = pl->d_pp_p.upload(pp[0])) || (rc = pl->d_pp_Px.upload(pp[1])) ||
            (rc = pl->d_pp_Py.upload(pp[2])) || (rc = pl->d_pp_Pz.upload(pp[3])) || (rc = pl->d_pp_c.upload(pp[4])))
            return rc;
    }
    int cs[7] = {0};
    for (int i = 0; i < np; ++i) cs[pr[i].cls + 1]++;
    for (int k = 0; k < 6; ++k) cs[k + 1] += cs[k];
    // angular factors of (mu nu|mu nu): (n_mu n_nu)^2 per pair class
    std::vector<double> angab(6 * 36, 1.0);
    for (int c = 0; c < 6; ++c) {
        const int la = kPairL[c][0], lb = kPairL[c][1];
        for (int ia = 0; ia < ncart(la); ++ia)
            for (int ib = 0; ib < ncart(lb); ++ib) {
                const int *ta = kCart.v[la][ia], *tb = kCart.v[lb][ib];
                const double f = ang_factor(ta[0], ta[1], ta[2]) * ang_factor(tb[0], tb[1], tb[2]);
                angab[c * 36 + ia * ncart(lb) + ib] = f * f;
            }
    }
    DevBuf<double> d_angab, d_Q;
    if ((rc = d_angab.upload(angab)) || (rc = d_Q.alloc(np))) return rc;
    for (int c = 0; c < 6; ++c) {
        const int n = cs[c + 1] - cs[c];
        if (!n) continue;
        const double *ang_c = d_angab.p + c * 36;
        switch (c) {
        case 0: launch_schwarz<0, 0>(pl, cs[c], n, ang_c, d_Q.p); break;
        case 1: launch_schwarz<1, 0>(pl, cs[c], n, ang_c, d_Q.p); break;
        case 2: launch_schwarz<1, 1>(pl, cs[c], n, ang_c, d_Q.p); break;
        case 3: launch_schwarz<2, 0>(pl, cs[c], n, ang_c, d_Q.p); break;
        case 4: launch_schwarz<2, 1>(pl, cs[c], n, ang_c, d_Q.p); break;
        default: launch_schwarz<2, 2>(pl, cs[c], n, ang_c, d_Q.p); break;
        }
    }
    HIP_TRY(hipGetLastError());
    std::vector<double> Q(np);
    HIP_TRY(hipMemcpy(Q.data(), d_Q.p, sizeof(double) * np, hipMemcpyDeviceToHost));
    d_Q.release();
    d_angab.release();

    // final order: class, contraction degree (descending), Q (descending)
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (pr[x].cls != pr[y].cls) return pr[x].cls < pr[y].cls;
        if (pr[x].K != pr[y].K) return pr[x].K > pr[y].K;
        return Q[x] > Q[y];
    });
    std::vector<PairRec> ps(np);
    pl->pair_Q.resize(np);
    pl->pair_K.resize(np);
    pl->user_pair_to_sorted.assign(np, -1);
    for (int i = 0; i < np; ++i) {
        ps[i] = pr[order[i]];
        pl->pair_Q[i] = Q[order[i]];
        pl->pair_K[i] = ps[i].K;
        pl->user_pair_to_sorted[ps[i].user] = i;
    }
    pl->npair = np;
    pl->pair_sa.resize(np);
    pl->pair_sb.resize(np);
    for (int i = 0; i < np; ++i) { pl->pair_sa[i] = ps[i].sa; pl->pair_sb[i] = ps[i].sb; }
    for (int k = 0; k < 7; ++k) pl->pc_start[k] = cs[k];
    pl->grp_start.clear();
    pl->pc_grp_start.assign(7, 0);
    for (int c = 0; c < 6; ++c) {
        pl->pc_grp_start[c] = (int)pl->grp_start.size();
        for (int i = cs[c]; i < cs[c + 1]; ++i)
            if (i == cs[c] || ps[i].K != ps[i - 1].K) pl->grp_start.push_back(i);
    }
    pl->pc_grp_start[6] = (int)pl->grp_start.size();
    pl->grp_start.push_back(np);
    // fused screening regions: one per (class, contraction group of the bra pair class, list)
    pl->pair_grp.assign(np, 0);
    for (int c = 0; c < 6; ++c)
        for (int g = pl->pc_grp_start[c]; g < pl->pc_grp_start[c + 1]; ++g)
            for (int i = pl->grp_start[g]; i < pl->grp_start[g + 1]; ++i) pl->pair_grp[i] = g - pl->pc_grp_start[c];
    pl->fgrp_off.assign(kNumClasses + 1, 0);
    for (int c = 0; c < kNumClasses; ++c) {
        int pb, pk;
        class_pk(c, pb, pk);
        pl->fgrp_off[c + 1] = pl->fgrp_off[c] + (pl->pc_grp_start[pb + 1] - pl->pc_grp_start[pb]);
    }
    build_pp(ps, off, cnt, pp);
    pl->pair_pmax.assign(np, 0.0);
    pl->pair_pmin.assign(np, 1e300);
    pl->pair_famp.assign(np, 0.0);
    for (int i = 0; i < np; ++i) {
        // FP32 routing proxy: a centre derivative scales an integral by about sqrt(zeta)
        for (int k = off[i]; k < off[i] + cnt[i]; ++k) {
            pl->pair_pmax[i] = std::max(pl->pair_pmax[i], pp[0][k]);
            pl->pair_pmin[i] = std::min(pl->pair_pmin[i], pp[0][k]);
            const double f = std::sqrt(std::max(pp[5][k], pp[6][k]));
            pl->pair_famp[i] = std::max(pl->pair_famp[i], f);
        }
    }
    if ((rc = pl->d_pair_pmax.upload(pl->pair_pmax)) || (rc = pl->d_pair_famp.upload(pl->pair_famp)) ||
        (rc = pl->d_pair_pmin.upload(pl->pair_pmin)))
        return rc;
    if ((rc = pl->d_pair_sa.upload(pl->pair_sa)) || (rc = pl->d_pair_sb.upload(pl->pair_sb)) ||
        (rc = pl->d_pair_ppoff.upload(off)) || (rc = pl->d_pair_npp.upload(cnt)) || (rc = pl->d_pair_K.upload(pl->pair_K)) ||
        (rc = pl->d_pair_Q.upload(pl->pair_Q)) || (rc = pl->d_grp_start.upload(pl->grp_start)) ||
        (rc = pl->d_pp_p.upload(pp[0])) || (rc = pl->d_pp_Px.upload(pp[1])) || (rc = pl->d_pp_Py.upload(pp[2])) ||
        (rc = pl->d_pp_Pz.upload(pp[3])) || (rc = pl->d_pp_c.upload(pp[4])))
        return rc;
    {
        // record layout read by the team kernels: p, 1/p, c, za, zb, Px, Py, Pz
        const size_t npp = pp[0].size();
        std::vector<double> rec(8 * npp);
        for (size_t k = 0; k < npp; ++k) {
            double *r = &rec[8 * k];
            r[0] = pp[0][k]; r[1] = pp[7][k]; r[2] = pp[4][k]; r[3] = pp[5][k];
            r[4] = pp[6][k]; r[5] = pp[1][k]; r[6] = pp[2][k]; r[7] = pp[3][k];
        }
        if ((rc = pl->d_pp_rec.upload(rec))) return rc;
    }
    // screening items: (class, bra pair), one wavefront each, indexed in int
    {
        long long items = 0;
        for (int c = 0; c < kNumClasses; ++c) {
            int pb, pk;
            class_pk(c, pb, pk);
            items += cs[pb + 1] - cs[pb];
        }
        if (items >= INT32_MAX) return fail(TDG_EUNSUPPORTED, "%lld screening items (class, bra pair) exceed 2^31", items);
    }
    pl->item_class_off.assign(kNumClasses + 1, 0);
    for (int c = 0; c < kNumClasses; ++c) {
        int pb, pk;
        class_pk(c, pb, pk);
        pl->item_class_off[c + 1] = pl->item_class_off[c] + (cs[pb + 1] - cs[pb]);
    }
    const int nitems = pl->item_class_off[kNumClasses];
    if ((rc = pl->d_item_cnt.alloc(std::max(nitems, 1))) || (rc = pl->d_item_off.alloc(std::max(nitems, 1))) ||
        (rc = pl->d_item_cnt32.alloc(std::max(nitems, 1))) || (rc = pl->d_item_off32.alloc(std::max(nitems, 1))) ||
        (rc = pl->d_prim_cnt.alloc(kNumClasses)) || (rc = pl->d_cand_cnt.alloc(kNumClasses)) || (rc = pl->d_mx.alloc(1)) ||
        (rc = pl->d_grad.alloc((size_t)3 * pl->n_atoms)) || (rc = pl->d_dens.alloc((size_t)3 * nbf * nbf)) ||
        (rc = pl->d_bmax.alloc((size_t)ns * ns)))
        return rc;
    HIP_TRY(hipEventCreate(&pl->ev0));
    HIP_TRY(hipEventCreate(&pl->ev1));
    for (auto &e : pl->ev_cls) HIP_TRY(hipEventCreate(&e));
    pl->nstreams = pl->prm.streams > 0 ? std::min(pl->prm.streams, tdg_plan::kMaxAux + 1) : tdg_plan::kMaxAux + 1;
    if (pl->nstreams > 1) {
        HIP_TRY(hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming));
        for (int k = 0; k + 1 < pl->nstreams; ++k) {
            // default priority (streams of other priorities are not used anywhere)
            HIP_TRY(hipStreamCreateWithFlags(&pl->aux[k], hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&pl->ev_join[k], hipEventDisableTiming));
        }
    }
    const bool lr = (pl->prm.terms & 4) && pl->prm.beta != 0.0;
    for (int pr = 0; pr < 2; ++pr)
        for (int c = 0; c < kNumClasses; ++c) {
            // the transfer form moves momentum A->B and C->D; with p or d functions on B or
            // D those steps cancel for tight exponents, so it is offered only when
            // l_B = l_D = 0 (and its kernel needs no scratch memory)
            int pb, pk;
            class_pk(c, pb, pk);
            const bool no_transfer = kPairL[pb][1] == 0 && kPairL[pk][1] == 0;
            pl->tf_ok[pr][0][c] = no_transfer && kScratch[c](0, pr, lr) == 0;
            pl->tf_ok[pr][1][c] = no_transfer && class_ncomp(c) <= 27 && kScratch[c](3, pr, lr) == 0;
            int v = pl->prm.kernel_variant >= 0 ? pl->prm.kernel_variant : default_variant(c);
            if ((v == 3 || v == 4) && class_ncomp(c) > 27) v = v == 3 ? 0 : 2;
            if (v == 0 && !pl->tf_ok[pr][0][c]) v = 2;
            if (v == 3 && !pl->tf_ok[pr][1][c]) v = 4;
            pl->variant[pr][c] = pl->bvariant[pr][c] = v;
        }
    for (int c = 0; c < kNumClasses; ++c) pl->split[c] = pl->bsplit[c] = 1;
    for (int pr = 0; pr < 2; ++pr)
        for (int c = 0; c < kNumClasses; ++c) pl->gpc[pr][c] = pl->bgpc[pr][c] = kGridPerCU;
    HIP_TRY(hipDeviceSynchronize());
    return TDG_OK;
}

static int check_basis(const tdg_basis_t *b)
{
    if (!b || !b->coords || !b->shell_atom || !b->shell_l || !b->shell_nprim || !b->shell_prim_off ||
        !b->shell_ao_off || !b->exps || !b->coefs)
        return fail(TDG_EINVAL, "null pointer in basis");
    if (b->n_atoms <= 0 || b->n_shells <= 0 || b->n_prims <= 0) return fail(TDG_EINVAL, "empty basis");
    if (b->spherical != 0 && b->spherical != 1) return fail(TDG_EINVAL, "spherical must be 0 or 1");
    for (int s = 0; s < b->n_shells; ++s) {
        if (b->shell_l[s] < 0 || b->shell_l[s] > 2) return fail(TDG_EUNSUPPORTED, "shell %d has l=%d (max 2)", s, b->shell_l[s]);
        if (b->shell_nprim[s] < 1 || b->shell_nprim[s] > TDG_MAX_NPRIM)
            return fail(TDG_EUNSUPPORTED, "shell %d has %d primitives (1..%d)", s, b->shell_nprim[s], TDG_MAX_NPRIM);
        if (b->shell_atom[s] < 0 || b->shell_atom[s] >= b->n_atoms) return fail(TDG_EINVAL, "shell %d atom index out of range", s);
        if (b->shell_prim_off[s] < 0 || b->shell_prim_off[s] + b->shell_nprim[s] > b->n_prims)
            return fail(TDG_EINVAL, "shell %d primitive range out of bounds", s);
        if (b->shell_ao_off[s] < 0) return fail(TDG_EINVAL, "shell %d negative AO offset", s);
        for (int k = 0; k < b->shell_nprim[s]; ++k)
            if (!(b->exps[b->shell_prim_off[s] + k] > 0.0)) return fail(TDG_EINVAL, "shell %d non-positive exponent", s);
    }
    return TDG_OK;
}

// ======================================================================= C ABI
extern "C" {

const char *tdg_last_error(void) { return g_err.c_str(); }

int tdg_plan_create(const tdg_basis_t *basis, const tdg_params_t *params, int device, tdg_plan_t **out)
{
    g_err.clear();
    if (!out || !params) return fail(TDG_EINVAL, "null argument");
    *out = nullptr;
    int rc = check_basis(basis);
    if (rc) return rc;
    if (params->precision != 0 && params->precision != 1)
        return fail(TDG_EUNSUPPORTED, "precision mode %d not available", params->precision);
    if ((params->terms & 4) && !(params->omega > 0.0)) return fail(TDG_EINVAL, "long-range term needs omega > 0");
    if (params->kernel_variant < -1 || params->kernel_variant > 4)
        return fail(TDG_EINVAL, "kernel_variant must be -1 or 0..4");
    if (params->screening != 0 && params->screening != 1)
        return fail(TDG_EINVAL, "screening must be 0 (Schwarz bound) or 1 (bound + learned veto)");
    if (params->deterministic != 0 && params->deterministic != 1)
        return fail(TDG_EINVAL, "deterministic must be 0 or 1");
    if (params->max_tasks < 0) return fail(TDG_EINVAL, "max_tasks must be >= 0");
    if (params->streams < 0) return fail(TDG_EINVAL, "streams must be >= 0");
    if (params->ml_min_components < 0) return fail(TDG_EINVAL, "ml_min_components must be >= 0");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(TDG_EINVAL, "device %d not present (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    tdg_plan *pl = new (std::nothrow) tdg_plan();
    if (!pl) return fail(TDG_ENOMEM, "host allocation failed");
    pl->device = device;
    pl->prm = *params;
    rc = build_plan(pl, basis);
    if (rc) {
        tdg_plan_destroy(pl);
        return rc;
    }
    *out = pl;
    return TDG_OK;
}

int tdg_plan_destroy(tdg_plan_t *pl)
{
    if (!pl) return TDG_OK;
    hipSetDevice(pl->device);
    DevBuf<double> *dbl[] = {&pl->d_coords, &pl->d_pair_Q, &pl->d_pp_p, &pl->d_pp_Px, &pl->d_pp_Py, &pl->d_pp_Pz,
                             &pl->d_pp_c, &pl->d_pp_rec, &pl->d_ang, &pl->d_in,
                             &pl->d_dens, &pl->d_grad};
    pl->d_bmax.release();
    for (auto *x : dbl) x->release();
    DevBuf<int> *ints[] = {&pl->d_shell_atom, &pl->d_shell_ao, &pl->d_shell_l, &pl->d_pair_sa, &pl->d_pair_sb,
                           &pl->d_pair_ppoff, &pl->d_pair_npp, &pl->d_pair_K, &pl->d_grp_start, &pl->d_item_cnt};
    for (auto *x : ints) x->release();
    pl->d_item_off.release();
    pl->d_prim_cnt.release();
    pl->d_cand_cnt.release();
    pl->d_grad_tune.release();
    pl->d_tune_tasks.release();
    pl->d_tune_mol.release();
    pl->d_pair_pmax.release();
    pl->d_pair_famp.release();
    pl->d_pair_pmin.release();
    pl->d_keep.release();
    pl->d_tasks2.release();
    pl->d_blkcnt.release();
    pl->d_segcnt.release();
    pl->d_item_cnt32.release();
    pl->d_item_off32.release();
    pl->d_ccnt.release();
    pl->d_fcap.release();
    pl->d_freg.release();
    pl->d_moves.release();
    pl->d_ftasks.release();
    pl->d_tout.release();
    pl->d_part.release();
    for (auto &e : pl->ev_cls)
        if (e) hipEventDestroy(e);
    for (auto &e : pl->ev_item)
        if (e) hipEventDestroy(e);
    for (int k = 0; k < tdg_plan::kMaxAux; ++k) {
        if (pl->aux[k]) hipStreamDestroy(pl->aux[k]);
        if (pl->ev_join[k]) hipEventDestroy(pl->ev_join[k]);
    }
    if (pl->ev_fork) hipEventDestroy(pl->ev_fork);
    pl->d_mx.release();
    pl->d_tasks.release();
    if (pl->ev0) hipEventDestroy(pl->ev0);
    if (pl->ev1) hipEventDestroy(pl->ev1);
    delete pl;
    return TDG_OK;
}

} // extern "C"
int tdg_plan_device_(const tdg_plan *pl) { return pl->device; }
extern "C" {

int tdg_plan_set_streams(tdg_plan_t *pl, int32_t streams)
{
    g_err.clear();
    if (!pl) return fail(TDG_EINVAL, "null plan");
    int avail = 1;
    while (avail <= tdg_plan::kMaxAux && pl->aux[avail - 1]) ++avail;
    if (streams < 1 || streams > avail)
        return fail(TDG_EINVAL, "streams must be 1..%d for this plan", avail);
    pl->nstreams = streams;
    return TDG_OK;
}

int tdg_plan_dims(const tdg_plan_t *pl, int32_t *n_bf, int32_t *n_atoms, int32_t *n_shells)
{
    if (!pl) return fail(TDG_EINVAL, "null plan");
    if (n_bf) *n_bf = pl->n_user;
    if (n_atoms) *n_atoms = pl->n_atoms;
    if (n_shells) *n_shells = pl->n_shells;
    return TDG_OK;
}

int tdg_plan_schwarz(const tdg_plan_t *pl, double *Q)
{
    if (!pl || !Q) return fail(TDG_EINVAL, "null argument");
    const long long ns = pl->n_shells;
    for (long long k = 0; k < ns * (ns + 1) / 2; ++k) Q[k] = pl->pair_Q[pl->user_pair_to_sorted[k]];
    return TDG_OK;
}

} // extern "C"

// --------------------------------------------------------------------------
// One or several molecules: per molecule the density preparation and the screening
// count pass; one host synchronisation for the task counts; the fill pass into one task list laid
// out per (class, precision) with the molecules concatenated; one launch per
// (class, precision) over all molecules (the class kernels).

// screening item of class c over its bras [skip, skip + nbra) (nbra < 0: all)
static void screen_add(tdg_plan *pl, ScreenTable &t, int c, int skip = 0, int nbra = -1)
{
    int pb, pk;
    class_pk(c, pb, pk);
    ScreenItem &it = t.it[t.n];
    it.cls = c; it.pb = pb; it.pk = pk;
    it.bra0 = pl->pc_start[pb] + skip;
    it.nbra = nbra >= 0 ? nbra : pl->pc_start[pb + 1] - pl->pc_start[pb] - skip;
    it.grp0 = pl->pc_grp_start[pk]; it.grp1 = pl->pc_grp_start[pk + 1];
    it.item_base = pl->item_class_off[c] + skip;
    it.bgrp0 = pl->pc_grp_start[pb]; it.bgrp1 = pl->pc_grp_start[pb + 1];
    it.fgrp_base = pl->fgrp_off.empty() ? 0 : pl->fgrp_off[c];
    if (it.nbra <= 0) return;
    t.wave_start[t.n + 1] = (int)std::min<long long>((long long)t.wave_start[t.n] + it.nbra, INT32_MAX);
    ++t.n;
}

template <int MODE>
static void screen_launch(const ScreenArgs &s, const ScreenTable &t, hipStream_t st)
{
    // screen_add keeps wave_start below 2^31 (one wavefront per (class, bra pair) item)
    if (t.n) hipLaunchKernelGGL(k_screen<MODE>, dim3((t.wave_start[t.n] + 3) / 4), dim3(256), 0, st, s, t);
}

static ScreenArgs screen_args(tdg_plan *pl)
{
    ScreenArgs s{};
    s.grp_start = pl->d_grp_start.p;
    s.pair_sa = pl->d_pair_sa.p; s.pair_sb = pl->d_pair_sb.p; s.pair_K = pl->d_pair_K.p;
    s.shell_atom = pl->d_shell_atom.p; s.pair_Q = pl->d_pair_Q.p;
    s.bmax = pl->d_bmax.p;
    s.n_shells = pl->n_shells; s.tau = pl->prm.schwarz_tol; s.mx = pl->d_mx.p;
    s.mixed = (pl->prm.precision == 1 && !pl->screen_fock) ? 1 : 0;
    s.keep_one_center = pl->screen_fock ? 1 : 0;
    s.tau_rel = pl->screen_fock == 2 ? 1 : 0;
    s.tau64 = pl->prm.mixed_tau64; s.p64 = pl->prm.mixed_p64;
    s.pair_pmax = pl->d_pair_pmax.p; s.pair_famp = pl->d_pair_famp.p;
    s.prim_cnt = pl->d_prim_cnt.p; s.cand_cnt = pl->d_cand_cnt.p;
    s.item_cnt = pl->d_item_cnt.p; s.item_off = pl->d_item_off.p;
    s.item_cnt32 = pl->d_item_cnt32.p; s.item_off32 = pl->d_item_off32.p;
    return s;
}

static bool class_active(tdg_plan *pl, int c)
{
    int pb, pk;
    class_pk(c, pb, pk);
    return pl->pc_start[pb + 1] > pl->pc_start[pb] && pl->pc_grp_start[pk + 1] > pl->pc_grp_start[pk];
}

// density preparation for one molecule (asynchronous): density records, block maxima, zeroed counters
static int prep_density(tdg_plan *pl, const double *P0, const double *PD, const double *R, int ptr_kind,
                          hipStream_t st)
{
    const int nbf = pl->n_bf, ns = pl->n_shells;
    const size_t nn = (size_t)pl->n_user * pl->n_user; // caller's matrices
    int rc;
    const double *dP0 = P0, *dPD = PD, *dR = R;
    if (ptr_kind == 0) {
        if ((rc = pl->d_in.alloc(3 * nn))) return rc;
        HIP_TRY(hipMemcpyAsync(pl->d_in.p, P0, nn * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(pl->d_in.p + nn, PD, nn * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(pl->d_in.p + 2 * nn, R, nn * 8, hipMemcpyHostToDevice, st));
        dP0 = pl->d_in.p;
        dPD = pl->d_in.p + nn;
        dR = pl->d_in.p + 2 * nn;
    }
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)pl->d_mx.p, 1);
    hipLaunchKernelGGL(k_zero, dim3((3 * pl->n_atoms + 255) / 256), dim3(256), 0, st, pl->d_grad.p,
                       (long long)3 * pl->n_atoms);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)pl->d_prim_cnt.p, (long long)kNumClasses);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)pl->d_cand_cnt.p, (long long)kNumClasses);
    const long long nblk = (long long)ns * ns;
    hipLaunchKernelGGL(k_density_prep, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, st, ns, nbf,
                       pl->d_shell_l.p, pl->d_shell_ao.p, pl->d_ang.p, dP0, dPD, dR, pl->d_dens.p, pl->d_bmax.p,
                       pl->d_mx.p, pl->sph, pl->n_user, pl->d_shell_ao_user.p);
    HIP_TRY(hipGetLastError());
    return TDG_OK;
}

// screening count pass for one molecule (asynchronous); counts copied to host buffers
static int count_pass(tdg_plan *pl, hipStream_t st)
{
    ScreenArgs s = screen_args(pl);
    ScreenTable t{};
    for (int c = 0; c < kNumClasses; ++c)
        if (class_active(pl, c)) screen_add(pl, t, c);
    screen_launch<0>(s, t, st);
    HIP_TRY(hipGetLastError());
    const int nitems = pl->item_class_off[kNumClasses];
    pl->h_cnt.assign(nitems, 0);
    pl->h_cnt32.assign(nitems, 0);
    pl->h_prim.assign(kNumClasses, 0);
    pl->h_cand.assign(kNumClasses, 0);
    if (nitems) HIP_TRY(hipMemcpyAsync(pl->h_cnt.data(), pl->d_item_cnt.p, sizeof(int) * nitems, hipMemcpyDeviceToHost, st));
    if (nitems && s.mixed)
        HIP_TRY(hipMemcpyAsync(pl->h_cnt32.data(), pl->d_item_cnt32.p, sizeof(int) * nitems, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(pl->h_prim.data(), pl->d_prim_cnt.p, 8 * kNumClasses, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(pl->h_cand.data(), pl->d_cand_cnt.p, 8 * kNumClasses, hipMemcpyDeviceToHost, st));
    return TDG_OK;
}

static FeatArgs feat_args(tdg_plan *pl)
{
    FeatArgs f{};
    f.pair_sa = pl->d_pair_sa.p; f.pair_sb = pl->d_pair_sb.p; f.shell_atom = pl->d_shell_atom.p;
    f.shell_l = pl->d_shell_l.p; f.pair_Q = pl->d_pair_Q.p; f.pair_pmin = pl->d_pair_pmin.p;
    f.pair_pmax = pl->d_pair_pmax.p; f.coords = pl->d_coords.p;
    f.bmax = pl->d_bmax.p; f.n_shells = pl->n_shells;
    return f;
}

// learned-screening veto on the screened task list of one molecule: each (class, precision) segment is
// filtered by the estimator and compacted (order kept) into the second task buffer;
// segment ends are updated (one host synchronisation)
static int ml_filter(tdg_plan *pl, int2 *&tasks, long long (*seg_begin)[2], long long (*seg_end)[2], hipStream_t st,
                     long long &skipped)
{
    const long long total = seg_end[kNumClasses - 1][1];
    int rc;
    if ((rc = pl->d_keep.alloc(std::max<long long>(total, 1))) || (rc = pl->d_tasks2.alloc(std::max<long long>(total, 1))) ||
        (rc = pl->d_segcnt.alloc(2 * kNumClasses)))
        return rc;
    const long long nbmax = (total + 1023) / 1024 + 2 * kNumClasses;
    if ((rc = pl->d_blkcnt.alloc(std::max<long long>(nbmax, 1)))) return rc;
    const float *w;
    const uint16_t *w1b, *w2b;
    mlp_device_ptrs(pl->ml, &w, &w1b, &w2b);
    const FeatArgs f = feat_args(pl);
    const float thr = (float)(pl->ml_log10 * 0.1);
    long long boff = 0;
    for (int c = 0; c < kNumClasses; ++c)
        for (int pr = 0; pr < 2; ++pr) {
            const long long b = seg_begin[c][pr], n = seg_end[c][pr] - b;
            if (!n) {
                hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)(pl->d_segcnt.p + 2 * c + pr), 1LL);
                continue;
            }
            if (class_ncomp(c) < pl->prm.ml_min_components) {
                // a class whose quartets cost less than the network: kept whole
                HIP_TRY(hipMemcpyAsync(pl->d_tasks2.p + b, tasks + b, sizeof(int2) * n, hipMemcpyDeviceToDevice, st));
                continue;
            }
            const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
            hipLaunchKernelGGL(k_ml_filter, dim3(grid), dim3(256), 0, st, tasks + b, n, f, w, w1b, w2b, thr,
                               pl->ml_tau_hi, pl->d_keep.p + b);
            const long long nb = (n + 1023) / 1024;
            hipLaunchKernelGGL(k_count_keep, dim3((unsigned)nb), dim3(1024), 0, st, pl->d_keep.p + b, n,
                               pl->d_blkcnt.p + boff);
            hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, pl->d_blkcnt.p + boff, nb,
                               pl->d_segcnt.p + 2 * c + pr);
            hipLaunchKernelGGL(k_scatter_keep, dim3((unsigned)nb), dim3(1024), 0, st, tasks + b, pl->d_keep.p + b, n,
                               pl->d_blkcnt.p + boff, pl->d_tasks2.p + b);
            boff += nb;
        }
    HIP_TRY(hipGetLastError());
    long long cnt[2 * kNumClasses];
    HIP_TRY(hipMemcpyAsync(cnt, pl->d_segcnt.p, sizeof cnt, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    skipped = 0;
    for (int c = 0; c < kNumClasses; ++c)
        for (int pr = 0; pr < 2; ++pr) {
            const long long n = seg_end[c][pr] - seg_begin[c][pr];
            const long long k = !n ? 0 : (class_ncomp(c) < pl->prm.ml_min_components ? n : cnt[2 * c + pr]);
            skipped += n - k;
            seg_end[c][pr] = seg_begin[c][pr] + k;
        }
    tasks = pl->d_tasks2.p;
    return TDG_OK;
}

static DerivArgs deriv_args(tdg_plan *pl)
{
    DerivArgs a{};
    a.coords = pl->d_coords.p; a.shell_atom = pl->d_shell_atom.p; a.shell_ao = pl->d_shell_ao.p;
    a.pair_sa = pl->d_pair_sa.p; a.pair_sb = pl->d_pair_sb.p; a.pair_ppoff = pl->d_pair_ppoff.p;
    a.pair_npp = pl->d_pair_npp.p;
    a.pp_rec = reinterpret_cast<const double2 *>(pl->d_pp_rec.p);
    a.dens = pl->d_dens.p; a.n_bf = pl->n_bf;
    a.omega = pl->prm.omega; a.alpha = pl->prm.alpha; a.beta = pl->prm.beta; a.terms = pl->prm.terms;
    a.grad = pl->d_grad.p; a.n_atoms = pl->n_atoms;
    a.lds_atoms = (3 * pl->n_atoms * 8 <= 24 * 1024) ? 1 : 0;
    return a;
}

// Screened tasks of one chunk: a contiguous range of screening items (single molecule)
// or every item of every molecule (batched), laid out per (class, precision) segment.
struct Chunk {
    long long seg_begin[kNumClasses][2], seg_end[kNumClasses][2];
    long long total = 0;
};

// screening of all classes in one launch (k_screen<2>) into regions sized from the previous call,
// then the used part of every region packed into one list per (class, list) in class order;
// ok = false when a region overflowed (the caller then runs the count and fill passes).
// The counts per region are left in pl->hcnt.
static int fused_screen(tdg_plan *pl, hipStream_t st, Chunk &ch, int2 *&tasks, bool &ok)
{
    const int nflat = 2 * pl->fgrp_off[kNumClasses];
    pl->freg.assign(nflat, 0);
    long long total = 0;
    for (int f = 0; f < nflat; ++f) {
        pl->freg[f] = total;
        total += pl->fcap[f];
    }
    int rc;
    if ((rc = pl->d_tasks.alloc(std::max<long long>(total, 1))) || (rc = pl->d_ccnt.alloc(std::max(nflat, 1))) ||
        (rc = pl->d_freg.upload(pl->freg)) || (rc = pl->d_fcap.upload(pl->fcap)))
        return rc;
    hipLaunchKernelGGL(k_zero, dim3((nflat + 255) / 256 + 1), dim3(256), 0, st, (double *)pl->d_ccnt.p, (long long)nflat);
    ScreenArgs s = screen_args(pl);
    s.tasks = pl->d_tasks.p;
    s.ccnt = pl->d_ccnt.p;
    s.freg = pl->d_freg.p;
    s.fcap = pl->d_fcap.p;
    ScreenTable t{};
    for (int c = 0; c < kNumClasses; ++c)
        if (class_active(pl, c)) screen_add(pl, t, c);
    screen_launch<2>(s, t, st);
    HIP_TRY(hipGetLastError());
    std::vector<unsigned long long> cnt(nflat);
    pl->h_prim.assign(kNumClasses, 0);
    pl->h_cand.assign(kNumClasses, 0);
    if (nflat) HIP_TRY(hipMemcpyAsync(cnt.data(), pl->d_ccnt.p, 8 * nflat, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(pl->h_prim.data(), pl->d_prim_cnt.p, 8 * kNumClasses, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(pl->h_cand.data(), pl->d_cand_cnt.p, 8 * kNumClasses, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    pl->hcnt.assign(nflat, 0);
    ok = true;
    for (int f = 0; f < nflat; ++f) {
        pl->hcnt[f] = (long long)cnt[f];
        ok &= pl->hcnt[f] <= pl->fcap[f];
    }
    if (!ok) return TDG_OK;
    // packed layout: class-major, FP64 list then FP32 list, bra groups in order
    std::vector<long long> moves;
    long long pos = 0;
    for (int c = 0; c < kNumClasses; ++c)
        for (int pr = 0; pr < 2; ++pr) {
            ch.seg_begin[c][pr] = pos;
            for (int g = pl->fgrp_off[c]; g < pl->fgrp_off[c + 1]; ++g) {
                const long long n = pl->hcnt[2 * g + pr];
                // one block per piece of at most kPackPiece tasks, so that large regions
                // are copied by many blocks
                for (long long k = 0; k < n; k += kPackPiece) {
                    moves.push_back(pl->freg[2 * g + pr] + k);
                    moves.push_back(pos + k);
                    moves.push_back(std::min(kPackPiece, n - k));
                }
                pos += n;
            }
            ch.seg_end[c][pr] = pos;
        }
    ch.total = pos;
    if ((rc = pl->d_ftasks.alloc(std::max<long long>(pos, 1))) || (rc = pl->d_moves.upload(moves))) return rc;
    const unsigned nmov = (unsigned)(moves.size() / 3);
    if (nmov) hipLaunchKernelGGL(k_pack_regions, dim3(nmov), dim3(256), 0, st, pl->d_tasks.p, pl->d_ftasks.p, pl->d_moves.p);
    HIP_TRY(hipGetLastError());
    tasks = pl->d_ftasks.p;
    return TDG_OK;
}

// region capacities for the next fused pass from this call's survivors per region
// (pl->hcnt, flat index 2 (fgrp_off[class] + group) + list)
static void learn_capacities(tdg_plan *pl)
{
    const long long limit = pl->prm.max_tasks > 0 ? pl->prm.max_tasks : (1LL << 31);
    const int nflat = 2 * pl->fgrp_off[kNumClasses];
    pl->fcap.assign(nflat, 0);
    long long total = 0;
    for (int f = 0; f < nflat; ++f) {
        const long long n = pl->hcnt[f];
        pl->fcap[f] = n + n / 4 + 64;
        total += pl->fcap[f];
    }
    pl->fused_ready = total <= limit;
}

// survivors per region from the count pass's per-bra counts (single molecule)
static void region_counts(tdg_plan *pl)
{
    const int nflat = 2 * pl->fgrp_off[kNumClasses];
    pl->hcnt.assign(nflat, 0);
    for (int c = 0; c < kNumClasses; ++c) {
        if (!class_active(pl, c)) continue;
        int pb, pk;
        class_pk(c, pb, pk);
        for (int k = pl->item_class_off[c]; k < pl->item_class_off[c + 1]; ++k) {
            const int bra = pl->pc_start[pb] + (k - pl->item_class_off[c]);
            const int f = 2 * (pl->fgrp_off[c] + pl->pair_grp[bra]);
            pl->hcnt[f] += pl->h_cnt[k];
            pl->hcnt[f + 1] += pl->h_cnt32[k];
        }
    }
}

// TDG_PROGRESS set in the environment: a line on stderr after every task-list chunk of a call
static bool progress_lines()
{
    static const bool on = std::getenv("TDG_PROGRESS") != nullptr;
    return on;
}

// timing events for n class-kernel items (created once, kept by the plan)
static int ensure_item_events(tdg_plan *pl, int n)
{
    while ((int)pl->ev_item.size() < n) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        pl->ev_item.push_back(e);
    }
    return TDG_OK;
}

// screened quartets of class c (both lists) from the count pass
static long long cls_count(const tdg_plan *pl, int c)
{
    long long n = 0;
    for (int k = pl->item_class_off[c]; k < pl->item_class_off[c + 1]; ++k)
        n += (long long)pl->h_cnt[k] + (pl->h_cnt32.empty() ? 0 : pl->h_cnt32[k]);
    return n;
}

// static_tasks (non-null): the allocation-free variant -- the task list of every chunk goes
// to static_tasks (at most static_cap tasks), and nothing that allocates device memory runs
// (no fused screening, no autotuning, no learned veto, no deterministic reduction)
static int run_molecules(int n, tdg_plan *const *pls, const double *const *P0, const double *const *PD,
                         const double *const *R, int ptr_kind, hipStream_t st, double *const *grad, tdg_stats_t *stats,
                         int2 *static_tasks = nullptr, long long static_cap = 0)
{
    const auto t_start = std::chrono::steady_clock::now();
    const bool noalloc = static_tasks != nullptr;
    tdg_plan *lead = pls[0];
    HIP_TRY(hipSetDevice(lead->device));
    int rc;
    const bool batched = n > 1;
    // deterministic mode (single molecule): tasks in count-pass order, default variants,
    // per-task values reduced in a fixed order (k_det_reduce, k_det_final)
    const bool det = !batched && lead->prm.deterministic;
    const bool use_ml = !batched && lead->prm.screening == 1;
    if (use_ml && !lead->ml) return fail(TDG_ESTATE, "screening = 1 needs an estimator (tdg_plan_set_screen_model)");
    // screening: one fused launch when the previous call sized the regions, else (and
    // after an overflow) the count pass, per-item offsets on the host and the fill pass
    bool fused = false;
    Chunk fch;
    int2 *ftasks = nullptr;
    for (int m = 0; m < n; ++m)
        if ((rc = prep_density(pls[m], P0[m], PD[m], R[m], ptr_kind, st))) return rc;
    if (!batched && !det && !noalloc && lead->fused_ready) {
        bool ok = false;
        if ((rc = fused_screen(lead, st, fch, ftasks, ok))) return rc;
        fused = ok;
        if (!ok) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)lead->d_prim_cnt.p, (long long)kNumClasses);
        if (!ok) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)lead->d_cand_cnt.p, (long long)kNumClasses);
    }
    if (!fused)
        for (int m = 0; m < n; ++m)
            if ((rc = count_pass(pls[m], st))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    // chunks of screening items (one molecule): at most max_tasks survivors each, so the
    // task list of a large system is never materialised whole
    std::vector<std::pair<int, int>> chunks;
    if (batched || fused) {
        chunks.push_back({0, 0});
    } else {
        long long cap = lead->prm.max_tasks > 0 ? lead->prm.max_tasks : (1LL << 31);
        if (det) cap = std::min(cap, kDetChunk);
        if (noalloc) cap = std::min(cap, static_cap);
        const int nitems = lead->item_class_off[kNumClasses];
        std::vector<char> act(kNumClasses);
        for (int c = 0; c < kNumClasses; ++c) act[c] = class_active(lead, c);
        int k0 = 0, c = 0;
        long long acc = 0;
        for (int k = 0; k < nitems; ++k) {
            while (k >= lead->item_class_off[c + 1]) ++c;
            const long long v = act[c] ? (long long)lead->h_cnt[k] + lead->h_cnt32[k] : 0;
            if (acc + v > cap && k > k0) {
                chunks.push_back({k0, k});
                k0 = k;
                acc = 0;
            }
            acc += v;
        }
        chunks.push_back({k0, nitems});
    }
    const bool lr = (lead->prm.terms & 4) && lead->prm.beta != 0.0;
    if (!lead->ncu) {
        hipDeviceProp_t prop;
        lead->ncu = hipGetDeviceProperties(&prop, lead->device) == hipSuccess ? prop.multiProcessorCount : 256;
    }
    const int ncu = lead->ncu;
    const int grid_max = ncu * kGridPerCU;
    int(*variant)[kNumClasses] = batched ? lead->bvariant : lead->variant;
    int(*gpc)[kNumClasses] = batched ? lead->bgpc : lead->gpc;
    int *split = batched ? lead->bsplit : lead->split;
    bool *tuned = batched ? lead->btuned : lead->tuned;
    long long tot_quartets = 0, tot_fp32 = 0, ml_skipped = 0;
    long long cls_q[kNumClasses] = {0}, cls_q32[kNumClasses] = {0};
    double cls_ms[kNumClasses] = {0.0}, kern_ms = 0.0;
    // class-kernel items: (molecule, class) with their FP64 and FP32 task ranges
    struct Item {
        int m, c;
        long long b[2], e[2];
        double cost;
    };
    std::vector<Item> items;
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        const int K0 = chunks[ci].first, K1 = chunks[ci].second;
        Chunk ch;
        int2 *tasks;
        // per molecule, the task ranges of each (class, list): [mb, me)
        std::vector<std::array<std::array<long long, 2>, kNumClasses>> mb(n), me(n);
        if (fused) {
            ch = fch;
            tasks = ftasks;
            for (int c = 0; c < kNumClasses; ++c)
                for (int pr = 0; pr < 2; ++pr) {
                    mb[0][c][pr] = ch.seg_begin[c][pr];
                    me[0][c][pr] = ch.seg_end[c][pr];
                }
        } else {
            // offsets of this chunk's items only: entry k - i0 of molecule m's vectors, with
            // [i0, i1) the chunk's items (all items of every molecule in a batch)
            std::vector<std::vector<long long>> offs(n), offs32(n);
            for (int m = 0; m < n; ++m) {
                const int i0 = batched ? 0 : K0, i1 = batched ? pls[m]->item_class_off[kNumClasses] : K1;
                offs[m].assign(std::max(i1 - i0, 1), 0);
                offs32[m].assign(std::max(i1 - i0, 1), 0);
            }
            long long total = 0;
            for (int c = 0; c < kNumClasses; ++c)
                for (int pr = 0; pr < 2; ++pr) {
                    ch.seg_begin[c][pr] = total;
                    for (int m = 0; m < n; ++m) {
                        tdg_plan *pl = pls[m];
                        const bool act = class_active(pl, c);
                        const int i0 = batched ? 0 : K0;
                        int lo = pl->item_class_off[c], hi = pl->item_class_off[c + 1];
                        if (!batched) { lo = std::max(lo, K0); hi = std::min(hi, K1); }
                        mb[m][c][pr] = total;
                        for (int k = lo; k < hi; ++k) {
                            if (pr == 0) offs[m][k - i0] = total; else offs32[m][k - i0] = total;
                            if (act) total += pr == 0 ? pl->h_cnt[k] : pl->h_cnt32[k];
                        }
                        me[m][c][pr] = total;
                    }
                    ch.seg_end[c][pr] = total;
                }
            ch.total = total;
            if (noalloc) {
                if (total > static_cap)
                    return fail(TDG_EUNSUPPORTED,
                                "%lld screened quartets of one bra pair exceed the static task buffer (%lld)", total,
                                static_cap);
                tasks = static_tasks;
            } else {
                if ((rc = lead->d_tasks.alloc(std::max<long long>(total, 1)))) return rc;
                tasks = lead->d_tasks.p;
            }
            for (int m = 0; m < n; ++m) {
                tdg_plan *pl = pls[m];
                const int i0 = batched ? 0 : K0, i1 = batched ? pl->item_class_off[kNumClasses] : K1;
                if (i1 > i0) {
                    HIP_TRY(hipMemcpyAsync(pl->d_item_off.p + i0, offs[m].data(), 8 * (i1 - i0),
                                           hipMemcpyHostToDevice, st));
                    if (pl->prm.precision == 1)
                        HIP_TRY(hipMemcpyAsync(pl->d_item_off32.p + i0, offs32[m].data(), 8 * (i1 - i0),
                                               hipMemcpyHostToDevice, st));
                }
                ScreenArgs s = screen_args(pl);
                s.tasks = tasks;
                ScreenTable t{};
                for (int c = 0; c < kNumClasses; ++c) {
                    if (!class_active(pl, c)) continue;
                    const int lo = std::max(pl->item_class_off[c], i0), hi = std::min(pl->item_class_off[c + 1], i1);
                    if (hi <= lo) continue;
                    screen_add(pl, t, c, lo - pl->item_class_off[c], hi - lo);
                }
                screen_launch<1>(s, t, st);
            }
            HIP_TRY(hipGetLastError());
            // the fill pass reads the offsets before the host vectors go out of scope
            HIP_TRY(hipStreamSynchronize(st));
        } // two-pass task generation
        if (use_ml) {
            long long sk = 0;
            if ((rc = ml_filter(lead, tasks, ch.seg_begin, ch.seg_end, st, sk))) return rc;
            ml_skipped += sk;
            for (int c = 0; c < kNumClasses; ++c)
                for (int pr = 0; pr < 2; ++pr) {
                    mb[0][c][pr] = ch.seg_begin[c][pr];
                    me[0][c][pr] = ch.seg_end[c][pr];
                }
        }
        // per-molecule kernel arguments
        std::vector<DerivArgs> margs(n);
        for (int m = 0; m < n; ++m) {
            margs[m] = deriv_args(pls[m]);
            if (det) margs[m].lds_atoms = 0;
        }
        bool need_tune = false;
        for (int c = 0; c < kNumClasses; ++c)
            need_tune |= !tuned[c] && ch.seg_end[c][1] > ch.seg_begin[c][0];
        if (lead->prm.autotune && lead->prm.kernel_variant < 0 && need_tune && !det && !noalloc) {
            // autotuner: time the kernel variants of each class on this call's task list (of a
            // batch: the molecule with the most tasks of the class), on a strided sample of at
            // most kTuneTasks tasks for a large class, into a scratch gradient, and keep the
            // fastest for later calls.  The wavefront design is a candidate for classes with
            // >= 27 components, the team designs for every class.  With the mixed route it also
            // decides the precision per class: the FP32-routed quartets run in FP32 only where
            // FP64 over the whole class measures slower.
            int tm_ = 0;
            DerivArgs at{};
            const int2 *tt = tasks;
            // fastest variant of precision pr over the task ranges [b0, e0) and [b1, e1) of tt (the
            // segments need not be adjacent)
            // time variant v of precision pr over the task ranges [b0, e0) and [b1, e1) of tt
            // (adjacent ranges run as one launch, as in the timed call): a warm-up round, then
            // the faster of two
            auto time_it = [&](int c, int pr, int v, int gmax, long long b0, long long e0, long long b1,
                               long long e1, float &ms) -> int {
                ms = 1e30f;
                const bool merge = e0 > b0 && e1 > b1 && e0 == b1;
                for (int rep = 0; rep < 3; ++rep) {
                    float t = 0.f;
                    HIP_TRY(hipEventRecord(lead->ev_cls[0], st));
                    for (int k = 0; k < (merge ? 1 : 2); ++k) {
                        const long long b = k ? b1 : b0, e = merge ? e1 : (k ? e1 : e0);
                        if (e <= b) continue;
                        at.tasks = tt + b;
                        at.ntasks = e - b;
                        HIP_TRY(kLaunch[c](v, pr, at, lr, st, gmax));
                    }
                    HIP_TRY(hipEventRecord(lead->ev_cls[1], st));
                    HIP_TRY(hipEventSynchronize(lead->ev_cls[1]));
                    HIP_TRY(hipEventElapsedTime(&t, lead->ev_cls[0], lead->ev_cls[1]));
                    if (rep) ms = std::min(ms, t);
                }
                return TDG_OK;
            };
            // fastest variant of precision pr over the ranges (the segments need not be adjacent)
            auto best_of = [&](int c, int pr, long long b0, long long e0, long long b1, long long e1, float &best,
                               int &bv) -> int {
                best = 0.f;
                bv = variant[pr][c];
                if (e0 <= b0 && e1 <= b1) return TDG_OK;
                best = 1e30f;
                for (int v = 0; v < kNumVariants; ++v) {
                    if (v == 1 && class_ncomp(c) < 27) continue;
                    if ((v == 3 || v == 4) && class_ncomp(c) > 27) continue;
                    if (v == 0 && !lead->tf_ok[pr][0][c]) continue;
                    if (v == 3 && !lead->tf_ok[pr][1][c]) continue;
                    float ms;
                    if ((rc = time_it(c, pr, v, grid_max, b0, e0, b1, e1, ms))) return rc;
                    if (ms < best) { best = ms; bv = v; }
                }
                return TDG_OK;
            };
            // launch shape of the chosen variant: blocks per compute unit (the blocks stride over
            // the tasks, so fewer blocks means more tasks per block)
            auto best_grid = [&](int c, int pr, int v, long long b0, long long e0, long long b1, long long e1,
                                 int &g) -> int {
                float best = 1e30f;
                g = kGridPerCU;
                if (e0 <= b0 && e1 <= b1) return TDG_OK;
                for (int cand : {4, 8, 16, 32}) {
                    float ms;
                    if ((rc = time_it(c, pr, v, ncu * cand, b0, e0, b1, e1, ms))) return rc;
                    if (ms < best) { best = ms; g = cand; }
                }
                return TDG_OK;
            };
            for (int c = 0; c < kNumClasses; ++c) {
                if (tuned[c] || ch.seg_end[c][1] <= ch.seg_begin[c][0]) continue;
                tuned[c] = true;
                // the molecule with the most tasks of the class
                tm_ = 0;
                long long most = -1;
                for (int m = 0; m < n; ++m) {
                    const long long k = (me[m][c][0] - mb[m][c][0]) + (me[m][c][1] - mb[m][c][1]);
                    if (k > most) { most = k; tm_ = m; }
                }
                tdg_plan *pm = pls[tm_];
                if ((rc = pm->d_grad_tune.alloc((size_t)3 * pm->n_atoms))) return rc;
                at = margs[tm_];
                at.grad = pm->d_grad_tune.p;
                at.task_out = nullptr;
                long long b0 = mb[tm_][c][0], e0 = me[tm_][c][0], b1 = mb[tm_][c][1], e1 = me[tm_][c][1];
                tt = tasks;
                const long long n0 = std::max(0LL, e0 - b0), n1 = std::max(0LL, e1 - b1);
                const long long stride = (n0 + n1 + kTuneTasks - 1) / kTuneTasks;
                if (stride > 1) {
                    // every stride-th task of each range, the two samples adjacent
                    const long long m0 = (n0 + stride - 1) / stride, m1 = (n1 + stride - 1) / stride;
                    if ((rc = lead->d_tune_tasks.alloc(m0 + m1))) return rc;
                    if (m0)
                        hipLaunchKernelGGL(k_sample_tasks, dim3((unsigned)((m0 + 255) / 256)), dim3(256), 0, st, tasks,
                                           nullptr, b0, stride, m0, lead->d_tune_tasks.p, nullptr);
                    if (m1)
                        hipLaunchKernelGGL(k_sample_tasks, dim3((unsigned)((m1 + 255) / 256)), dim3(256), 0, st, tasks,
                                           nullptr, b1, stride, m1, lead->d_tune_tasks.p + m0, nullptr);
                    HIP_TRY(hipGetLastError());
                    tt = lead->d_tune_tasks.p;
                    b0 = 0; e0 = m0; b1 = m0; e1 = m0 + m1;
                }
                float t_all = 0.f, t64 = 0.f, t32 = 0.f;
                int v_all = 0, v64 = 0, v32 = 0;
                if ((rc = best_of(c, 0, b0, e0, b1, e1, t_all, v_all))) return rc;
                if (e1 > b1) {
                    if ((rc = best_of(c, 0, b0, e0, 0, 0, t64, v64)) || (rc = best_of(c, 1, 0, 0, b1, e1, t32, v32)))
                        return rc;
                }
                if (e1 > b1 && t64 + t32 < 0.97f * t_all) { // FP32 only for a clear gain
                    split[c] = 1;
                    variant[0][c] = v64;
                    variant[1][c] = v32;
                    if ((rc = best_grid(c, 0, v64, b0, e0, 0, 0, gpc[0][c])) ||
                        (rc = best_grid(c, 1, v32, 0, 0, b1, e1, gpc[1][c])))
                        return rc;
                } else {
                    split[c] = e1 > b1 ? 0 : split[c];
                    variant[0][c] = v_all;
                    if ((rc = best_grid(c, 0, v_all, b0, e0, b1, e1, gpc[0][c]))) return rc;
                }
            }
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (det) {
            // every class writes its quartets' twelve values; zeroed first (the wavefront
            // kernels add their lanes' values)
            const long long nv = 12 * std::max<long long>(ch.seg_end[kNumClasses - 1][1], 1);
            if ((rc = lead->d_tout.alloc(nv))) return rc;
            hipLaunchKernelGGL(k_zero, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, lead->d_tout.p, nv);
        }
        // The class launches of all molecules are independent (each adds into its molecule's
        // gradient with atomics, or writes its own quartets' values), so they form one launch
        // graph spread over the plan's streams, which the GPU's hardware queues run side by
        // side: small classes and small molecules fill the compute units next to the large
        // ones instead of after them.  Largest expected work first (primitive quartets times
        // roots times components), each to the stream with the least expected work so far.
        items.clear();
        for (int m = 0; m < n; ++m)
            for (int c = 0; c < kNumClasses; ++c) {
                if (me[m][c][0] <= mb[m][c][0] && me[m][c][1] <= mb[m][c][1]) continue;
                int pb, pk;
                class_pk(c, pb, pk);
                const int L = kPairL[pb][0] + kPairL[pb][1] + kPairL[pk][0] + kPairL[pk][1];
                const long long nq = (me[m][c][0] - mb[m][c][0]) + (me[m][c][1] - mb[m][c][1]);
                const long long nall = chunks.size() == 1 ? nq : cls_count(pls[m], c);
                const double prim = nall > 0 ? (double)pls[m]->h_prim[c] * nq / nall : 0.0;
                Item it{m, c, {mb[m][c][0], mb[m][c][1]}, {me[m][c][0], me[m][c][1]},
                        prim * (L / 2 + 1) * (class_ncomp(c) + 30.0)};
                items.push_back(it);
            }
        std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
        if ((rc = ensure_item_events(lead, 2 * (int)items.size()))) return rc;
        HIP_TRY(hipEventRecord(lead->ev0, st));
        const int nst = lead->nstreams;
        if (nst > 1) {
            HIP_TRY(hipEventRecord(lead->ev_fork, st));
            for (int k = 0; k + 1 < nst; ++k) HIP_TRY(hipStreamWaitEvent(lead->aux[k], lead->ev_fork, 0));
        }
        double load[tdg_plan::kMaxAux + 1] = {0.0};
        for (size_t ii = 0; ii < items.size(); ++ii) {
            const Item &it = items[ii];
            const int c = it.c;
            int k = 0;
            for (int q = 1; q < nst; ++q)
                if (load[q] < load[k]) k = q;
            load[k] += it.cost;
            hipStream_t sc = k == 0 ? st : lead->aux[k - 1];
            DerivArgs a = margs[it.m];
            auto set_span = [&](long long b, long long e) {
                a.tasks = tasks + b;
                a.ntasks = e - b;
                a.task_out = det ? lead->d_tout.p + 12 * b : nullptr;
            };
            HIP_TRY(hipEventRecord(lead->ev_item[2 * ii], sc));
            // a class that is not split runs its FP32-routed range with the FP64 kernel: one
            // launch when the two ranges are adjacent, else one per range
            if (!split[c] && it.e[0] == it.b[1]) {
                set_span(it.b[0], it.e[1]);
                if (a.ntasks) HIP_TRY(kLaunch[c](variant[0][c], 0, a, lr, sc, ncu * gpc[0][c]));
            } else {
                for (int pr = 0; pr < 2; ++pr) {
                    set_span(it.b[pr], it.e[pr]);
                    if (a.ntasks <= 0) continue;
                    const int prec = split[c] ? pr : 0;
                    HIP_TRY(kLaunch[c](variant[prec][c], prec, a, lr, sc, ncu * gpc[prec][c]));
                }
            }
            HIP_TRY(hipEventRecord(lead->ev_item[2 * ii + 1], sc));
        }
        for (int k = 0; k + 1 < nst; ++k) {
            HIP_TRY(hipEventRecord(lead->ev_join[k], lead->aux[k]));
            HIP_TRY(hipStreamWaitEvent(st, lead->ev_join[k], 0));
        }
        if (det) {
            // per-atom sums in a fixed order, segment by segment (a learned veto leaves
            // unused entries between the compacted segments)
            const int n3 = 3 * lead->n_atoms;
            const int use_lds = (size_t)n3 * sizeof(double) <= 64 * 1024 ? 1 : 0;
            if ((rc = lead->d_part.alloc((size_t)kDetBlocks * n3))) return rc;
            for (int c = 0; c < kNumClasses; ++c)
                for (int pr = 0; pr < 2; ++pr) {
                    const long long b = ch.seg_begin[c][pr], nt = ch.seg_end[c][pr] - b;
                    if (nt <= 0) continue;
                    const long long per = std::max<long long>(256, (nt + kDetBlocks - 1) / kDetBlocks);
                    const int nblk = (int)((nt + per - 1) / per);
                    hipLaunchKernelGGL(k_det_reduce, dim3(nblk), dim3(kWave), use_lds ? (size_t)n3 * sizeof(double) : 0,
                                       st, tasks + b, nt, per, lead->d_tout.p + 12 * b, lead->d_pair_sa.p,
                                       lead->d_pair_sb.p, lead->d_shell_atom.p, lead->n_atoms, use_lds,
                                       lead->d_part.p);
                    hipLaunchKernelGGL(k_det_final, dim3((unsigned)((n3 + 3) / 4)), dim3(256), 0, st, lead->d_part.p,
                                       nblk, n3, lead->d_grad.p);
                }
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipEventRecord(lead->ev1, st));
        for (int c = 0; c < kNumClasses; ++c) {
            const long long n64 = ch.seg_end[c][0] - ch.seg_begin[c][0], n32 = ch.seg_end[c][1] - ch.seg_begin[c][1];
            cls_q[c] += n64 + n32;
            cls_q32[c] += split[c] ? n32 : 0;
            tot_quartets += n64 + n32;
            tot_fp32 += split[c] ? n32 : 0;
        }
        if (progress_lines()) {
            HIP_TRY(hipEventSynchronize(lead->ev1));
            fprintf(stderr, "tdgrad: chunk %zu of %zu done, %lld quartets so far, %.1f s\n", ci + 1, chunks.size(),
                    tot_quartets,
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
            fflush(stderr);
        }
        if (stats || chunks.size() > 1) {
            // per-chunk timing (the next chunk reuses the event objects)
            HIP_TRY(hipEventSynchronize(lead->ev1));
            for (size_t ii = 0; ii < items.size(); ++ii) {
                float cm = 0.f;
                HIP_TRY(hipEventElapsedTime(&cm, lead->ev_item[2 * ii], lead->ev_item[2 * ii + 1]));
                cls_ms[items[ii].c] += cm;
            }
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, lead->ev0, lead->ev1));
            kern_ms += ms;
        }
    }
    if (!batched && chunks.size() == 1) {
        if (!fused) region_counts(lead);
        learn_capacities(lead);
    }
    for (int m = 0; m < n; ++m) {
        tdg_plan *pl = pls[m];
        const size_t bytes = sizeof(double) * 3 * pl->n_atoms;
        HIP_TRY(hipMemcpyAsync(grad[m], pl->d_grad.p, bytes,
                               ptr_kind == 0 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    }
    if (ptr_kind == 0 || stats) HIP_TRY(hipStreamSynchronize(st));
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        for (int c = 0; c < kNumClasses; ++c) {
            stats->class_quartets[c] = cls_q[c];
            stats->class_fp32_quartets[c] = cls_q32[c];
            for (int m = 0; m < n; ++m) {
                stats->class_prim_quartets[c] += (long long)pls[m]->h_prim[c];
                stats->prim_quartets += (long long)pls[m]->h_prim[c];
                stats->candidates += (long long)pls[m]->h_cand[c];
            }
            stats->class_ms[c] = cls_ms[c];
            stats->class_variant[c] = variant[0][c] | (variant[1][c] << 3) | (split[c] ? 0 : 64) |
                                      (gpc[0][c] << 8) | (gpc[1][c] << 16);
        }
        stats->quartets = tot_quartets;
        stats->fp32_quartets = tot_fp32;
        stats->ml_skipped = ml_skipped;
        stats->chunks = (int64_t)chunks.size();
        stats->ms_kernels = kern_ms;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return TDG_OK;
}

extern "C" {

int tdg_grad_jk(tdg_plan_t *pl, const double *P0, const double *PD, const double *R, int32_t ptr_kind,
                void *hip_stream, double *grad, tdg_stats_t *stats)
{
    g_err.clear();
    if (!pl) return fail(TDG_EINVAL, "null plan");
    if (!P0 || !PD || !R || !grad) return fail(TDG_EINVAL, "null density or output pointer");
    if (ptr_kind != 0 && ptr_kind != 1) return fail(TDG_EINVAL, "ptr_kind must be 0 or 1");
    return run_molecules(1, &pl, &P0, &PD, &R, ptr_kind, (hipStream_t)hip_stream, &grad, stats);
}

} // extern "C"

// Task list of the allocation-free entry point: one per GPU, in a file-scope device array
// (its host-side name is not a device address: host code uses the address that
// hipGetSymbolAddress returns for the current device).  Fully written by the fill pass of
// every chunk before the class kernels read it, so nothing needs clearing between calls.
constexpr long long kStaticTasks = 1LL << 23; // 8,388,608 tasks, 64 MiB
static __device__ __align__(256) int2 scratch[kStaticTasks];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static int2 *g_scratch_ptr[kMaxDevices] = {};

extern "C" {

int tdg_grad_jk_noalloc(tdg_plan_t *pl, const double *P0, const double *PD, const double *R, void *hip_stream,
                        double *grad, tdg_stats_t *stats)
{
    g_err.clear();
    if (!pl) return fail(TDG_EINVAL, "null plan");
    if (!P0 || !PD || !R || !grad) return fail(TDG_EINVAL, "null density or output pointer");
    if (pl->prm.deterministic) return fail(TDG_EUNSUPPORTED, "the allocation-free call has no deterministic mode");
    if (pl->prm.screening != 0) return fail(TDG_EUNSUPPORTED, "the allocation-free call has no learned veto");
    if (pl->device < 0 || pl->device >= kMaxDevices) return fail(TDG_EUNSUPPORTED, "device index %d", pl->device);
    HIP_TRY(hipSetDevice(pl->device));
    int2 *tasks = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[pl->device]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(TDG_EDEVICE, "hipGetSymbolAddress of the static task buffer failed: %s",
                            hipGetErrorString(e));
            g_scratch_ptr[pl->device] = static_cast<int2 *>(p);
        }
        tasks = g_scratch_ptr[pl->device];
    }
    return run_molecules(1, &pl, &P0, &PD, &R, 1, (hipStream_t)hip_stream, &grad, stats, tasks, kStaticTasks);
}

int tdg_grad_jk_batch(int32_t n, tdg_plan_t *const *plans, const double *const *P0, const double *const *PD,
                      const double *const *R, int32_t ptr_kind, void *hip_stream, double *const *grad,
                      tdg_stats_t *stats)
{
    g_err.clear();
    if (n <= 0 || !plans || !P0 || !PD || !R || !grad) return fail(TDG_EINVAL, "bad batch arguments");
    if (ptr_kind != 0 && ptr_kind != 1) return fail(TDG_EINVAL, "ptr_kind must be 0 or 1");
    for (int m = 0; m < n; ++m) {
        if (!plans[m] || !P0[m] || !PD[m] || !R[m] || !grad[m]) return fail(TDG_EINVAL, "null entry %d in batch", m);
        const tdg_params_t &x = plans[m]->prm, &y = plans[0]->prm;
        if (plans[m]->device != plans[0]->device || x.omega != y.omega || x.alpha != y.alpha || x.beta != y.beta ||
            x.terms != y.terms || x.precision != y.precision)
            return fail(TDG_EINVAL, "plan %d differs from plan 0 in device or method parameters", m);
        for (int k = 0; k < m; ++k)
            if (plans[k] == plans[m]) return fail(TDG_EINVAL, "plan %d appears twice in the batch", m);
        if (x.deterministic != y.deterministic)
            return fail(TDG_EINVAL, "plan %d differs from plan 0 in the deterministic mode", m);
    }
    if (plans[0]->prm.deterministic) {
        // one molecule after another (the fixed-order reduction is per molecule)
        tdg_stats_t acc{}, one{};
        for (int m = 0; m < n; ++m) {
            const int rc = run_molecules(1, plans + m, P0 + m, PD + m, R + m, ptr_kind, (hipStream_t)hip_stream,
                                         grad + m, stats ? &one : nullptr);
            if (rc) return rc;
            if (stats) {
                acc.quartets += one.quartets; acc.prim_quartets += one.prim_quartets;
                acc.candidates += one.candidates; acc.fp32_quartets += one.fp32_quartets;
                acc.chunks += one.chunks; acc.ms_total += one.ms_total; acc.ms_kernels += one.ms_kernels;
                for (int c = 0; c < kNumClasses; ++c) {
                    acc.class_quartets[c] += one.class_quartets[c];
                    acc.class_prim_quartets[c] += one.class_prim_quartets[c];
                    acc.class_fp32_quartets[c] += one.class_fp32_quartets[c];
                    acc.class_ms[c] += one.class_ms[c];
                    acc.class_variant[c] = one.class_variant[c];
                }
            }
        }
        if (stats) *stats = acc;
        return TDG_OK;
    }
    return run_molecules(n, plans, P0, PD, R, ptr_kind, (hipStream_t)hip_stream, grad, stats);
}

int tdg_plan_set_screen_model(tdg_plan_t *pl, const tdg_mlp_t *model, double log10_threshold, double tau_hi)
{
    g_err.clear();
    if (!pl) return fail(TDG_EINVAL, "null plan");
    pl->ml = model;
    pl->ml_log10 = log10_threshold;
    pl->ml_tau_hi = tau_hi;
    return TDG_OK;
}

int tdg_collect(tdg_plan_t *pl, const double *P0, const double *PD, const double *R, int32_t ptr_kind,
                void *hip_stream, float *feat, float *target, int64_t cap, int64_t stride, int64_t *n_out)
{
    g_err.clear();
    if (!pl || !P0 || !PD || !R || !feat || !target || !n_out || cap < 0 || stride < 1)
        return fail(TDG_EINVAL, "bad arguments");
    if (pl->prm.precision != 0) return fail(TDG_EINVAL, "collection needs an FP64 plan");
    if (ptr_kind != 0 && ptr_kind != 1) return fail(TDG_EINVAL, "ptr_kind must be 0 or 1");
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(pl->device));
    int rc;
    if ((rc = prep_density(pl, P0, PD, R, ptr_kind, st)) || (rc = count_pass(pl, st))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<long long> offs(pl->item_class_off[kNumClasses]);
    long long seg_begin[kNumClasses], total = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        seg_begin[c] = total;
        const bool act = class_active(pl, c);
        for (int k = pl->item_class_off[c]; k < pl->item_class_off[c + 1]; ++k) {
            offs[k] = total;
            if (act) total += pl->h_cnt[k];
        }
    }
    if ((rc = pl->d_tasks.alloc(std::max<long long>(total, 1)))) return rc;
    if (!offs.empty())
        HIP_TRY(hipMemcpyAsync(pl->d_item_off.p, offs.data(), 8 * offs.size(), hipMemcpyHostToDevice, st));
    ScreenArgs s = screen_args(pl);
    s.tasks = pl->d_tasks.p;
    ScreenTable t{};
    for (int c = 0; c < kNumClasses; ++c)
        if (class_active(pl, c)) screen_add(pl, t, c);
    screen_launch<1>(s, t, st);
    DevBuf<double> contrib;
    if ((rc = contrib.alloc(std::max<long long>(12 * total, 1)))) return rc;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((12 * total + 255) / 256 + 1)), dim3(256), 0, st, contrib.p, 12 * total);
    const bool lr = (pl->prm.terms & 4) && pl->prm.beta != 0.0;
    DerivArgs a = deriv_args(pl);
    int ncu = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    for (int c = 0; c < kNumClasses; ++c) {
        const long long n = (c + 1 < kNumClasses ? seg_begin[c + 1] : total) - seg_begin[c];
        if (!n) continue;
        a.tasks = pl->d_tasks.p + seg_begin[c];
        a.ntasks = n;
        a.task_out = contrib.p + 12 * seg_begin[c];
        // the plan's FP64 variant of the class (allowed forms only; tuned if a call tuned it)
        HIP_TRY(kLaunch[c](pl->variant[0][c], 0, a, lr, st, ncu * kGridPerCU));
    }
    const long long ns = (total + stride - 1) / stride;
    const long long nout = std::min<long long>(ns, cap);
    if (nout > 0)
        hipLaunchKernelGGL(k_collect, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, pl->d_tasks.p, total,
                           (long long)stride, feat_args(pl), contrib.p, feat, target, (long long)cap, 0LL);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    contrib.release();
    *n_out = nout;
    return TDG_OK;
}

} // extern "C"

// ----------------------------------------------------------------------------------
// Verification entry points and geometry updates.

// fill pass for the screening items [K0, K1) of one molecule into pl->d_tasks (after a count
// pass): per class the FP64-routed list, then the FP32-routed list (mixed plans)
static int fill_items(tdg_plan *pl, hipStream_t st, int K0, int K1, Chunk &ch)
{
    int rc;
    // offsets of the items [K0, K1) only (a large system has tens of millions of items)
    std::vector<long long> offs(std::max(K1 - K0, 1), 0), offs32(std::max(K1 - K0, 1), 0);
    long long total = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        const bool act = class_active(pl, c);
        const int lo = std::max(pl->item_class_off[c], K0), hi = std::min(pl->item_class_off[c + 1], K1);
        for (int pr = 0; pr < 2; ++pr) {
            ch.seg_begin[c][pr] = total;
            for (int k = lo; k < hi; ++k) {
                (pr ? offs32 : offs)[k - K0] = total;
                if (act) total += pr ? pl->h_cnt32[k] : pl->h_cnt[k];
            }
            ch.seg_end[c][pr] = total;
        }
    }
    ch.total = total;
    if ((rc = pl->d_tasks.alloc(std::max<long long>(total, 1)))) return rc;
    if (K1 > K0) {
        HIP_TRY(hipMemcpyAsync(pl->d_item_off.p + K0, offs.data(), 8 * (K1 - K0), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(pl->d_item_off32.p + K0, offs32.data(), 8 * (K1 - K0), hipMemcpyHostToDevice, st));
    }
    ScreenArgs s = screen_args(pl);
    s.tasks = pl->d_tasks.p;
    ScreenTable t{};
    for (int c = 0; c < kNumClasses; ++c) {
        if (!class_active(pl, c)) continue;
        const int lo = std::max(pl->item_class_off[c], K0), hi = std::min(pl->item_class_off[c + 1], K1);
        if (hi > lo) screen_add(pl, t, c, lo - pl->item_class_off[c], hi - lo);
    }
    screen_launch<1>(s, t, st);
    HIP_TRY(hipGetLastError());
    // the offsets are read by the fill pass before the host vectors go out of scope
    HIP_TRY(hipStreamSynchronize(st));
    return TDG_OK;
}

extern "C" {

int tdg_plan_update_coords(tdg_plan_t *pl, const double *coords)
{
    g_err.clear();
    if (!pl || !coords) return fail(TDG_EINVAL, "null argument");
    for (int k = 0; k < 3 * pl->n_atoms; ++k)
        if (!std::isfinite(coords[k])) return fail(TDG_EINVAL, "coordinate %d is not finite", k);
    HIP_TRY(hipSetDevice(pl->device));
    tdg_basis_t b{};
    b.n_atoms = pl->n_atoms;
    b.coords = coords;
    b.n_shells = pl->n_shells;
    b.shell_atom = pl->shell_atom.data();
    b.shell_l = pl->shell_l.data();
    b.shell_nprim = pl->b_nprim.data();
    b.shell_prim_off = pl->b_primoff.data();
    b.shell_ao_off = pl->shell_ao_user.data();
    b.spherical = pl->sph;
    b.n_prims = pl->n_prims;
    b.exps = pl->b_exps.data();
    b.coefs = pl->b_coefs.data();
    tdg_plan *np = new (std::nothrow) tdg_plan();
    if (!np) return fail(TDG_ENOMEM, "host allocation failed");
    np->device = pl->device;
    np->prm = pl->prm;
    int rc = build_plan(np, &b);
    if (rc) {
        const std::string msg = g_err;
        tdg_plan_destroy(np);
        g_err = msg;
        return rc;
    }
    // state that does not depend on the geometry: tuned variants, precision split,
    // region capacities (the contraction groups are the same), estimator
    std::memcpy(np->variant, pl->variant, sizeof np->variant);
    std::memcpy(np->bvariant, pl->bvariant, sizeof np->bvariant);
    std::memcpy(np->split, pl->split, sizeof np->split);
    std::memcpy(np->gpc, pl->gpc, sizeof np->gpc);
    std::memcpy(np->bgpc, pl->bgpc, sizeof np->bgpc);
    std::memcpy(np->bsplit, pl->bsplit, sizeof np->bsplit);
    std::memcpy(np->tuned, pl->tuned, sizeof np->tuned);
    std::memcpy(np->btuned, pl->btuned, sizeof np->btuned);
    if (np->fgrp_off == pl->fgrp_off) {
        np->fcap = pl->fcap;
        np->fused_ready = pl->fused_ready;
    }
    np->ml = pl->ml;
    np->ml_log10 = pl->ml_log10;
    np->ml_tau_hi = pl->ml_tau_hi;
    np->ncu = pl->ncu;
    // the caller's handle keeps pointing at pl: move the new tables in, the old ones out
    tdg_plan old = std::move(*pl);
    *pl = std::move(*np);
    *np = std::move(old);
    tdg_plan_destroy(np);
    return TDG_OK;
}

int tdg_screen_list(tdg_plan_t *pl, const double *P0, const double *PD, const double *R, int32_t ptr_kind,
                    void *hip_stream, int32_t *quartets, int64_t cap, int64_t stride, int64_t *n_out)
{
    g_err.clear();
    if (!pl || !P0 || !PD || !R || !n_out || cap < 0 || stride < 1 || (cap > 0 && !quartets))
        return fail(TDG_EINVAL, "bad arguments");
    if (ptr_kind != 0 && ptr_kind != 1) return fail(TDG_EINVAL, "ptr_kind must be 0 or 1");
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(pl->device));
    int rc;
    if ((rc = prep_density(pl, P0, PD, R, ptr_kind, st)) || (rc = count_pass(pl, st))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    const int nitems = pl->item_class_off[kNumClasses];
    long long total = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        if (!class_active(pl, c)) continue;
        for (int k = pl->item_class_off[c]; k < pl->item_class_off[c + 1]; ++k)
            total += (long long)pl->h_cnt[k] + pl->h_cnt32[k];
    }
    *n_out = total;
    // the list is filled in chunks of bra pairs holding at most kListChunk quartets, and
    // every stride-th quartet (in the order of the chunks) is kept
    constexpr long long kListChunk = 1LL << 27;
    long long written = 0, seen = 0;
    int K0 = 0;
    while (K0 < nitems && written < cap) {
        int K1 = K0;
        long long acc = 0;
        for (int c = 0; K1 < nitems; ++K1) {
            while (K1 >= pl->item_class_off[c + 1]) ++c;
            const long long v = class_active(pl, c) ? (long long)pl->h_cnt[K1] + pl->h_cnt32[K1] : 0;
            if (acc + v > kListChunk && K1 > K0) break;
            acc += v;
        }
        Chunk ch;
        if ((rc = fill_items(pl, st, K0, K1, ch))) return rc;
        const long long L = ch.total;
        const long long j0 = (stride - seen % stride) % stride;
        long long m = L > j0 ? (L - j0 + stride - 1) / stride : 0;
        m = std::min<long long>(m, cap - written);
        if (m > 0) {
            DevBuf<int2> d_s;
            if ((rc = d_s.alloc(m))) return rc;
            hipLaunchKernelGGL(k_sample_tasks, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, pl->d_tasks.p,
                               nullptr, j0, (long long)stride, m, d_s.p, nullptr);
            std::vector<int2> h(m);
            const hipError_t e = hipMemcpyAsync(h.data(), d_s.p, sizeof(int2) * m, hipMemcpyDeviceToHost, st);
            const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(st) : e;
            d_s.release();
            if (e2 != hipSuccess) return fail(TDG_EDEVICE, "survivor copy failed: %s", hipGetErrorString(e2));
            for (long long k = 0; k < m; ++k) {
                int32_t *q = quartets + 4 * (written + k);
                q[0] = pl->pair_sa[h[k].x];
                q[1] = pl->pair_sb[h[k].x];
                q[2] = pl->pair_sa[h[k].y];
                q[3] = pl->pair_sb[h[k].y];
            }
            written += m;
        }
        seen += L;
        K0 = K1;
        if (progress_lines()) {
            fprintf(stderr, "tdgrad: survivor list, %lld of %lld quartets listed, %lld kept\n", seen, total, written);
            fflush(stderr);
        }
    }
    return TDG_OK;
}

int tdg_quartet_contribs(tdg_plan_t *pl, const double *P0, const double *PD, const double *R, int32_t ptr_kind,
                         void *hip_stream, int64_t n, const int32_t *quartets, int32_t precision, double *out)
{
    g_err.clear();
    if (!pl || !P0 || !PD || !R || n < 0 || (n > 0 && (!quartets || !out))) return fail(TDG_EINVAL, "bad arguments");
    if (ptr_kind != 0 && ptr_kind != 1) return fail(TDG_EINVAL, "ptr_kind must be 0 or 1");
    if (precision != 0 && precision != 1) return fail(TDG_EINVAL, "precision must be 0 or 1");
    const int ns = pl->n_shells;
    // canonical task of every quartet and the centre (A, B, C, D) behind each listed shell
    std::vector<int2> task(n);
    std::vector<int> cls(n), pos(4 * n);
    for (long long k = 0; k < n; ++k) {
        const int *q = quartets + 4 * k;
        for (int x = 0; x < 4; ++x)
            if (q[x] < 0 || q[x] >= ns) return fail(TDG_EINVAL, "quartet %lld: shell index out of range", k);
        auto sorted_pair = [&](int x, int y) {
            const long long u = x >= y ? (long long)x * (x + 1) / 2 + y : (long long)y * (y + 1) / 2 + x;
            return pl->user_pair_to_sorted[u];
        };
        int p1 = sorted_pair(q[0], q[1]), p2 = sorted_pair(q[2], q[3]);
        auto pcls = [&](int i) { return pair_class(pl->shell_l[pl->pair_sa[i]], pl->shell_l[pl->pair_sb[i]]); };
        const bool swap_pairs = pcls(p1) < pcls(p2);
        const int bra = swap_pairs ? p2 : p1, ket = swap_pairs ? p1 : p2;
        task[k] = make_int2(bra, ket);
        int pb = pcls(bra), pk = pcls(ket), c = 0;
        for (int x = 0; x < kNumClasses; ++x) {
            int b_, k_;
            class_pk(x, b_, k_);
            if (b_ == pb && k_ == pk) c = x;
        }
        cls[k] = c;
        // listed position -> centre: the pair (q0, q1) is the bra unless swapped; within a
        // pair the first centre is the pair's first shell (equal shells: in order)
        for (int half = 0; half < 2; ++half) {
            const int pi = half == 0 ? p1 : p2;
            const bool is_bra = (half == 0) != swap_pairs;
            const int base = is_bra ? 0 : 2;
            const int s0 = q[2 * half], s1 = q[2 * half + 1];
            const bool flip = s0 != s1 && pl->pair_sa[pi] != s0;
            pos[4 * k + 2 * half] = base + (flip ? 1 : 0);
            pos[4 * k + 2 * half + 1] = base + (flip ? 0 : 1);
        }
    }
    if (n == 0) return TDG_OK;
    // tasks grouped by class (stable), one launch per class
    std::vector<long long> order(n);
    std::iota(order.begin(), order.end(), 0LL);
    std::stable_sort(order.begin(), order.end(), [&](long long x, long long y) { return cls[x] < cls[y]; });
    std::vector<int2> sorted(n);
    for (long long k = 0; k < n; ++k) sorted[k] = task[order[k]];
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(pl->device));
    int rc;
    if ((rc = prep_density(pl, P0, PD, R, ptr_kind, st))) return rc;
    DevBuf<int2> d_t;
    DevBuf<double> d_o;
    if ((rc = d_t.alloc(n)) || (rc = d_o.alloc(12 * n))) {
        d_t.release();
        return rc;
    }
    int err = TDG_OK;
    do {
        if (hipMemcpyAsync(d_t.p, sorted.data(), sizeof(int2) * n, hipMemcpyHostToDevice, st) != hipSuccess) {
            err = fail(TDG_EDEVICE, "task upload failed");
            break;
        }
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((12 * n + 255) / 256)), dim3(256), 0, st, d_o.p, 12 * n);
        const bool lr = (pl->prm.terms & 4) && pl->prm.beta != 0.0;
        if (!pl->ncu) {
            hipDeviceProp_t prop;
            pl->ncu = hipGetDeviceProperties(&prop, pl->device) == hipSuccess ? prop.multiProcessorCount : 256;
        }
        DerivArgs a = deriv_args(pl);
        a.lds_atoms = 0;
        long long b = 0;
        while (b < n && err == TDG_OK) {
            const int c = cls[order[b]];
            long long e = b;
            while (e < n && cls[order[e]] == c) ++e;
            a.tasks = d_t.p + b;
            a.ntasks = e - b;
            a.task_out = d_o.p + 12 * b;
            if (kLaunch[c](pl->variant[precision][c], precision, a, lr, st, pl->ncu * kGridPerCU) != hipSuccess)
                err = fail(TDG_EDEVICE, "class %d launch failed", c);
            b = e;
        }
        if (err) break;
        std::vector<double> h(12 * n);
        if (hipMemcpyAsync(h.data(), d_o.p, sizeof(double) * 12 * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            err = fail(TDG_EDEVICE, "result copy failed");
            break;
        }
        for (long long k = 0; k < n; ++k) {
            const long long q = order[k];
            for (int x = 0; x < 4; ++x)
                for (int d = 0; d < 3; ++d) out[12 * q + 3 * x + d] = h[12 * k + 3 * pos[4 * q + x] + d];
        }
    } while (0);
    d_t.release();
    d_o.release();
    return err;
}

int tdg_fock(tdg_plan_t *pl, const double *B, int32_t ptr_kind, void *hip_stream, double cJ, double cK,
             double cKlr, int32_t relative, double *F, tdg_stats_t *stats)
{
    g_err.clear();
    if (!pl || !B || !F) return fail(TDG_EINVAL, "bad arguments");
    if (ptr_kind != 0 && ptr_kind != 1) return fail(TDG_EINVAL, "ptr_kind must be 0 or 1");
    if (!std::isfinite(cJ) || !std::isfinite(cK) || !std::isfinite(cKlr))
        return fail(TDG_EINVAL, "coefficients must be finite");
    if (cKlr != 0.0 && !(pl->prm.omega > 0.0)) return fail(TDG_EINVAL, "cKlr != 0 needs a plan with omega > 0");
    if (relative != 0 && relative != 1) return fail(TDG_EINVAL, "relative must be 0 or 1");
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(pl->device));
    const int nbf = pl->n_bf, ns = pl->n_shells;
    const size_t nn = (size_t)nbf * nbf;            // internal Cartesian accumulator
    const size_t nu = (size_t)pl->n_user * pl->n_user; // caller's B and F
    int rc;
    const double *dB = B;
    if (ptr_kind == 0) {
        if ((rc = pl->d_in.alloc(3 * nu))) return rc;
        HIP_TRY(hipMemcpyAsync(pl->d_in.p, B, nu * 8, hipMemcpyHostToDevice, st));
        dB = pl->d_in.p;
    }
    if ((rc = pl->d_fockG.alloc(nn))) return rc;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)pl->d_mx.p, 1);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)pl->d_prim_cnt.p, (long long)kNumClasses);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (double *)pl->d_cand_cnt.p, (long long)kNumClasses);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, pl->d_fockG.p, (long long)nn);
    const long long nblk = (long long)ns * ns;
    hipLaunchKernelGGL(k_fock_prep, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, st, ns, nbf, pl->d_shell_l.p,
                       pl->d_shell_ao.p, pl->d_ang.p, dB, pl->d_dens.p, pl->d_bmax.p, pl->d_mx.p, pl->sph,
                       pl->n_user, pl->d_shell_ao_user.p);
    HIP_TRY(hipGetLastError());
    // the screening passes of this call keep one-centre quartets and route nothing to FP32
    struct FockScreen {
        tdg_plan *p;
        ~FockScreen() { p->screen_fock = 0; }
    } guard{pl};
    pl->screen_fock = relative ? 2 : 1;
    if ((rc = count_pass(pl, st))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    if (!pl->ncu) {
        hipDeviceProp_t prop;
        pl->ncu = hipGetDeviceProperties(&prop, pl->device) == hipSuccess ? prop.multiProcessorCount : 256;
    }
    FockArgs fa{};
    fa.coords = pl->d_coords.p; fa.shell_atom = pl->d_shell_atom.p; fa.shell_ao = pl->d_shell_ao.p;
    fa.pair_sa = pl->d_pair_sa.p; fa.pair_sb = pl->d_pair_sb.p; fa.pair_ppoff = pl->d_pair_ppoff.p;
    fa.pair_npp = pl->d_pair_npp.p;
    fa.pp_rec = reinterpret_cast<const double2 *>(pl->d_pp_rec.p);
    fa.bmat = pl->d_dens.p; fa.n_bf = nbf;
    fa.omega = pl->prm.omega; fa.cJ = cJ; fa.cK = cK; fa.cKlr = cKlr;
    fa.G = pl->d_fockG.p;
    const bool lr = cKlr != 0.0;
    const int nitems = pl->item_class_off[kNumClasses];
    long long cls_q[kNumClasses] = {0};
    long long total = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        if (!class_active(pl, c)) continue;
        for (int k = pl->item_class_off[c]; k < pl->item_class_off[c + 1]; ++k) cls_q[c] += pl->h_cnt[k];
        total += cls_q[c];
    }
    // the task list is built in chunks of bra pairs holding at most 2^27 quartets; the kernels
    // of a chunk run before the next chunk's fill pass rewrites the list (same stream)
    constexpr long long kFockChunk = 1LL << 27;
    long long nchunks = 0;
    double kms = 0.0, cls_ms[kNumClasses] = {0.0};
    int K0 = 0;
    while (K0 < nitems) {
        int K1 = K0;
        long long acc = 0;
        for (int c = 0; K1 < nitems; ++K1) {
            while (K1 >= pl->item_class_off[c + 1]) ++c;
            const long long v = class_active(pl, c) ? (long long)pl->h_cnt[K1] : 0;
            if (acc + v > kFockChunk && K1 > K0) break;
            acc += v;
        }
        Chunk ch;
        if ((rc = fill_items(pl, st, K0, K1, ch))) return rc;
        ++nchunks;
        // class launches largest expected work first (primitive quartets x roots x
        // (components + 30)), each to the least loaded of the plan's streams, forked from
        // and joined back into the caller's stream; with stats every launch runs alone on
        // the caller's stream and is timed
        int order[kNumClasses], nord = 0;
        double cost[kNumClasses] = {0.0};
        for (int c = 0; c < kNumClasses; ++c) {
            const long long nq = ch.seg_end[c][0] - ch.seg_begin[c][0];
            if (nq <= 0) continue;
            int pb, pk;
            class_pk(c, pb, pk);
            const int L = kPairL[pb][0] + kPairL[pb][1] + kPairL[pk][0] + kPairL[pk][1];
            const double prim = cls_q[c] > 0 ? (double)pl->h_prim[c] * nq / cls_q[c] : 0.0;
            cost[c] = prim * (L / 2 + 1) * (class_ncomp(c) + 30.0);
            order[nord++] = c;
        }
        std::stable_sort(order, order + nord, [&](int x, int y) { return cost[x] > cost[y]; });
        const int nst = stats ? 1 : pl->nstreams;
        if (nst > 1) {
            HIP_TRY(hipEventRecord(pl->ev_fork, st));
            for (int k = 0; k + 1 < nst; ++k) HIP_TRY(hipStreamWaitEvent(pl->aux[k], pl->ev_fork, 0));
        }
        double load[tdg_plan::kMaxAux + 1] = {0.0};
        for (int oi = 0; oi < nord; ++oi) {
            const int c = order[oi];
            int k = 0;
            for (int q = 1; q < nst; ++q)
                if (load[q] < load[k]) k = q;
            load[k] += cost[c];
            hipStream_t sc = k == 0 ? st : pl->aux[k - 1];
            fa.tasks = pl->d_tasks.p + ch.seg_begin[c][0];
            fa.ntasks = ch.seg_end[c][0] - ch.seg_begin[c][0];
            if (stats) HIP_TRY(hipEventRecord(pl->ev0, st));
            if (kFock[c](fa, lr, sc, pl->ncu * kGridPerCU) != hipSuccess)
                return fail(TDG_EDEVICE, "Fock class %d launch failed", c);
            if (stats) {
                HIP_TRY(hipEventRecord(pl->ev1, st));
                HIP_TRY(hipEventSynchronize(pl->ev1));
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, pl->ev0, pl->ev1));
                cls_ms[c] += ms;
                kms += ms;
            }
        }
        for (int k = 0; k + 1 < nst; ++k) {
            HIP_TRY(hipEventRecord(pl->ev_join[k], pl->aux[k]));
            HIP_TRY(hipStreamWaitEvent(st, pl->ev_join[k], 0));
        }
        K0 = K1;
    }
    double *dF = F;
    if (ptr_kind == 0) dF = pl->d_in.p + nu; // staging slot behind the copy of B
    hipLaunchKernelGGL(k_fock_finish, dim3((unsigned)((nu + 255) / 256)), dim3(256), 0, st, nbf, pl->d_ang.p,
                       pl->d_fockG.p, dF, pl->sph, pl->n_user, pl->d_ao_shell_user.p, pl->d_shell_ao_user.p,
                       pl->d_shell_ao.p, pl->d_shell_l.p);
    HIP_TRY(hipGetLastError());
    if (ptr_kind == 0) {
        HIP_TRY(hipMemcpyAsync(F, dF, nu * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    if (stats) {
        HIP_TRY(hipStreamSynchronize(st));
        std::memset(stats, 0, sizeof(*stats));
        stats->quartets = total;
        for (int c = 0; c < kNumClasses; ++c) {
            stats->class_quartets[c] = cls_q[c];
            stats->class_ms[c] = cls_ms[c];
            stats->class_prim_quartets[c] = (int64_t)pl->h_prim[c];
            stats->prim_quartets += (int64_t)pl->h_prim[c];
            stats->candidates += (int64_t)pl->h_cand[c];
        }
        stats->chunks = nchunks;
        stats->ms_kernels = kms;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return TDG_OK;
}

} // extern "C"

// device-side Rys rule for verification
__global__ void k_rys_rule(int n, double T, double *u, double *w)
{
    const int r = threadIdx.x;
    if (r < n) rys_root_rt(n, T, r, u[r], w[r]);
}

extern "C" int tdg_rys_rule(int32_t n, double T, double *u, double *w)
{
    g_err.clear();
    if (n < 1 || n > 5 || !u || !w || !(T >= 0.0)) return fail(TDG_EINVAL, "bad arguments");
    double *d = nullptr;
    HIP_TRY(hipMalloc((void **)&d, 2 * 8 * sizeof(double)));
    hipLaunchKernelGGL(k_rys_rule, dim3(1), dim3(64), 0, 0, n, T, d, d + 8);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(u, d, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(w, d + 8, n * sizeof(double), hipMemcpyDeviceToHost);
    hipFree(d);
    if (e != hipSuccess) return fail(TDG_EDEVICE, "rys rule: %s", hipGetErrorString(e));
    return TDG_OK;
}
