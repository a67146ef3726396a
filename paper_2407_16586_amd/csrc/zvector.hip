// Z-vector (coupled-perturbed) equations of section II.B, eqs cphf and cphf_a, solved by the
// Krylov subspace method of the same section without storing A: every product A b runs as a
// Fock-type matrix build (eqs sigma and zfock, tdg_fock) between two dense transformations.
// The exchange-correlation kernel terms are not part of the products (no grids here).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/tdgrad.h"

extern "C" int tdg_set_error_(int code, const char *msg); // defined in tdgrad.hip
int tdg_plan_device_(const tdg_plan_t *pl);                // defined in tdgrad.hip

#define ZV_TRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return tdg_set_error_(TDG_EDEVICE, hipGetErrorString(e_));           \
    } while (0)

namespace {

// C[M][N] = op(A) op(B) (row-major, leading dimensions lda, ldb, ldc); op = transpose when
// ta / tb is set (A then stored [K][M], B stored [N][K]).  16 x 16 output tiles, the K
// dimension staged through LDS 16 at a time.
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const double *A, int lda, int ta,
                                              const double *B, int ldb, int tb, double *C, int ldc)
{
    __shared__ double sa[16][17], sb[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    double acc = 0.0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int ak = k0 + tx, bk = k0 + ty;
        sa[ty][tx] = (row < M && ak < K) ? (ta ? A[(size_t)ak * lda + row] : A[(size_t)row * lda + ak]) : 0.0;
        sb[ty][tx] = (bk < K && col < N) ? (tb ? B[(size_t)col * ldb + bk] : B[(size_t)bk * ldb + col]) : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += sa[ty][k] * sb[k][tx];
        __syncthreads();
    }
    if (row < M && col < N) C[(size_t)row * ldc + col] = acc;
}

// per-block partial sums of x . y (fixed order: the host adds the blocks in order)
__global__ void __launch_bounds__(256) k_dot(long long n, const double *x, const double *y, double *part)
{
    __shared__ double s[256];
    double v = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        v += x[i] * y[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_axpy(long long n, double a, const double *x, double *y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

__global__ void k_scal(long long n, double a, double *x)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= a;
}

// y[a][i] = x[a][i] / d_ai with d_ai = eps_i - eps_a (virtual a, occupied i)
__global__ void k_dinv(int nv, int no, const double *eo, const double *ev, const double *x, double *y)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)nv * no) return;
    const int a = (int)(k / no), i = (int)(k % no);
    y[k] = x[k] / (eo[i] - ev[a]);
}

constexpr int kDotBlocks = 256;

struct Dev {
    std::vector<double *> bufs;
    ~Dev()
    {
        for (double *p : bufs)
            if (p) hipFree(p);
    }
    double *get(size_t n)
    {
        double *p = nullptr;
        if (hipMalloc((void **)&p, sizeof(double) * (n ? n : 1)) != hipSuccess) return nullptr;
        bufs.push_back(p);
        return p;
    }
};

int gemm(int M, int N, int K, const double *A, int lda, int ta, const double *B, int ldb, int tb, double *C, int ldc)
{
    dim3 grid((N + 15) / 16, (M + 15) / 16);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, nullptr, M, N, K, A, lda, ta, B, ldb, tb, C, ldc);
    ZV_TRY(hipGetLastError());
    return TDG_OK;
}

int dot(long long n, const double *x, const double *y, double *part, double *out)
{
    hipLaunchKernelGGL(k_dot, dim3(kDotBlocks), dim3(256), 0, nullptr, n, x, y, part);
    ZV_TRY(hipGetLastError());
    double h[kDotBlocks];
    ZV_TRY(hipMemcpy(h, part, sizeof(h), hipMemcpyDeviceToHost));
    double s = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) s += h[b];
    *out = s;
    return TDG_OK;
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

// solve the k x k system S a = r by Gaussian elimination with partial pivoting (S, r copied)
bool small_solve(int k, std::vector<double> S, std::vector<double> r, std::vector<double> &a)
{
    for (int c = 0; c < k; ++c) {
        int p = c;
        for (int i = c + 1; i < k; ++i)
            if (std::fabs(S[i * k + c]) > std::fabs(S[p * k + c])) p = i;
        if (S[p * k + c] == 0.0) return false;
        if (p != c) {
            for (int j = 0; j < k; ++j) std::swap(S[c * k + j], S[p * k + j]);
            std::swap(r[c], r[p]);
        }
        for (int i = c + 1; i < k; ++i) {
            const double f = S[i * k + c] / S[c * k + c];
            for (int j = c; j < k; ++j) S[i * k + j] -= f * S[c * k + j];
            r[i] -= f * r[c];
        }
    }
    a.assign(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
        double v = r[i];
        for (int j = i + 1; j < k; ++j) v -= S[i * k + j] * a[j];
        a[i] = v / S[i * k + i];
    }
    return true;
}

} // namespace

extern "C" int tdg_zvector(tdg_plan_t *plan, int32_t n_occ, int32_t n_vir, const double *C_occ, const double *C_vir,
                           const double *eps_occ, const double *eps_vir, const double *L, double cJ, double cK,
                           double cKlr, int32_t relative, double tol, int32_t max_iter, double *Z,
                           int32_t *iterations, double *residual)
{
    if (!plan || !C_occ || !C_vir || !eps_occ || !eps_vir || !L || !Z || n_occ <= 0 || n_vir <= 0 || max_iter < 1 ||
        !(tol > 0.0))
        return tdg_set_error_(TDG_EINVAL, "bad arguments");
    int32_t nbf = 0;
    int rc = tdg_plan_dims(plan, &nbf, nullptr, nullptr);
    if (rc) return rc;
    for (int i = 0; i < n_occ; ++i)
        for (int a = 0; a < n_vir; ++a)
            if (!(eps_occ[i] < eps_vir[a])) return tdg_set_error_(TDG_EINVAL, "every occupied energy must lie below every virtual one");
    ZV_TRY(hipSetDevice(tdg_plan_device_(plan)));
    const long long nvo = (long long)n_vir * n_occ;
    const size_t nn = (size_t)nbf * nbf;
    Dev dv;
    double *dCo = dv.get((size_t)nbf * n_occ), *dCv = dv.get((size_t)nbf * n_vir);
    double *deo = dv.get(n_occ), *dev = dv.get(n_vir);
    double *db0 = dv.get(nvo), *dr = dv.get(nvo), *dT = dv.get((size_t)nbf * (n_occ > n_vir ? n_occ : n_vir));
    double *dB = dv.get(nn), *dF = dv.get(nn), *dS = dv.get(nvo), *dpart = dv.get(kDotBlocks);
    if (!dCo || !dCv || !deo || !dev || !db0 || !dr || !dT || !dB || !dF || !dS || !dpart)
        return tdg_set_error_(TDG_ENOMEM, "device allocation failed");
    ZV_TRY(hipMemcpy(dCo, C_occ, sizeof(double) * nbf * n_occ, hipMemcpyHostToDevice));
    ZV_TRY(hipMemcpy(dCv, C_vir, sizeof(double) * nbf * n_vir, hipMemcpyHostToDevice));
    ZV_TRY(hipMemcpy(deo, eps_occ, sizeof(double) * n_occ, hipMemcpyHostToDevice));
    ZV_TRY(hipMemcpy(dev, eps_vir, sizeof(double) * n_vir, hipMemcpyHostToDevice));
    ZV_TRY(hipMemcpy(dr, L, sizeof(double) * nvo, hipMemcpyHostToDevice));
    // b0 = d^-1 L
    hipLaunchKernelGGL(k_dinv, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, n_vir, n_occ, deo, dev, dr, db0);
    ZV_TRY(hipGetLastError());
    double nb0 = 0.0;
    if ((rc = dot(nvo, db0, db0, dpart, &nb0))) return rc;
    nb0 = std::sqrt(nb0);
    if (nb0 == 0.0) {
        std::memset(Z, 0, sizeof(double) * nvo);
        if (iterations) *iterations = 0;
        if (residual) *residual = 0.0;
        return TDG_OK;
    }
    // orthonormal subspace vectors q_k and their scaled products s_k = d^-1 A q_k
    std::vector<double *> q, s;
    double *q0 = dv.get(nvo);
    if (!q0) return tdg_set_error_(TDG_ENOMEM, "device allocation failed");
    ZV_TRY(hipMemcpy(q0, db0, sizeof(double) * nvo, hipMemcpyDeviceToDevice));
    hipLaunchKernelGGL(k_scal, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, nvo, 1.0 / nb0, q0);
    q.push_back(q0);
    std::vector<double> a, G; // G: the subspace matrix of (I - A'), G_ij = delta_ij - q_i . s_j
    double rn = nb0;
    int it = 0;
    for (it = 0; it < max_iter; ++it) {
        const int k = (int)q.size() - 1;
        // s_k = d^-1 C_v^T F(C_v q_k C_o^T) C_o
        if ((rc = gemm(nbf, n_occ, n_vir, dCv, n_vir, 0, q[k], n_occ, 0, dT, n_occ))) return rc;  // C_v q: [nbf][no]
        if ((rc = gemm(nbf, nbf, n_occ, dT, n_occ, 0, dCo, n_occ, 1, dB, nbf))) return rc;        // (C_v q) C_o^T
        if ((rc = tdg_fock(plan, dB, 1, nullptr, cJ, cK, cKlr, relative, dF, nullptr))) return rc;
        if ((rc = gemm(n_vir, nbf, nbf, dCv, n_vir, 1, dF, nbf, 0, dT, nbf))) return rc;          // C_v^T F: [nv][nbf]
        double *sk = dv.get(nvo);
        if (!sk) return tdg_set_error_(TDG_ENOMEM, "device allocation failed");
        if ((rc = gemm(n_vir, n_occ, nbf, dT, nbf, 0, dCo, n_occ, 0, dS, n_occ))) return rc;      // (C_v^T F) C_o
        hipLaunchKernelGGL(k_dinv, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, n_vir, n_occ, deo, dev, dS, sk);
        ZV_TRY(hipGetLastError());
        s.push_back(sk);
        // grow G to (k+1) x (k+1): G_ij = delta_ij - q_i . s_j
        const int m = k + 1;
        std::vector<double> Gn((size_t)m * m, 0.0);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) Gn[(size_t)i * m + j] = G[(size_t)i * k + j];
        for (int i = 0; i < m; ++i) {
            double v;
            if ((rc = dot(nvo, q[i], s[k], dpart, &v))) return rc;
            Gn[(size_t)i * m + k] = (i == k ? 1.0 : 0.0) - v;
            if (i < k) {
                if ((rc = dot(nvo, q[k], s[i], dpart, &v))) return rc;
                Gn[(size_t)k * m + i] = -v;
            }
        }
        G.swap(Gn);
        std::vector<double> x(m, 0.0);
        x[0] = nb0; // q_i . b0 = |b0| for i = 0, else 0 (orthonormal subspace)
        if (!small_solve(m, G, x, a)) return tdg_set_error_(TDG_ESTATE, "singular subspace matrix");
        // residual r = b0 - sum_j a_j (q_j - s_j)
        ZV_TRY(hipMemcpy(dr, db0, sizeof(double) * nvo, hipMemcpyDeviceToDevice));
        for (int j = 0; j < m; ++j) {
            hipLaunchKernelGGL(k_axpy, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, nvo, -a[j], q[j], dr);
            hipLaunchKernelGGL(k_axpy, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, nvo, a[j], s[j], dr);
        }
        ZV_TRY(hipGetLastError());
        if ((rc = dot(nvo, dr, dr, dpart, &rn))) return rc;
        rn = std::sqrt(rn);
        if (rn <= tol * nb0 || it + 1 == max_iter) {
            ++it;
            break;
        }
        // next subspace vector: the residual orthogonalised against the subspace (twice) and
        // normalised to one -- the normalisation before the Fock build that section III.B
        // describes, which with relative screening also keeps the screening relative
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < m; ++j) {
                double v;
                if ((rc = dot(nvo, q[j], dr, dpart, &v))) return rc;
                hipLaunchKernelGGL(k_axpy, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, nvo, -v, q[j], dr);
            }
        double nr = 0.0;
        if ((rc = dot(nvo, dr, dr, dpart, &nr))) return rc;
        nr = std::sqrt(nr);
        if (!(nr > 1e-14 * nb0)) {
            ++it;
            break;
        }
        double *qn = dv.get(nvo);
        if (!qn) return tdg_set_error_(TDG_ENOMEM, "device allocation failed");
        ZV_TRY(hipMemcpy(qn, dr, sizeof(double) * nvo, hipMemcpyDeviceToDevice));
        hipLaunchKernelGGL(k_scal, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, nvo, 1.0 / nr, qn);
        q.push_back(qn);
    }
    // Z = sum_j a_j q_j
    ZV_TRY(hipMemset(dr, 0, sizeof(double) * nvo));
    for (size_t j = 0; j < a.size(); ++j)
        hipLaunchKernelGGL(k_axpy, dim3(blocks_for(nvo)), dim3(256), 0, nullptr, nvo, a[j], q[j], dr);
    ZV_TRY(hipGetLastError());
    ZV_TRY(hipMemcpy(Z, dr, sizeof(double) * nvo, hipMemcpyDeviceToHost));
    if (iterations) *iterations = it;
    if (residual) *residual = rn / nb0;
    return TDG_OK;
}
