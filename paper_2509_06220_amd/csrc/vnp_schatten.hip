// Schatten p-norm of a matrix (Novakovic, arXiv 2509.06220, Sect. 4: with G = U S V*, the
// Schatten p-norm of G is the vector p-norm of its singular values).
//
// 1. The matrix is copied with an exact power-of-two scale that brings its largest entry
//    into [1/2, 1) (gebrd's Householder norms would overflow or underflow near the ends
//    of the exponent range), and rocSOLVER's gebrd reduces the copy to a bidiagonal B by
//    Householder transformations (backward stable).
// 2. The singular values of B are the non-negative eigenvalues of its Golub-Kahan form:
//    the symmetric tridiagonal matrix of order 2k with zero diagonal and off-diagonal
//    b = (d_1, e_1, d_2, e_2, ..., e_{k-1}, d_k), whose eigenvalues are +-s_i.  Its Sturm
//    count (the number of negative pivots of the LDL^T factorisation of T - x I) is the
//    number of eigenvalues below x, so for x > 0 the number of singular values below x is
//    that count minus k.  Bisection on the count finds each s_i independently: one thread
//    per singular value (tgk_bisect_kernel).  The count is exact for a matrix whose
//    off-diagonal entries differ from b by a few ulps relatively, which keeps the
//    singular values accurate relative to their own size down to the stopping floor.
// 3. Their p-norm is the library's own xNRMP (xNRMF for p = 2) on the canonical tree.
//
// The off-diagonal entries are scaled again by an exact power of two so that the largest
// has magnitude in [1/2, 1) before they are squared, and the singular values are scaled
// back at the end; a matrix with an Inf or NaN entry gives NaN.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "../../include/vnp.h"
#include "vnp_batch.hpp"

namespace {

struct SvdWorkspace {
    rocblas_handle handle = nullptr;
    void *a = nullptr;  // copy of the matrix (m x n, leading dimension m)
    size_t a_bytes = 0;
    void *s = nullptr;  // k singular values, then gebrd's d (k), e (k), tauq (k), taup (k)
    size_t s_bytes = 0;
    void *bb = nullptr;  // squared scaled off-diagonal of the Golub-Kahan form (2k), then 4 parameters
    size_t bb_bytes = 0;
};

std::mutex g_svd_mu;
std::map<std::pair<int, void *>, SvdWorkspace> g_svd;

int grow(void **p, size_t *cap, size_t bytes, hipStream_t st)
{
    if (*cap >= bytes) return 0;
    hipError_t e;
    if (*p) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return (int)e;
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    e = hipMalloc(p, bytes);
    if (e != hipSuccess) return (int)e;
    *cap = bytes;
    return 0;
}

constexpr int PREP_THREADS = 1024;
// bisection stops once hi <= U 2^-STOP_FLOOR_LOG2 (U bounds every singular value)
constexpr int STOP_FLOOR_LOG2 = 200;

// Parameters after the 2k squared entries: [0] the off-diagonal scale, [1] the bound U of
// the scaled singular values, [2] non-finite flag, [3] the matrix scale exponent e (the
// singular values of the copy times 2^e are those of G).
constexpr int PAR_SCALE = 0, PAR_BOUND = 1, PAR_BAD = 2, PAR_MSCALE = 3;

// max |A_ij| and whether A holds a non-finite value, in two steps: blocks over (row
// chunks x column groups) write per-block partials (at most MAX_PARTS), then one block
// reduces them into par: the power-of-two exponent e with max |A| in [2^(e-1), 2^e)
// (0 for an all-zero or non-finite A) and the non-finite flag.  A maximum is exact in any
// order.
constexpr int MAX_PARTS = 1024;

template <typename T>
__global__ void __launch_bounds__(256)
    matrix_max_kernel(const T *A, int64_t m, int64_t n, int64_t lda, double *pmax, double *pbad)
{
    __shared__ double smax[256];
    __shared__ int sbad[256];
    double mx = 0.0;
    int bad = 0;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
            const double v = __builtin_fabs((double)A[j * lda + i]);
            bad |= !(v <= __builtin_huge_val());
            mx = v > mx ? v : mx;
        }
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = smax[threadIdx.x] > smax[threadIdx.x + w] ? smax[threadIdx.x] : smax[threadIdx.x + w];
            sbad[threadIdx.x] |= sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int b = blockIdx.y * gridDim.x + blockIdx.x;
        pmax[b] = smax[0];
        pbad[b] = sbad[0] ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(PREP_THREADS)
    matrix_scale_kernel(const double *pmax, const double *pbad, int nparts, double *par)
{
    __shared__ double smax[PREP_THREADS];
    __shared__ int sbad[PREP_THREADS];
    double mx = 0.0;
    int bad = 0;
    for (int b = threadIdx.x; b < nparts; b += PREP_THREADS) {
        mx = pmax[b] > mx ? pmax[b] : mx;
        bad |= pbad[b] != 0.0;
    }
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = PREP_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = smax[threadIdx.x] > smax[threadIdx.x + w] ? smax[threadIdx.x] : smax[threadIdx.x + w];
            sbad[threadIdx.x] |= sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double amax = smax[0];
        par[PAR_MSCALE] = (amax > 0.0 && !sbad[0]) ? (double)__builtin_amdgcn_frexp_exp(amax) : 0.0;
        par[PAR_BAD] = sbad[0] ? 1.0 : 0.0;
    }
}

// The scaled contiguous copy a = A 2^-e (exact in binary64, then converted to T).
template <typename T>
__global__ void __launch_bounds__(256)
    scaled_copy_kernel(const T *A, int64_t m, int64_t n, int64_t lda, const double *par, T *a)
{
    const int ne = -(int)par[PAR_MSCALE];
    const int64_t total = m * n, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t j = t / m, i = t - j * m;
        a[t] = T(__builtin_amdgcn_ldexp((double)A[j * lda + i], ne));
    }
}

// Off-diagonal entry j (0 <= j < 2k - 1) of the Golub-Kahan form of the bidiagonal (d, e).
template <typename T>
__device__ __forceinline__ double gk_offdiag(const T *d, const T *e, int64_t j)
{
    return (double)((j & 1) ? e[j >> 1] : d[j >> 1]);
}

// One block: the power-of-two scale that brings max |b_j| into [1/2, 1), the squares of the
// scaled entries, and the parameters: the scale, U (bound of the scaled singular values)
// and the non-finite flag (set here or by matrix_scale_kernel).
template <typename T>
__global__ void __launch_bounds__(PREP_THREADS) tgk_prepare_kernel(const T *d, const T *e, int64_t k, double *bb)
{
    __shared__ double smax[PREP_THREADS];
    __shared__ int sbad[PREP_THREADS];
    const int64_t nb = 2 * k - 1;
    double mx = 0.0;
    int bad = 0;
    for (int64_t j = threadIdx.x; j < nb; j += PREP_THREADS) {
        const double b = __builtin_fabs(gk_offdiag(d, e, j));
        bad |= !(b <= __builtin_huge_val());  // Inf or NaN
        mx = b > mx ? b : mx;
    }
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = PREP_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = smax[threadIdx.x] > smax[threadIdx.x + w] ? smax[threadIdx.x] : smax[threadIdx.x + w];
            sbad[threadIdx.x] |= sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    const double bmax = smax[0];
    // 2^-e with bmax = f 2^e, f in [1/2, 1); 1 for a zero bidiagonal
    const double scale = (bmax > 0.0 && !sbad[0]) ? __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(bmax)) : 1.0;
    for (int64_t j = threadIdx.x; j < nb; j += PREP_THREADS) {
        const double b = gk_offdiag(d, e, j) * scale;
        bb[j] = b * b;
    }
    if (threadIdx.x == 0) {
        double *par = bb + 2 * k;
        par[PAR_SCALE] = scale;
        par[PAR_BOUND] = 2.0 * (bmax * scale) * (1.0 + 0x1p-40);  // Gershgorin: row sums of |T| <= 2 max |b|
        par[PAR_BAD] = (sbad[0] || par[PAR_BAD] != 0.0) ? 1.0 : 0.0;
    }
}

// Number of eigenvalues of the scaled Golub-Kahan form below x (> 0): negative pivots of
// the LDL^T factorisation of T - x I, with tiny pivots replaced by -pivmin.
__device__ __forceinline__ int64_t tgk_count_below(const double *bb, int64_t n2, double x)
{
    constexpr double PIVMIN = 0x1p-1000;
    double q = -x;
    int64_t c = 1;  // q_0 = -x < 0
    for (int64_t j = 1; j < n2; j++) {
        q = -x - bb[j - 1] / q;
        q = __builtin_fabs(q) < PIVMIN ? -PIVMIN : q;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

// Thread i finds the i-th smallest singular value by bisection on [0, U]: the invariant is
// #(s < lo) <= i < #(s < hi).  It stops when the interval is within REL of hi, when no
// double lies strictly inside, or when hi falls below the floor.
template <typename T>
__global__ void __launch_bounds__(256) tgk_bisect_kernel(const double *bb, int64_t k, T *s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const double *par = bb + 2 * k;
    const double scale = par[PAR_SCALE], U = par[PAR_BOUND];
    if (par[PAR_BAD] != 0.0) {
        s[i] = T(__builtin_nan(""));
        return;
    }
    constexpr double REL = sizeof(T) == 8 ? 0x1p-52 : 0x1p-30;
    const double floor = __builtin_amdgcn_ldexp(U, -STOP_FLOOR_LOG2);
    double lo = 0.0, hi = U;
    while (hi > floor && hi - lo > REL * hi) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (tgk_count_below(bb, 2 * k, mid) - k > i)
            hi = mid;
        else
            lo = mid;
    }
    s[i] = T(__builtin_amdgcn_ldexp((0.5 * (lo + hi)) / scale, (int)par[PAR_MSCALE]));
}

template <typename T>
int schatten(int64_t m, int64_t n, const T *A, int64_t lda, double p, T *res, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (m == 0 || n == 0) {
        if constexpr (sizeof(T) == 8)
            return vnp_dnrmf(0, nullptr, 1, reinterpret_cast<double *>(res), stream);
        else
            return vnp_snrmf(0, nullptr, 1, reinterpret_cast<float *>(res), stream);
    }
    const int64_t k = std::min(m, n);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    std::lock_guard<std::mutex> lk(g_svd_mu);
    SvdWorkspace &w = g_svd[std::make_pair(dev, stream)];
    if (!w.handle && rocblas_create_handle(&w.handle) != rocblas_status_success) return (int)hipErrorUnknown;
    if (rocblas_set_stream(w.handle, st) != rocblas_status_success) return (int)hipErrorUnknown;
    int rc = grow(&w.a, &w.a_bytes, sizeof(T) * (size_t)m * (size_t)n, st);
    if (!rc) rc = grow(&w.s, &w.s_bytes, sizeof(T) * (size_t)(5 * k), st);
    if (!rc) rc = grow(&w.bb, &w.bb_bytes, sizeof(double) * (size_t)(2 * k + 4 + 2 * MAX_PARTS), st);
    if (rc) return rc;
    T *a = static_cast<T *>(w.a), *s = static_cast<T *>(w.s);
    T *bd = s + k, *be = s + 2 * k, *tauq = s + 3 * k, *taup = s + 4 * k;  // B's diagonal, off-diagonal
    double *bb = static_cast<double *>(w.bb);
    double *par = bb + 2 * k;
    // row chunks of 256 x column groups, at most MAX_PARTS blocks
    const int gx = (int)std::min<int64_t>((m + 255) / 256, 64);
    const int gy = (int)std::min<int64_t>(n, MAX_PARTS / gx);
    double *pmax = par + 4, *pbad = pmax + MAX_PARTS;
    hipLaunchKernelGGL((matrix_max_kernel<T>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, A, m, n, lda, pmax,
                       pbad);
    hipLaunchKernelGGL(matrix_scale_kernel, dim3(1), dim3(PREP_THREADS), 0, st, (const double *)pmax,
                       (const double *)pbad, gx * gy, par);
    const int64_t cblocks = std::min<int64_t>((m * n + 255) / 256, 4096);
    hipLaunchKernelGGL((scaled_copy_kernel<T>), dim3((unsigned)cblocks), dim3(256), 0, st, A, m, n, lda,
                       (const double *)par, a);
    e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    rocblas_status rs;
    if constexpr (sizeof(T) == 8)
        rs = rocsolver_dgebrd(w.handle, (rocblas_int)m, (rocblas_int)n, a, (rocblas_int)m, bd, be, tauq, taup);
    else
        rs = rocsolver_sgebrd(w.handle, (rocblas_int)m, (rocblas_int)n, a, (rocblas_int)m, bd, be, tauq, taup);
    if (rs != rocblas_status_success) return (int)hipErrorUnknown;
    hipLaunchKernelGGL((tgk_prepare_kernel<T>), dim3(1), dim3(PREP_THREADS), 0, st, bd, be, k, bb);
    hipLaunchKernelGGL((tgk_bisect_kernel<T>), dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, bb, k, s);
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return (int)le;
    if constexpr (sizeof(T) == 8)
        return p == 2.0 ? vnp_dnrmf(k, s, 1, res, stream) : vnp_dnrmp(k, s, 1, p, res, stream);
    else
        return p == 2.0 ? vnp_snrmf(k, s, 1, res, stream) : vnp_snrmp(k, s, 1, (float)p, res, stream);
}

template <typename T>
int check(int64_t m, int64_t n, const void *A, int64_t lda, T p, const void *res)
{
    if (m < 0 || m > 0x7fffffff) return -1;
    if (n < 0 || n > 0x7fffffff) return -2;
    if (m > 0 && n > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1) || lda > 0x7fffffff) return -4;
    if (!vnp::p_ok(p)) return -5;
    if (!res) return -6;
    return 0;
}

}  // namespace

extern "C" {

int vnp_dschatten(int64_t m, int64_t n, const double *A, int64_t lda, double p, double *res, void *stream)
{
    const int a = check(m, n, A, lda, p, res);
    return a ? a : schatten<double>(m, n, A, lda, p, res, stream);
}

int vnp_sschatten(int64_t m, int64_t n, const float *A, int64_t lda, float p, float *res, void *stream)
{
    const int a = check(m, n, A, lda, p, res);
    return a ? a : schatten<float>(m, n, A, lda, p, res, stream);
}

}  // extern "C"

namespace vnp {

int release_svd_workspaces()
{
    std::lock_guard<std::mutex> lk(g_svd_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto it = g_svd.begin(); it != g_svd.end();) {
        if (it->first.first == dev) {
            SvdWorkspace &w = it->second;
            if (w.handle) (void)rocblas_destroy_handle(w.handle);
            if (w.a) (void)hipFree(w.a);
            if (w.s) (void)hipFree(w.s);
            if (w.bb) (void)hipFree(w.bb);
            it = g_svd.erase(it);
        } else {
            ++it;
        }
    }
    return 0;
}

}  // namespace vnp
