// Schatten p-norm of a matrix (Novakovic, arXiv 2509.06220, Sect. 4: with G = U S V*, the
// Schatten p-norm of G is the vector p-norm of its singular values).  The singular values
// come from rocSOLVER's gesvd (no singular vectors) on a copy of the matrix; their p-norm
// is the library's own xNRMP (xNRMF for p = 2) on the canonical tree.  A tiny kernel turns
// the result into NaN when the SVD reports no convergence.
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
    void *s = nullptr;  // singular values, then the superdiagonal scratch E
    size_t s_bytes = 0;
    rocblas_int *info = nullptr;
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

template <typename T>
__global__ void nan_if_failed(const rocblas_int *info, T *res)
{
    if (*info != 0) *res = T(__builtin_nan(""));
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
    if (!w.handle) {
        if (rocblas_create_handle(&w.handle) != rocblas_status_success) return (int)hipErrorUnknown;
        e = hipMalloc(reinterpret_cast<void **>(&w.info), sizeof(rocblas_int));
        if (e != hipSuccess) return (int)e;
    }
    if (rocblas_set_stream(w.handle, st) != rocblas_status_success) return (int)hipErrorUnknown;
    int rc = grow(&w.a, &w.a_bytes, sizeof(T) * (size_t)m * (size_t)n, st);
    if (!rc) rc = grow(&w.s, &w.s_bytes, sizeof(T) * (size_t)(2 * k), st);
    if (rc) return rc;
    T *a = static_cast<T *>(w.a), *s = static_cast<T *>(w.s);
    e = hipMemcpy2DAsync(a, sizeof(T) * (size_t)m, A, sizeof(T) * (size_t)lda, sizeof(T) * (size_t)m, (size_t)n,
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return (int)e;
    rocblas_status rs;
    if constexpr (sizeof(T) == 8)
        rs = rocsolver_dgesvd(w.handle, rocblas_svect_none, rocblas_svect_none, (rocblas_int)m, (rocblas_int)n, a,
                              (rocblas_int)m, s, nullptr, 1, nullptr, 1, s + k, rocblas_outofplace, w.info);
    else
        rs = rocsolver_sgesvd(w.handle, rocblas_svect_none, rocblas_svect_none, (rocblas_int)m, (rocblas_int)n, a,
                              (rocblas_int)m, s, nullptr, 1, nullptr, 1, s + k, rocblas_outofplace, w.info);
    if (rs != rocblas_status_success) return (int)hipErrorUnknown;
    if constexpr (sizeof(T) == 8)
        rc = p == 2.0 ? vnp_dnrmf(k, s, 1, res, stream) : vnp_dnrmp(k, s, 1, p, res, stream);
    else
        rc = p == 2.0 ? vnp_snrmf(k, s, 1, res, stream) : vnp_snrmp(k, s, 1, (float)p, res, stream);
    if (rc) return rc;
    hipLaunchKernelGGL((nan_if_failed<T>), dim3(1), dim3(1), 0, st, w.info, res);
    return (int)hipGetLastError();
}

int check(int64_t m, int64_t n, const void *A, int64_t lda, double p, const void *res)
{
    if (m < 0 || m > 0x7fffffff) return -1;
    if (n < 0 || n > 0x7fffffff) return -2;
    if (m > 0 && n > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1) || lda > 0x7fffffff) return -4;
    if (!(p > 0)) return -5;
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
            if (w.info) (void)hipFree(w.info);
            it = g_svd.erase(it);
        } else {
            ++it;
        }
    }
    return 0;
}

}  // namespace vnp
