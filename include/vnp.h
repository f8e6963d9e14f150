/*
 * vnp -- recursive hypot-based vector norms on AMD Instinct MI355X (gfx950).
 *
 * Method: V. Novakovic, "Recursive vectorized computation of the vector p-norm"
 * (arXiv 2509.06220).  The Frobenius norm of x (Sect. 1, Eq. (12I)) is computed by a
 * pairwise tree whose every node combines two partial norms with a hypotenuse (Eq. (hr):
 * ||x|| = hypot(||x_I||, ||x_J||) for any split into disjoint parts I, J); the p-norm
 * (Eq. (p)) by the same tree with the node M (1 + (m/M)^p)^(1/p) (Sect. 4, Eq. (sp)).
 *
 * The tree is fixed by the logical index alone (a perfect binary tree over a fixed
 * bit order, zero-padded), so every result is bitwise reproducible across runs, grid
 * and block shapes, pointer alignment, plain / batched / served calls and streams.
 * vnp_tree_id() names the tree and node; results are bitwise comparable only within
 * one tree id.  The paper's own vector algorithms have the same property for a fixed
 * vector width (Sect. 3).
 *
 * Conventions for every call:
 *   - Pointers named x, offsets, res, ... are DEVICE pointers owned by the caller
 *     (res may also be host-mapped pinned memory).  The library never frees or keeps
 *     them, never writes to x, and accesses them only from work enqueued on `stream`.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All calls are
 *     asynchronous and stream-ordered; results are visible after the stream completes.
 *   - Return value, LAPACK INFO style: 0 = success; -k = argument k is invalid (nothing
 *     is enqueued); > 0 = a HIP runtime error code.  Errors of earlier asynchronous work
 *     surface at the next synchronization, not here.  Nothing aborts or throws across
 *     the ABI.
 *   - n <= 0 (or nseg segments of length 0) give a result of +0.
 *   - "p invalid" below: p <= 0, p NaN, or p so small that 1/p rounded once in the
 *     working precision exceeds 2^1000 (D) or overflows (S): p below about 2^-1000 for D,
 *     2^-128 for S (the node of Sect. 4 is built from RN(1/p)).  A binary32 call rounds p
 *     to binary32 first.
 *   - Special values: any NaN element gives NaN; otherwise any infinite element gives
 *     +inf; otherwise the tree result, which is +inf only if the norm overflows.
 *   - Calls on different streams may run concurrently; each (device, stream) pair gets
 *     its own workspace, created on first use and released by vnp_finalize().
 *   - Work enqueued by a call consists of kernel launches only, so a call can be captured
 *     in a HIP graph once its stream's workspace is large enough (after one call of the
 *     same or a larger size on that stream; a call that must grow the workspace
 *     allocates and synchronizes the stream).  A p-norm with a p other than 1, 2 or
 *     inf also needs its p's constant table on the device, which the first call with
 *     that p (on that device) builds and uploads with a synchronous copy; it is kept
 *     until vnp_finalize().
 */
#ifndef VNP_H
#define VNP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VNP_VERSION_MAJOR 0
#define VNP_VERSION_MINOR 1

/* Data types. */
#define VNP_F64 0
#define VNP_F32 1

/* Status codes beyond the INFO convention. */
#define VNP_OK 0
#define VNP_EAGAIN 100000 /* resource temporarily exhausted (server pool full) */
#define VNP_ENOTFOUND 100001 /* unknown ticket */
#define VNP_EPENDING 100002 /* ticket not complete yet */
#define VNP_ECANCELED 100003 /* request dropped unlaunched by vnp_server_destroy */
#define VNP_ENOMEM 100004 /* request larger than the server's whole pool; host allocation failed */

/* ------------------------------------------------------------------------------------
 * Single vector.  Paper: xNRMF (Sect. 1; the recommended algorithm of Sect. 3) and
 * xNRMP (Sect. 4), over n elements with the BLAS stride convention of xNRM2 (Sect. 3):
 * logical element i (0 <= i < n) is x[i * incx] for incx >= 1 and
 * x[(n - 1 - i) * (-incx)] for incx <= -1.  incx == 0 is invalid (-3).
 * The result is written to *res (one element of the working precision).
 * Errors: n > VNP_MAX_N -> -1; x == NULL with n > 0 -> -2; incx == 0 -> -3;
 * p invalid -> -4 (nrmp only); res == NULL -> -4 (nrmf) / -5 (nrmp).
 * ---------------------------------------------------------------------------------- */
#define VNP_MAX_N (((int64_t)1) << 40)

int vnp_dnrmf(int64_t n, const double *x, int64_t incx, double *res, void *stream);
int vnp_snrmf(int64_t n, const float *x, int64_t incx, float *res, void *stream);

/* vnp_dnrmf for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same kernels and bits as vnp_dnrmf,
 * with the block roots kept in a fixed device array of VNP_NOALLOC_MAX_ROOTS doubles (64 KiB,
 * one per device, held until the process ends) instead of a per-stream workspace.  It never
 * calls hipMalloc or hipFree.  Every call on a device shares that device's array: calls
 * that overlap on one device (another stream, another thread) race and must be serialized by
 * the caller.  With the automatic launch shape every n <= VNP_MAX_N fits (at most 4096 roots
 * on a 256-CU device); a shape forced by vnp_set_launch_shape that needs more roots -> -1.
 * Other errors as vnp_dnrmf. */
#define VNP_NOALLOC_MAX_ROOTS 8192
int vnp_dnrmf_noalloc(int64_t n, const double *x, int64_t incx, double *res, void *stream);

/* p-norm.  p = 1 uses |a| + |b| nodes (Eq. (vp1)); p = +inf, and p at or above the
 * cutoff of Sect. 4 (2^53 for D, 2^24 for S), use max(|a|, |b|) (Eq. (vpI)); p = 2 uses
 * the Frobenius node; other p > 0 use the node of Listing 5 (0 < p < 1 gives the
 * quasi-norm of Sect. 4).  In binary64 the levels inside each tile of the tree (8191 of
 * every 8192 nodes) evaluate that node on log2 of the partial norms (the same rounded
 * exponents RN(p/2), RN(1/p)), the levels above on the values; the relative error of one
 * node stays below 4 max(1, 1/p) eps. */
int vnp_dnrmp(int64_t n, const double *x, int64_t incx, double p, double *res, void *stream);
int vnp_snrmp(int64_t n, const float *x, int64_t incx, float p, float *res, void *stream);

/* Schatten p-norm of a matrix (Sect. 4): with G = U S V*, the p-norm of the singular
 * values s (p = 1 nuclear, p = 2 Frobenius, p = inf spectral norm).  G is m x n column-
 * major at A with leading dimension lda (device, not modified).  A copy of G, scaled by a
 * power of two, is reduced to bidiagonal form by rocSOLVER's gebrd in a per-stream
 * workspace; the library's bisection kernel takes the singular values from the bidiagonal's
 * Golub-Kahan form, and their p-norm is vnp_xnrmp (vnp_xnrmf for p = 2) on the canonical
 * tree, written to *res.  A matrix with an Inf or NaN entry gives NaN.  The call allocates
 * on first use and may synchronize its stream when the workspace grows.
 * m, n, lda <= 2^31 - 1.
 * Errors: m invalid -> -1; n invalid -> -2; A == NULL -> -3; lda < max(1, m) -> -4;
 * p invalid -> -5; res == NULL -> -6. */
int vnp_dschatten(int64_t m, int64_t n, const double *A, int64_t lda, double p, double *res, void *stream);
int vnp_sschatten(int64_t m, int64_t n, const float *A, int64_t lda, float p, float *res, void *stream);

/* Frobenius norm of a complex vector (DZNRMF: double complex, SCNRMF: single complex):
 * z holds n complex elements as (re, im) pairs, element k at z + 2 k incz for incz >= 1
 * (BLAS reverse order for incz <= -1).  Since |z_k|^2 = re^2 + im^2 (Sect. 1), the norm
 * is that of the real view (re_0, im_0, re_1, im_1, ...) of 2n elements, reduced by the
 * canonical tree: for incz == 1 bitwise vnp_dnrmf / vnp_snrmf on the 2n reals, and any
 * stride gives the bits of the contiguous copy.  Errors: n > VNP_MAX_N / 2 -> -1;
 * z == NULL with n > 0 -> -2; incz == 0 -> -3; res == NULL -> -4. */
int vnp_dznrmf(int64_t n, const double *z, int64_t incz, double *res, void *stream);
int vnp_scnrmf(int64_t n, const float *z, int64_t incz, float *res, void *stream);

/* ------------------------------------------------------------------------------------
 * Batched segments in one launch.  Paper: norms of the columns of a multi-dimensional
 * array, computed independently (Sect. 3.1).  x holds n_total elements; segment s is
 * x[offsets[s] .. offsets[s+1]) (offsets: device int64 array of nseg + 1 entries; a
 * negative length counts as empty) and its norm goes to res[s].  Each segment's result is
 * bitwise equal to the single-vector call on it.  Segments are processed in one
 * persistent launch, preceded by a one-block setup launch and followed by a finish
 * launch that reduces the run roots of long segments, with a per-stream workspace.
 * Errors: nseg < 0 -> -1; offsets == NULL -> -2; n_total < 0 or > VNP_MAX_N -> -3;
 * x == NULL -> -4; res == NULL -> -5 (p-norm: p invalid -> -5, res == NULL -> -6).
 * A segment reaching outside [0, n_total) is detected on the device: then every res[s]
 * is NaN and no data is read.
 * ---------------------------------------------------------------------------------- */
int vnp_dnrmf_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const double *x, double *res,
                      void *stream);
int vnp_snrmf_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const float *x, float *res,
                      void *stream);
int vnp_dnrmp_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const double *x, double p,
                      double *res, void *stream);
int vnp_snrmp_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const float *x, float p, float *res,
                      void *stream);

/* Column norms of an m x ncols column-major matrix with leading dimension lda >= m
 * (Sect. 3.1): res[j] = ||A(:, j)||, each bitwise equal to vnp_dnrmf on that column.
 * Errors: m < 0 -> -1; ncols < 0 -> -2; A == NULL -> -3; lda < max(1, m) -> -4;
 * res == NULL -> -5. */
int vnp_dnrmf_cols(int64_t m, int64_t ncols, const double *A, int64_t lda, double *res, void *stream);
int vnp_snrmf_cols(int64_t m, int64_t ncols, const float *A, int64_t lda, float *res, void *stream);

/* Norm of a whole array with a leading dimension (Sect. 3.1): the m x ncols column-major
 * array A (column j at A + j lda; for a higher-dimensional A(LDA, N2, ..., Nk), ncols =
 * N2 ... Nk).  Frobenius (xNRMF_MAT) or entrywise p-norm (xNRMP_MAT, p as in xNRMP).
 * Stored contiguously (lda == m, or one column), the array is one vector: the result is
 * bitwise that of vnp_xnrmf / vnp_xnrmp on its m ncols elements.  Otherwise the column
 * norms (each bitwise the single-vector result of that column) are reduced by the perfect
 * binary tree over the column index (zero-padded, with the same node), one value written
 * to *res.  Rows m .. lda-1 are never read.  Device pointers; stream-ordered.
 * Errors: m < 0 -> -1; ncols < 0 -> -2; A == NULL (with m, ncols > 0) -> -3;
 * lda < max(1, m) or the array spans more than VNP_MAX_N elements -> -4; p invalid
 * -> -5 (p variants); res == NULL -> -5 (-6 for the p variants). */
int vnp_dnrmf_mat(int64_t m, int64_t ncols, const double *A, int64_t lda, double *res, void *stream);
int vnp_snrmf_mat(int64_t m, int64_t ncols, const float *A, int64_t lda, float *res, void *stream);
int vnp_dnrmp_mat(int64_t m, int64_t ncols, const double *A, int64_t lda, double p, double *res, void *stream);
int vnp_snrmp_mat(int64_t m, int64_t ncols, const float *A, int64_t lda, float p, float *res, void *stream);

/* ------------------------------------------------------------------------------------
 * Plans: one batched workload (fixed buffers and segment count) prepared once -- launch
 * shape chosen by timing candidates on `stream` when autotune is set (the shape never
 * changes a result), longest segments scheduled first when host offsets are given, and
 * the setup + batched launches captured in a HIP graph -- then replayed by
 * vnp_plan_exec.  The plan owns its workspace and, for a p-norm, its copy of the p
 * node's table (so it stays valid across vnp_finalize; a plan's replays must not overlap
 * each other); the caller's buffers must stay valid and keep their sizes while the plan
 * exists; their contents may change between replays.
 * Errors (create): plan == NULL -> -1; invalid descriptor -> -2; > 0 HIP error.
 * ---------------------------------------------------------------------------------- */
typedef struct vnp_plan vnp_plan;

typedef struct {
    int dtype;                /* VNP_F64 or VNP_F32 */
    double p;                 /* 2.0 for the Frobenius norm; > 0, may be +inf */
    int64_t nseg;             /* number of segments */
    const int64_t *offsets;   /* device, nseg + 1 entries */
    const int64_t *h_offsets; /* optional host copy of offsets (enables longest-first order) */
    int64_t n_total;          /* elements in x */
    const void *x;            /* device data */
    void *res;                /* device results, nseg elements */
    int autotune;             /* 0: default shape; 1: the cached choice, else time and cache; 2: time and replace */
} vnp_plan_desc;

int vnp_plan_create(vnp_plan **plan, const vnp_plan_desc *desc, void *stream);
int vnp_plan_exec(vnp_plan *plan, void *stream);
int vnp_plan_destroy(vnp_plan *plan);
/* Chosen launch shape: resident blocks, waves per block, tiles per work item. */
int vnp_plan_info(const vnp_plan *plan, int *blocks, int *waves, int *tiles_per_item);
/* The autotune cache.  With autotune = 1, vnp_plan_create takes the shape chosen before
 * for the same device (architecture and CU count), dtype, node kind (hypot, sum, max or
 * generic p), size class (floor log2 of nseg and of n_total), alignment of x and tree id
 * (vnp_tree_id) if there is one, and otherwise times the candidates and records the
 * choice; autotune = 2 always times and replaces the record.  Records live for the
 * process and, when the environment variable VNP_AUTOTUNE_CACHE names a file, in that
 * file as JSON: read at the first lookup, and after each new record merged with the
 * file's current records and rewritten through a temporary file and a rename.  A shape
 * never changes a result, so a stale record costs only time; a file that cannot be read
 * or written is ignored.  vnp_autotune_cache_clear
 * drops the process's records (the file is read again at the next lookup); returns 0. */
int vnp_autotune_cache_clear(void);

/* ------------------------------------------------------------------------------------
 * Library information.
 * ---------------------------------------------------------------------------------- */
const char *vnp_version(void);
/* 32-bit id of the canonical tree and node for a dtype (VNP_F64 / VNP_F32). */
uint32_t vnp_tree_id(int dtype);
/* Elements per tile of the canonical tree for a dtype. */
int64_t vnp_tile_elems(int dtype);
/* Release the current device's per-stream workspaces and p-norm tables.  Not
 * thread-safe with calls in flight. */
int vnp_finalize(void);

/* Launch-shape override for tests and tuning: waves per block and tiles per wave
 * (powers of two, at most 16 and 2^12; 0 = automatic).  Results never depend on it.
 * Process-wide. */
int vnp_set_launch_shape(int waves_per_block, int tiles_per_wave);

#ifdef __cplusplus
}
#endif

#endif /* VNP_H */
