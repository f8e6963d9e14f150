/*
 * vnp oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference for the recursive hypot-based vector norms of
 * V. Novakovic, "Recursive vectorized computation of the vector p-norm"
 * (arXiv 2509.06220).  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library; the GPU library never does, and the two share
 * no code.  Everything here is written from the paper's text:
 *
 *   - cr_hypot[f]: the correctly rounded hypotenuse RN(sqrt(x^2 + y^2)) (Sect. 1,
 *     Eq. (hypot) with |eps_h| <= eps; the A algorithms of Table 2).  Evaluated in
 *     extended precision; whenever that value is not provably inside the rounding
 *     interval, the rounding is decided by exact integer comparison of x^2 + y^2
 *     with the squared midpoints.
 *   - v1_hypot[f]: the branch-free node of Listing 2 (H algorithms).
 *   - cr_pow[f]: x^y correctly rounded, from a binary128 powq value; the cases
 *     binary128 cannot decide go to MPFR's correctly rounded mpfr_pow.
 *   - v1_lp[f]: the p-norm node of Listing 5 / Eq. (sp), (qp) with cr_pow; p = 1
 *     and p = infinity use the sumabs / maxabs nodes of Eq. (vp1) / (vpI); p at or
 *     above the cutoff of Sect. 4 (2^53 for D, 2^24 for S) uses maxabs.
 *   - R: the scalar recursion of Sect. 2 (Listing 1): ceil split, the left part at
 *     most one element longer; n = 1 gives |x|, n = 2 one node.  A = R with
 *     cr_hypot, H = R with v1_hypot, A_p = R with v1_lp.
 *   - Z: the vector recursion of Sect. 3 (Listing 4) with P lanes: lane l reduces
 *     x[l], x[l+P], ... (zero-padded tail) by R's tree with the v1 node, then A
 *     reduces the P lane values (the recommended xNRMF: Z paired with A).
 *   - an exact sum of squares (fixed-point superaccumulator) and a binary128
 *     p-norm reference for the "exact" norm of Sect. 2's tester.
 *
 * Threads split the top levels of the same recursion (as OpenCilk does in
 * Listing 1), so results are bitwise independent of the thread count.
 */
#include <float.h>
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* 192-bit unsigned integers for exact comparisons                     */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t w[3];
} u192;

static int u192_sq_shl(uint64_t X, int s, u192 *r)
{
    unsigned __int128 p = (unsigned __int128)X * X;
    uint64_t w0 = (uint64_t)p, w1 = (uint64_t)(p >> 64), w2 = 0;
    if (s < 0 || s > 191) return -1;
    while (s >= 64) {
        if (w2) return -1;
        w2 = w1;
        w1 = w0;
        w0 = 0;
        s -= 64;
    }
    if (s) {
        if (w2 >> (64 - s)) return -1;
        w2 = (w2 << s) | (w1 >> (64 - s));
        w1 = (w1 << s) | (w0 >> (64 - s));
        w0 <<= s;
    }
    r->w[0] = w0;
    r->w[1] = w1;
    r->w[2] = w2;
    return 0;
}

static int u192_add(u192 *a, const u192 *b)
{
    unsigned __int128 c = 0;
    for (int i = 0; i < 3; ++i) {
        c += (unsigned __int128)a->w[i] + b->w[i];
        a->w[i] = (uint64_t)c;
        c >>= 64;
    }
    return c ? -1 : 0;
}

static int u192_cmp(const u192 *a, const u192 *b)
{
    for (int i = 2; i >= 0; --i) {
        if (a->w[i] != b->w[i]) return a->w[i] < b->w[i] ? -1 : 1;
    }
    return 0;
}

/* v = V * 2^e with V odd (v > 0 finite). */
static void split_d(double v, uint64_t *V, int *e)
{
    int ex;
    double f = frexp(v, &ex);
    uint64_t m = (uint64_t)ldexp(f, 53);
    int s = __builtin_ctzll(m);
    *V = m >> s;
    *e = ex - 53 + s;
}

static void split_ld(long double v, uint64_t *V, int *e)
{
    int ex;
    long double f = frexpl(v, &ex);
    uint64_t m = (uint64_t)ldexpl(f, 64);
    int s = __builtin_ctzll(m);
    *V = m >> s;
    *e = ex - 64 + s;
}

static volatile int64_t g_exact_failures = 0;

/* Sign of a^2 + b^2 - m^2, exactly.  a >= b >= 0 finite doubles, m > 0 finite long double,
 * and all nonzero values within a factor 2^90 of each other. */
static int cmp_sumsq_sq(double a, double b, long double m)
{
    uint64_t A = 0, B = 0, M;
    int ea = 0, eb = 0, em;
    int z;
    split_ld(m, &M, &em);
    z = 2 * em;
    if (a > 0) {
        split_d(a, &A, &ea);
        if (2 * ea < z) z = 2 * ea;
    }
    if (b > 0) {
        split_d(b, &B, &eb);
        if (2 * eb < z) z = 2 * eb;
    }
    u192 s = {{0, 0, 0}}, t, mm;
    int bad = 0;
    if (a > 0) {
        bad |= u192_sq_shl(A, 2 * ea - z, &t);
        bad |= u192_add(&s, &t);
    }
    if (b > 0) {
        bad |= u192_sq_shl(B, 2 * eb - z, &t);
        bad |= u192_add(&s, &t);
    }
    bad |= u192_sq_shl(M, 2 * em - z, &mm);
    if (bad) {
        __atomic_add_fetch(&g_exact_failures, 1, __ATOMIC_RELAXED);
        return 0;
    }
    return u192_cmp(&s, &mm);
}

int64_t vnpo_exact_failures(void) { return g_exact_failures; }

/* ------------------------------------------------------------------ */
/* Correctly rounded hypotenuse                                        */
/* ------------------------------------------------------------------ */
static double even_d(double u, double v)
{
    uint64_t bu;
    memcpy(&bu, &u, 8);
    return (bu & 1) ? v : u;
}

static float even_f(float u, float v)
{
    uint32_t bu;
    memcpy(&bu, &u, 4);
    return (bu & 1) ? v : u;
}

/* RN(sqrt(x^2 + y^2)) in binary64 (C99 conventions for infinities and NaNs). */
double vnpo_cr_hypot(double x, double y)
{
    double a = fabs(x), b = fabs(y);
    if (isinf(a) || isinf(b)) return INFINITY;
    if (isnan(a) || isnan(b)) return NAN;
    if (a < b) {
        double t = a;
        a = b;
        b = t;
    }
    if (b == 0.0) return a;
    /* b / a < 2^-27: a(sqrt(1 + (b/a)^2) - 1) < a 2^-55 < ulp(a) / 2, so RN gives a. */
    if (b < ldexp(a, -27)) return a;
    const long double A = a, B = b;
    const long double t = sqrtl(A * A + B * B); /* relative error below 2^-62 */
    double c = (double)t;
    if (isinf(c)) c = DBL_MAX;
    for (int it = 0; it < 8; ++it) {
        const double up = nextafter(c, INFINITY);
        const double dn = nextafter(c, 0.0);
        const long double mhi = isinf(up) ? (long double)DBL_MAX + ldexpl(1.0L, 970) : ((long double)c + up) / 2;
        const long double mlo = ((long double)c + dn) / 2;
        const long double tol = t * 0x1p-58L;
        if (t > mlo + tol && t < mhi - tol) return c;
        const int shi = cmp_sumsq_sq(a, b, mhi);
        if (shi > 0) {
            if (isinf(up)) return INFINITY;
            c = up;
            continue;
        }
        if (shi == 0) return even_d(c, up);
        const int slo = cmp_sumsq_sq(a, b, mlo);
        if (slo < 0) {
            c = dn;
            continue;
        }
        if (slo == 0) return even_d(dn, c);
        return c;
    }
    __atomic_add_fetch(&g_exact_failures, 1, __ATOMIC_RELAXED);
    return c;
}

/* RN(sqrt(x^2 + y^2)) in binary32. */
float vnpo_cr_hypotf(float x, float y)
{
    double a = fabs((double)x), b = fabs((double)y);
    if (isinf(a) || isinf(b)) return INFINITY;
    if (isnan(a) || isnan(b)) return NAN;
    if (a < b) {
        double t = a;
        a = b;
        b = t;
    }
    if (b == 0.0) return (float)a;
    /* b / a < 2^-12: the excess a 2^-25 is below ulp_S(a) / 2. */
    if (b < ldexp(a, -12)) return (float)a;
    const double t = sqrt(a * a + b * b); /* squares exact; relative error below 2^-52 */
    float c = (float)t;
    if (isinf(c)) c = FLT_MAX;
    for (int it = 0; it < 8; ++it) {
        const float up = nextafterf(c, INFINITY);
        const float dn = nextafterf(c, 0.0f);
        const double mhi = isinf(up) ? (double)FLT_MAX + ldexp(1.0, 103) : ((double)c + up) / 2;
        const double mlo = ((double)c + dn) / 2;
        const double tol = t * 0x1p-49;
        if (t > mlo + tol && t < mhi - tol) return c;
        const int shi = cmp_sumsq_sq(a, b, mhi);
        if (shi > 0) {
            if (isinf(up)) return INFINITY;
            c = up;
            continue;
        }
        if (shi == 0) return even_f(c, up);
        const int slo = cmp_sumsq_sq(a, b, mlo);
        if (slo < 0) {
            c = dn;
            continue;
        }
        if (slo == 0) return even_f(dn, c);
        return c;
    }
    __atomic_add_fetch(&g_exact_failures, 1, __ATOMIC_RELAXED);
    return c;
}

/* ------------------------------------------------------------------ */
/* Listing 2: v1_hypot                                                 */
/* ------------------------------------------------------------------ */
double vnpo_v1_hypot(double x, double y)
{
    const double X = fabs(x);
    const double Y = fabs(y);
    const double m = fmin(X, Y);
    const double M = fmax(X, Y);
    const double q = m / M;
    const double Q = fmax(q, 0.0);
    const double S = fma(Q, Q, 1.0);
    const double s = sqrt(S);
    return M * s;
}

float vnpo_v1_hypotf(float x, float y)
{
    const float X = fabsf(x);
    const float Y = fabsf(y);
    const float m = fminf(X, Y);
    const float M = fmaxf(X, Y);
    const float q = m / M;
    const float Q = fmaxf(q, 0.0f);
    const float S = fmaf(Q, Q, 1.0f);
    const float s = sqrtf(S);
    return M * s;
}

/* ------------------------------------------------------------------ */
/* Correctly rounded pow: binary128 powq, MPFR for the hard cases       */
/* ------------------------------------------------------------------ */
/* When the binary128 value lies within 2^-104 (relative) of a rounding boundary,
 * the result is recomputed with MPFR's correctly rounded mpfr_pow (GNU MPFR, loaded
 * at run time through its documented C API).  Such calls are counted; calls MPFR
 * could not settle (library missing) are counted separately as unresolved. */
#include <dlfcn.h>

typedef struct {
    long prec;
    int sign;
    long exp;
    void *d;
} mpfr_s;

static struct {
    int state; /* 0 unknown, 1 loaded, -1 unavailable */
    void (*init2)(mpfr_s *, long);
    void (*clear)(mpfr_s *);
    int (*set_d)(mpfr_s *, double, int);
    int (*pow)(mpfr_s *, const mpfr_s *, const mpfr_s *, int);
    double (*get_d)(const mpfr_s *, int);
    float (*get_flt)(const mpfr_s *, int);
} g_mpfr;

static int mpfr_load(void)
{
    if (__atomic_load_n(&g_mpfr.state, __ATOMIC_ACQUIRE)) return g_mpfr.state > 0;
#pragma omp critical(vnpo_mpfr_load)
    if (!g_mpfr.state) {
        void *h = dlopen("libmpfr.so.6", RTLD_NOW | RTLD_LOCAL);
        if (h) {
            g_mpfr.init2 = (void (*)(mpfr_s *, long))dlsym(h, "mpfr_init2");
            g_mpfr.clear = (void (*)(mpfr_s *))dlsym(h, "mpfr_clear");
            g_mpfr.set_d = (int (*)(mpfr_s *, double, int))dlsym(h, "mpfr_set_d");
            g_mpfr.pow = (int (*)(mpfr_s *, const mpfr_s *, const mpfr_s *, int))dlsym(h, "mpfr_pow");
            g_mpfr.get_d = (double (*)(const mpfr_s *, int))dlsym(h, "mpfr_get_d");
            g_mpfr.get_flt = (float (*)(const mpfr_s *, int))dlsym(h, "mpfr_get_flt");
        }
        const int ok = h && g_mpfr.init2 && g_mpfr.clear && g_mpfr.set_d && g_mpfr.pow && g_mpfr.get_d &&
                       g_mpfr.get_flt;
        __atomic_store_n(&g_mpfr.state, ok ? 1 : -1, __ATOMIC_RELEASE);
    }
    return g_mpfr.state > 0;
}

/* x^y rounded to nearest at `prec` bits (53 or 24); returns 0 if MPFR is unavailable. */
static int mpfr_pow_rn(double x, double y, int prec, double *out)
{
    if (!mpfr_load()) return 0;
    mpfr_s X, Y, R;
    g_mpfr.init2(&X, 64);
    g_mpfr.init2(&Y, 64);
    g_mpfr.init2(&R, prec);
    g_mpfr.set_d(&X, x, 0);
    g_mpfr.set_d(&Y, y, 0);
    g_mpfr.pow(&R, &X, &Y, 0); /* MPFR_RNDN = 0 */
    *out = prec == 24 ? (double)g_mpfr.get_flt(&R, 0) : g_mpfr.get_d(&R, 0);
    g_mpfr.clear(&X);
    g_mpfr.clear(&Y);
    g_mpfr.clear(&R);
    return 1;
}

static volatile int64_t g_pow_ambiguous = 0, g_pow_unresolved = 0;

int64_t vnpo_pow_ambiguous(void) { return g_pow_ambiguous; }
int64_t vnpo_pow_unresolved(void) { return g_pow_unresolved; }

void vnpo_reset_counters(void)
{
    g_pow_ambiguous = 0;
    g_pow_unresolved = 0;
    g_exact_failures = 0;
}

/* x^y for x >= 0 and y > 0 finite (the only arguments Listing 5 produces). */
double vnpo_cr_pow(double x, double y)
{
    if (isnan(x) || isnan(y)) return NAN;
    if (x == 0.0) return 0.0;
    if (x == 1.0) return 1.0;
    if (y == 1.0) return x;
    const __float128 t = powq((__float128)x, (__float128)y);
    double c = (double)t;
    if (c == 0.0 || isinf(c)) return c; /* far outside the range a node can reach */
    const double up = nextafter(c, INFINITY), dn = nextafter(c, 0.0);
    const __float128 mhi = ((__float128)c + up) / 2, mlo = ((__float128)c + dn) / 2;
    const __float128 tol = t * 0x1p-104Q;
    if (!(t > mlo + tol && t < mhi - tol)) {
        double r;
        __atomic_add_fetch(&g_pow_ambiguous, 1, __ATOMIC_RELAXED);
        if (mpfr_pow_rn(x, y, 53, &r)) return r;
        __atomic_add_fetch(&g_pow_unresolved, 1, __ATOMIC_RELAXED);
    }
    return c;
}

float vnpo_cr_powf(float x, float y)
{
    if (isnan(x) || isnan(y)) return NAN;
    if (x == 0.0f) return 0.0f;
    if (x == 1.0f) return 1.0f;
    if (y == 1.0f) return x;
    const __float128 t = powq((__float128)x, (__float128)y);
    float c = (float)t;
    if (c == 0.0f || isinf(c)) return c;
    const float up = nextafterf(c, INFINITY), dn = nextafterf(c, 0.0f);
    const __float128 mhi = ((__float128)c + up) / 2, mlo = ((__float128)c + dn) / 2;
    const __float128 tol = t * 0x1p-104Q;
    if (!(t > mlo + tol && t < mhi - tol)) {
        double r;
        __atomic_add_fetch(&g_pow_ambiguous, 1, __ATOMIC_RELAXED);
        if (mpfr_pow_rn(x, y, 24, &r)) return (float)r;
        __atomic_add_fetch(&g_pow_unresolved, 1, __ATOMIC_RELAXED);
    }
    return c;
}

/* The MPFR route alone, for tests. */
double vnpo_mpfr_pow(double x, double y, int prec)
{
    double r;
    return mpfr_pow_rn(x, y, prec, &r) ? r : NAN;
}

/* ------------------------------------------------------------------ */
/* Listing 5: v1_lp, and the p = 1 / p = infinity nodes                 */
/* ------------------------------------------------------------------ */
double vnpo_v1_lp(double p, double x, double y)
{
    const double X = fabs(x);
    const double Y = fabs(y);
    const double m = fmin(X, Y);
    const double M = fmax(X, Y);
    const double q = m / M;
    const double Q = fmax(q, 0.0);
    const double S = vnpo_cr_pow(Q, p * 0.5);
    const double Z = fma(S, S, 1.0);
    const double C = vnpo_cr_pow(Z, 1.0 / p);
    return M * C;
}

float vnpo_v1_lpf(float p, float x, float y)
{
    const float X = fabsf(x);
    const float Y = fabsf(y);
    const float m = fminf(X, Y);
    const float M = fmaxf(X, Y);
    const float q = m / M;
    const float Q = fmaxf(q, 0.0f);
    const float S = vnpo_cr_powf(Q, p * 0.5f);
    const float Z = fmaf(S, S, 1.0f);
    const float C = vnpo_cr_powf(Z, 1.0f / p);
    return M * C;
}

/* ------------------------------------------------------------------ */
/* Nodes and the recursion R                                          */
/* ------------------------------------------------------------------ */
enum { NODE_CR = 0, NODE_V1 = 1, NODE_LP = 2, NODE_SUM = 3, NODE_MAX = 4, NODE_TRACE = 5 };

typedef struct {
    int kind;
    double p;
    int64_t *log; /* NODE_TRACE: pairs of (left, right) operand ids */
    int64_t nlog;
} node_t;

static double node_d(node_t *nd, double a, double b)
{
    switch (nd->kind) {
    case NODE_CR:
        return vnpo_cr_hypot(a, b);
    case NODE_V1:
        return vnpo_v1_hypot(a, b);
    case NODE_LP:
        return vnpo_v1_lp(nd->p, a, b);
    case NODE_SUM:
        return fabs(a) + fabs(b);
    case NODE_MAX:
        return fmax(fabs(a), fabs(b));
    default: { /* trace: operands are ids; the result is a fresh id */
        const int64_t k = nd->nlog++;
        nd->log[2 * k] = (int64_t)fabs(a);
        nd->log[2 * k + 1] = (int64_t)fabs(b);
        return (double)(1000000 + k);
    }
    }
}

static float node_s(node_t *nd, float a, float b)
{
    switch (nd->kind) {
    case NODE_CR:
        return vnpo_cr_hypotf(a, b);
    case NODE_V1:
        return vnpo_v1_hypotf(a, b);
    case NODE_LP:
        return vnpo_v1_lpf((float)nd->p, a, b);
    case NODE_SUM:
        return fabsf(a) + fabsf(b);
    case NODE_MAX:
        return fmaxf(fabsf(a), fabsf(b));
    default:
        return 0.0f;
    }
}

/* Elements e_r = (r < nvalid ? x[r * stride] : 0), r in [0, m): R's tree over them. */
static double R_d(node_t *nd, const double *x, int64_t stride, int64_t m, int64_t nvalid, int spawn)
{
    if (m == 1) return nvalid > 0 ? fabs(x[0]) : 0.0;
    if (m == 2) return node_d(nd, nvalid > 0 ? x[0] : 0.0, nvalid > 1 ? x[stride] : 0.0);
    const int64_t p = (m >> 1) + (m & 1);
    const int64_t q = m - p;
    const int64_t vl = nvalid < p ? nvalid : p;
    const int64_t vr = nvalid > p ? nvalid - p : 0;
    double fp, fq;
    if (spawn > 0) {
#pragma omp task shared(fp) firstprivate(nd, x, stride, p, vl, spawn)
        fp = R_d(nd, x, stride, p, vl, spawn - 1);
        fq = R_d(nd, x + p * stride, stride, q, vr, spawn - 1);
#pragma omp taskwait
    } else {
        fp = R_d(nd, x, stride, p, vl, 0);
        fq = R_d(nd, x + p * stride, stride, q, vr, 0);
    }
    return node_d(nd, fp, fq);
}

static float R_s(node_t *nd, const float *x, int64_t stride, int64_t m, int64_t nvalid, int spawn)
{
    if (m == 1) return nvalid > 0 ? fabsf(x[0]) : 0.0f;
    if (m == 2) return node_s(nd, nvalid > 0 ? x[0] : 0.0f, nvalid > 1 ? x[stride] : 0.0f);
    const int64_t p = (m >> 1) + (m & 1);
    const int64_t q = m - p;
    const int64_t vl = nvalid < p ? nvalid : p;
    const int64_t vr = nvalid > p ? nvalid - p : 0;
    float fp, fq;
    if (spawn > 0) {
#pragma omp task shared(fp) firstprivate(nd, x, stride, p, vl, spawn)
        fp = R_s(nd, x, stride, p, vl, spawn - 1);
        fq = R_s(nd, x + p * stride, stride, q, vr, spawn - 1);
#pragma omp taskwait
    } else {
        fp = R_s(nd, x, stride, p, vl, 0);
        fq = R_s(nd, x + p * stride, stride, q, vr, 0);
    }
    return node_s(nd, fp, fq);
}

static int spawn_levels(int nthreads)
{
    int s = 0;
    while ((1 << s) < nthreads) ++s;
    return nthreads > 1 ? s + 3 : 0;
}

static double run_R_d(node_t *nd, const double *x, int64_t stride, int64_t m, int64_t nvalid, int nthreads)
{
    double r = 0.0;
    if (nthreads <= 1 || m < 4096) return R_d(nd, x, stride, m, nvalid, 0);
#pragma omp parallel num_threads(nthreads)
#pragma omp single
    r = R_d(nd, x, stride, m, nvalid, spawn_levels(nthreads));
    return r;
}

static float run_R_s(node_t *nd, const float *x, int64_t stride, int64_t m, int64_t nvalid, int nthreads)
{
    float r = 0.0f;
    if (nthreads <= 1 || m < 4096) return R_s(nd, x, stride, m, nvalid, 0);
#pragma omp parallel num_threads(nthreads)
#pragma omp single
    r = R_s(nd, x, stride, m, nvalid, spawn_levels(nthreads));
    return r;
}

/* ------------------------------------------------------------------ */
/* Entry points.  n >= 1 and finite inputs; the contract for n <= 0,   */
/* NaN and infinity is applied by the Python wrapper.                  */
/* node: 0 = cr_hypot (A), 1 = v1_hypot (H).                           */
/* ------------------------------------------------------------------ */
/* ------------------------------------------------------------------ */
/* Theorem 1's algorithm: one accumulator of squares updated by fma in  */
/* the working precision, then a square root (the linear-error         */
/* baseline the recursive algorithms are compared with, Sect. 2).      */
/* ------------------------------------------------------------------ */
double vnpo_dnrm_acc(int64_t n, const double *x)
{
    double g = 0.0;
    for (int64_t i = 0; i < n; ++i) g = fma(x[i], x[i], g);
    return sqrt(g);
}

float vnpo_snrm_acc(int64_t n, const float *x)
{
    float g = 0.0f;
    for (int64_t i = 0; i < n; ++i) g = fmaf(x[i], x[i], g);
    return sqrtf(g);
}

double vnpo_dnrmf_R(int64_t n, const double *x, int node, int nthreads)
{
    node_t nd = {node == 1 ? NODE_V1 : NODE_CR, 0.0, NULL, 0};
    return run_R_d(&nd, x, 1, n, n, nthreads);
}

float vnpo_snrmf_R(int64_t n, const float *x, int node, int nthreads)
{
    node_t nd = {node == 1 ? NODE_V1 : NODE_CR, 0.0, NULL, 0};
    return run_R_s(&nd, x, 1, n, n, nthreads);
}

static node_t pnode(double p, int is_single)
{
    node_t nd = {NODE_LP, p, NULL, 0};
    const double cutoff = is_single ? 0x1p24 : 0x1p53;
    if (p == 1.0)
        nd.kind = NODE_SUM;
    else if (isinf(p) || p >= cutoff)
        nd.kind = NODE_MAX;
    return nd;
}

double vnpo_dnrmp_R(int64_t n, const double *x, double p, int nthreads)
{
    node_t nd = pnode(p, 0);
    return run_R_d(&nd, x, 1, n, n, nthreads);
}

float vnpo_snrmp_R(int64_t n, const float *x, float p, int nthreads)
{
    node_t nd = pnode(p, 1);
    return run_R_s(&nd, x, 1, n, n, nthreads);
}

static int cmp_d(const void *a, const void *b)
{
    const double u = *(const double *)a, v = *(const double *)b;
    return (u > v) - (u < v);
}

static int cmp_f(const void *a, const void *b)
{
    const float u = *(const float *)a, v = *(const float *)b;
    return (u > v) - (u < v);
}

/* Z with P lanes (Listing 4, zero-padded tail), then A over the P lane values.
 * pnorm: 0 = Frobenius (v1_hypot lanes, cr_hypot finish); otherwise the p-node. */
static double Z_d(int64_t n, const double *x, int P, int sort, int nthreads, node_t lane, node_t fin)
{
    const int64_t m = (n + P - 1) / P;
    double *f = (double *)malloc(sizeof(double) * (size_t)P);
    for (int l = 0; l < P; ++l) {
        const int64_t nv = l < n ? (n - l + P - 1) / P : 0;
        f[l] = nv > 0 ? run_R_d(&lane, x + l, P, m, nv, nthreads) : 0.0;
    }
    if (sort) qsort(f, (size_t)P, sizeof(double), cmp_d);
    const double r = R_d(&fin, f, 1, P, P, 0);
    free(f);
    return r;
}

static float Z_s(int64_t n, const float *x, int P, int sort, int nthreads, node_t lane, node_t fin)
{
    const int64_t m = (n + P - 1) / P;
    float *f = (float *)malloc(sizeof(float) * (size_t)P);
    for (int l = 0; l < P; ++l) {
        const int64_t nv = l < n ? (n - l + P - 1) / P : 0;
        f[l] = nv > 0 ? run_R_s(&lane, x + l, P, m, nv, nthreads) : 0.0f;
    }
    if (sort) qsort(f, (size_t)P, sizeof(float), cmp_f);
    const float r = R_s(&fin, f, 1, P, P, 0);
    free(f);
    return r;
}

double vnpo_dnrmf_Z(int64_t n, const double *x, int P, int sort, int nthreads)
{
    node_t lane = {NODE_V1, 0.0, NULL, 0}, fin = {NODE_CR, 0.0, NULL, 0};
    return Z_d(n, x, P, sort, nthreads, lane, fin);
}

float vnpo_snrmf_Z(int64_t n, const float *x, int P, int sort, int nthreads)
{
    node_t lane = {NODE_V1, 0.0, NULL, 0}, fin = {NODE_CR, 0.0, NULL, 0};
    return Z_s(n, x, P, sort, nthreads, lane, fin);
}

double vnpo_dnrmp_Z(int64_t n, const double *x, double p, int P, int nthreads)
{
    node_t nd = pnode(p, 0);
    return Z_d(n, x, P, 0, nthreads, nd, nd);
}

float vnpo_snrmp_Z(int64_t n, const float *x, float p, int P, int nthreads)
{
    node_t nd = pnode(p, 1);
    return Z_s(n, x, P, 0, nthreads, nd, nd);
}

/* Tree shape of R (lanes == 0) or of Z's lanes + final A (lanes == P) over n leaves with
 * ids 1..n: log receives (left id, right id) per node in completion order, a node's own id
 * being 1000000 + its position in the log.  Returns the number of nodes. */
int64_t vnpo_trace(int64_t n, int lanes, int64_t *log)
{
    double *ids = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) ids[i] = (double)(i + 1);
    node_t nd = {NODE_TRACE, 0.0, log, 0};
    if (lanes <= 0) {
        (void)R_d(&nd, ids, 1, n, n, 0);
    } else {
        const int64_t m = (n + lanes - 1) / lanes;
        double *f = (double *)malloc(sizeof(double) * (size_t)lanes);
        for (int l = 0; l < lanes; ++l) {
            const int64_t nv = l < n ? (n - l + lanes - 1) / lanes : 0;
            f[l] = nv > 0 ? R_d(&nd, ids + l, lanes, m, nv, 0) : 0.0;
        }
        (void)R_d(&nd, f, 1, lanes, lanes, 0);
        free(f);
    }
    free(ids);
    return nd.nlog;
}

/* ------------------------------------------------------------------ */
/* Exact sum of squares: fixed-point superaccumulator, bit 0 = 2^-2148 */
/* ------------------------------------------------------------------ */
#define SA_LIMBS 72
#define SA_BIAS 2148

static void sa_add(uint64_t *acc, const uint64_t *w, int k, int nw)
{
    unsigned __int128 c = 0;
    int i = 0;
    for (; i < nw; ++i) {
        c += (unsigned __int128)acc[k + i] + w[i];
        acc[k + i] = (uint64_t)c;
        c >>= 64;
    }
    for (i = k + nw; c && i < SA_LIMBS; ++i) {
        c += acc[i];
        acc[i] = (uint64_t)c;
        c >>= 64;
    }
}

static void sa_add_sq(uint64_t *acc, double v)
{
    if (v == 0.0) return;
    uint64_t V;
    int e;
    split_d(fabs(v), &V, &e); /* |v| = V 2^e, e >= -1074 */
    const unsigned __int128 p = (unsigned __int128)V * V;
    const int sh = 2 * e + SA_BIAS;
    const int k = sh / 64, off = sh % 64;
    uint64_t w[3];
    w[0] = (uint64_t)(p << off);
    w[1] = (uint64_t)((p << off) >> 64);
    w[2] = off ? (uint64_t)(p >> (128 - off)) : 0;
    sa_add(acc, w, k, 3);
}

int vnpo_sa_limbs(void) { return SA_LIMBS; }
int vnpo_sa_bias(void) { return SA_BIAS; }

/* out[SA_LIMBS]: sum of x_i^2 as an integer multiple of 2^-2148 (little-endian limbs).
 * x holds n finite values; is_single selects float input. */
int vnpo_sumsq_exact(int64_t n, const void *x, int is_single, uint64_t *out, int nthreads)
{
    memset(out, 0, sizeof(uint64_t) * SA_LIMBS);
    if (nthreads < 1) nthreads = 1;
    uint64_t *parts = (uint64_t *)calloc((size_t)nthreads * SA_LIMBS, sizeof(uint64_t));
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int t = 0; t < nthreads; ++t) {
        const int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
        uint64_t *acc = parts + (size_t)t * SA_LIMBS;
        for (int64_t i = lo; i < hi; ++i)
            sa_add_sq(acc, is_single ? (double)((const float *)x)[i] : ((const double *)x)[i]);
    }
    for (int t = 0; t < nthreads; ++t) sa_add(out, parts + (size_t)t * SA_LIMBS, 0, SA_LIMBS);
    free(parts);
    return 0;
}

/* ------------------------------------------------------------------ */
/* binary128 p-norm reference: (sum |x_i|^p)^(1/p), error ~1e-25       */
/* ------------------------------------------------------------------ */
static __float128 powabs_q(__float128 a, __float128 p, int twop_int)
{
    if (a == 0) return 0;
    if (twop_int > 0 && twop_int <= 64) { /* p = k/2: a^floor(p) * sqrt(a)^(2p mod 2) */
        __float128 r = 1;
        for (int i = 0; i < twop_int / 2; ++i) r *= a;
        if (twop_int & 1) r *= sqrtq(a);
        return r;
    }
    return powq(a, p);
}

/* Returns the binary128 value as hi + lo doubles. x: n finite values. */
void vnpo_pnorm_quad(int64_t n, const void *x, int is_single, double p, int nthreads, double *hi, double *lo)
{
    double amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double v = fabs(is_single ? (double)((const float *)x)[i] : ((const double *)x)[i]);
        if (v > amax) amax = v;
    }
    if (amax == 0.0 || n <= 0) {
        *hi = 0.0;
        *lo = 0.0;
        return;
    }
    int E;
    frexp(amax, &E);
    const __float128 scale = ldexpq(1.0Q, -E), pq = p;
    int twop = -1;
    if (p * 2 == floor(p * 2) && p * 2 <= 64) twop = (int)(p * 2);
    if (nthreads < 1) nthreads = 1;
    __float128 *part = (__float128 *)calloc((size_t)nthreads, sizeof(__float128));
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int t = 0; t < nthreads; ++t) {
        const int64_t a = n * t / nthreads, b = n * (t + 1) / nthreads;
        __float128 s = 0;
        for (int64_t i = a; i < b; ++i) {
            const double v = fabs(is_single ? (double)((const float *)x)[i] : ((const double *)x)[i]);
            s += powabs_q((__float128)v * scale, pq, twop);
        }
        part[t] = s;
    }
    __float128 s = 0;
    for (int t = 0; t < nthreads; ++t) s += part[t];
    free(part);
    const __float128 r = (p == 2.0 ? sqrtq(s) : powq(s, 1.0Q / pq)) / scale;
    *hi = (double)r;
    *lo = (double)(r - (__float128)*hi);
}

/* The p-norm recursion R with the Listing 5 node evaluated in binary128, using the
 * method's own rounded exponents half_p = RN(p/2) and inv_p = RN(1/p) (Sect. 4 rounds
 * them once): node(a, b) = M (1 + (m/M)^(2 half_p))^inv_p.  This is the paper's "exact"
 * reference for p-norms (Sect. 5: the recursion followed at high precision), which keeps
 * the effect of rounding 1/p and removes only the rounding of the node evaluations.
 * Operands are scaled by a power of two so nothing over- or underflows; NaN/Inf follow
 * the library contract (NaN dominates, else Inf). */
static __float128 lpq_node(__float128 a, __float128 b, __float128 hp, __float128 ip)
{
    const __float128 M = a > b ? a : b, m = a > b ? b : a;
    if (M == 0) return 0;
    const __float128 S = powq(m / M, hp);
    return M * powq(1 + S * S, ip);
}

/* depth < par: the two halves are evaluated as parallel tasks (same tree, any thread count) */
static __float128 lpq_rec(const void *x, int is_single, int64_t lo, int64_t n, __float128 scale, __float128 hp,
                          __float128 ip, int par)
{
    if (n == 1) {
        const double v = is_single ? (double)((const float *)x)[lo] : ((const double *)x)[lo];
        return fabsq((__float128)v * scale);
    }
    const int64_t left = (n + 1) / 2;
    __float128 a, b;
    if (par > 0 && n > 4096) {
#pragma omp task shared(a)
        a = lpq_rec(x, is_single, lo, left, scale, hp, ip, par - 1);
        b = lpq_rec(x, is_single, lo + left, n - left, scale, hp, ip, par - 1);
#pragma omp taskwait
    } else {
        a = lpq_rec(x, is_single, lo, left, scale, hp, ip, 0);
        b = lpq_rec(x, is_single, lo + left, n - left, scale, hp, ip, 0);
    }
    return lpq_node(a, b, hp, ip);
}

void vnpo_pnorm_R_quad(int64_t n, const void *x, int is_single, double half_p, double inv_p, int nthreads,
                       double *hi, double *lo)
{
    double amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double v = fabs(is_single ? (double)((const float *)x)[i] : ((const double *)x)[i]);
        if (v > amax) amax = v;
    }
    *hi = 0.0;
    *lo = 0.0;
    if (amax == 0.0 || n <= 0) return;
    int E;
    frexp(amax, &E);
    const __float128 scale = ldexpq(1.0Q, -E);
    if (nthreads < 1) nthreads = 1;
    int par = 0;
    while ((1 << par) < 2 * nthreads && par < 12) ++par;
    __float128 r = 0;
#pragma omp parallel num_threads(nthreads)
#pragma omp single
    r = lpq_rec(x, is_single, 0, n, scale, (__float128)half_p, (__float128)inv_p, par);
    r /= scale;
    *hi = (double)r;
    *lo = (double)(r - (__float128)*hi);
}

/* powq at binary128, for tests of the pow evaluation (returns hi + lo doubles). */
void vnpo_powq2(double x, double y, double *hi, double *lo)
{
    const __float128 r = powq((__float128)x, (__float128)y);
    *hi = (double)r;
    *lo = (double)(r - (__float128)*hi);
}
