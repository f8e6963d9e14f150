// p-norm node (Novakovic, arXiv 2509.06220, Sect. 4).
//
// For partial p-norms a, b >= 0 with M = max, m = min:
//     node(a, b) = M C,  C = Z^(1/p),  Z = fma(S, S, 1),  S = Q^(p/2),  Q = m / M
// (Eq. (sp), (qp); Listing 5 forms 1 + Q^p as fma(S, S, 1) the same way).  p/2 and 1/p
// are rounded once and hoisted out of the recursion (Sect. 4); binary32 uses RN32(p/2)
// and RN32(1/p) and evaluates the node in binary64, rounding the node value to binary32.
//
// The two powers are evaluated on the ranges the node produces, without the
// general-purpose library routines and without a division:
//   S = 2^((p/2) log2 Q),  log2 Q = (e_m - e_M) + log2 f_m - log2 f_M  (frexp parts f in
//   [1/2, 1), exponents e).  log2 f: the top LP_TAB_BITS fraction bits of f pick c_j ~ 1/f
//   and l_j = log2(2 / c_j) from a table in LDS; log2 f = (l_j - 1) + log2(1 + t) with
//   t = fma(f, c_j, -1), |t| <= 1.01 * 2^-8, and log2(1 + t) = t g(t), g of degree 5.
//   2^y splits y = k + f, |f| <= 1/2, evaluates 2^f by a degree-11 polynomial in f and
//   scales by 2^k.
//   C = Z^a, a = RN(1/p), Z in [1, 2]: with a = a' 2^s, a' <= 2, C = (Z^a')^(2^s).  The top
//   LP_TAB_BITS fraction bits of Z pick c'_j = RN(2^7 / (2^7 + j)) (the reciprocal of the
//   interval's left end), R_j = (1/c'_j)^a' and rho_j = R_j - 1 (both rounded from an
//   extended-precision value; one device table per (device, p), built and uploaded by
//   make_lp_node on first use); with t = fma(Z, c'_j, -1) in
//   [0, 2^-7), Z^a' = R_j (1 + t)^a' and (1 + t)^a' = 1 + u, u = t (b_1 + b_2 t + ... +
//   b_7 t^6) with the binomial coefficients b_k of a'.  Then Z^a' = 1 + fma(u, R_j, rho_j):
//   Z = 1 gives exactly 1, and R_j's rounding touches only the small product.
// (Coefficients and tables: Chebyshev fits and 60-digit values written by lp_coeffs.py.)
//
// Errors: the log2 table values carry 2^-54 absolute, the polynomials 2^-61.7
// (log2(1 + t), absolute) and 2^-55.5 (2^f, relative); the binomial series omits less than
// 2^-61.9.  An absolute error d in log2 Q changes C by at most (ln 2 / 2) d relatively,
// whatever p is (the error of S^2 is weighted by S^2 / (p (1 + S^2)) in C); each squaring
// doubles the relative error of Z^a', so p < 1/2 costs about 2^s ulps more.
//
// Special operands: M is taken as the larger bit pattern, so a NaN operand becomes M and
// the node returns NaN; an infinite M (and no NaN) returns +inf; m = 0 returns M.  Their
// intermediate values are finite or NaN and are discarded by the final select.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "vnp_internal.hpp"
#include "vnp_lp_table.hpp"

namespace vnp {

constexpr int LP_TAB_N = 1 << LP_TAB_BITS;

// The tables in LDS: one copy per block, filled by lp_table_fill at kernel entry.
__device__ __forceinline__ double2 *lp_table()
{
    __shared__ double2 tab[LP_TAB_N];
    return tab;
}
// c'_j, R_j, rho_j, then b_1 .. b_7 (and a zero), then the 2^f coefficients of f^11 .. f^1,
// then the log2(1 + t) / t coefficients of t^5 .. t^0
constexpr int LP_EXP_OFF = 3 * LP_TAB_N + 8;
constexpr int LP_LOG_OFF = LP_EXP_OFF + 11;
__device__ __forceinline__ double *lp_ptable()
{
    __shared__ double tab[LP_LOG_OFF + 6];
    return tab;
}

// Every thread of the block calls this before the first node evaluation.  rr: the per-p
// device table (R_0 .. R_127, rho_0 .. rho_127); b: the binomial coefficients.
__device__ __forceinline__ void lp_table_fill(const double *rr, const double *b)
{
    double2 *tab = lp_table();
    double *pt = lp_ptable();
    for (int i = threadIdx.x; i < LP_TAB_N; i += blockDim.x) {
        tab[i] = make_double2(lp_tab_src[i][0], lp_tab_src[i][1]);
        pt[i] = lp_ptab_src[i];
        pt[LP_TAB_N + i] = rr[i];
        pt[2 * LP_TAB_N + i] = rr[LP_TAB_N + i];
    }
    if (threadIdx.x < 8) pt[3 * LP_TAB_N + threadIdx.x] = b[threadIdx.x];
    if (threadIdx.x < 11) {
        // 2^f on |f| <= 1/2, degree 11 (Chebyshev fit, relative error 2^-55.5), f^11 first
        constexpr double E[11] = {0x1.e9ec1fcb69a7fp-32, 0x1.e6228acd1c6e5p-28, 0x1.b524ebd13a55fp-24,
                                  0x1.62bfc2c86d700p-20, 0x1.ffcbfc6da6ed1p-17, 0x1.430913112c61bp-13,
                                  0x1.5d87fe78a3f9cp-10, 0x1.3b2ab6fb9f1a5p-7,  0x1.c6b08d704a0c6p-5,
                                  0x1.ebfbdff82c5aep-3,  0x1.62e42fefa39efp-1};
        pt[LP_EXP_OFF + threadIdx.x] = E[threadIdx.x];
    }
    if (threadIdx.x < 6) {
        // log2(1 + t) = t g(t), |t| <= 1.01 * 2^-8, g of degree 5 (absolute error 2^-61.7)
        constexpr double G[6] = {-0x1.ec72d2e6fb6e9p-3, 0x1.277807fe93552p-2, -0x1.715476524c17ep-2,
                                 0x1.ec709dc324b6cp-2,  -0x1.71547652b82fep-1, 0x1.71547652b82fep+0};
        pt[LP_LOG_OFF + threadIdx.x] = G[threadIdx.x];
    }
    __syncthreads();
}

// log2 f - (l_j - 1) for f in [1/2, 1), and l_j through `l`.
__device__ __forceinline__ double log2_part(double f, double &l)
{
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(f) >> 32);
    const double2 e = lp_table()[(hi >> (20 - LP_TAB_BITS)) & (LP_TAB_N - 1)];
    l = e.y;
    const double t = __builtin_fma(f, e.x, -1.0);
    const double *G = lp_ptable() + LP_LOG_OFF;  // the same address in every lane (see exp2_poly)
    double g = G[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) g = __builtin_fma(g, t, G[i]);
    return t * g;
}

// 2^y for finite y in [-2100, 2100] (0 and +inf beyond the binary64 range).  The
// coefficients are read from LDS (lp_table_fill): as immediates they exhaust the scalar
// registers of the streaming kernel, and the compiler then rebuilds each 64-bit
// coefficient with two vector moves at every use (about a fifth of the node's VALU
// instructions); from LDS they are loaded once into vector registers.
__device__ __forceinline__ double exp2_poly(double y)
{
    const double k = __builtin_rint(y);
    const double f = y - k;  // exact, |f| <= 1/2
    const double *E = lp_ptable() + LP_EXP_OFF;  // the same address in every lane
    double t = E[0];
#pragma unroll
    for (int i = 1; i < 11; ++i) t = __builtin_fma(t, f, E[i]);
    t = __builtin_fma(t, f, 1.0);
    return __builtin_amdgcn_ldexp(t, (int)k);
}

// Z^a for Z in [1, 2] (a = a' 2^s, see above); b: the binomial coefficients b_1 .. b_7.
__device__ __forceinline__ double pow_z(double Z, int sq, const double *b)
{
    const double Zc = __builtin_fmin(Z, 0x1.fffffffffffffp0);  // Z = 2 as its predecessor: within Z's rounding
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(Zc) >> 32);
    const uint32_t j = (hi >> (20 - LP_TAB_BITS)) & (LP_TAB_N - 1);
    const double *pt = lp_ptable();
    const double t = __builtin_fma(Zc, pt[j], -1.0);  // in [0, 2^-7)
    double q = b[6];
    q = __builtin_fma(q, t, b[5]);
    q = __builtin_fma(q, t, b[4]);
    q = __builtin_fma(q, t, b[3]);
    q = __builtin_fma(q, t, b[2]);
    q = __builtin_fma(q, t, b[1]);
    q = __builtin_fma(q, t, b[0]);
    double C = 1.0 + __builtin_fma(t * q, pt[LP_TAB_N + j], pt[2 * LP_TAB_N + j]);
    for (int i = 0; i < sq; ++i) C *= C;
    return C;
}

__device__ __forceinline__ double lp_core(double a, double b, double half_p, int sq, const double *bc)
{
    const uint64_t ia = (uint64_t)__double_as_longlong(a), ib = (uint64_t)__double_as_longlong(b);
    const double M = __longlong_as_double((long long)(ia > ib ? ia : ib));
    const double m = __longlong_as_double((long long)(ia > ib ? ib : ia));
    double lM, lm;
    const double pM = log2_part(__builtin_amdgcn_frexp_mant(M), lM);
    const double pm = log2_part(__builtin_amdgcn_frexp_mant(m), lm);
    const int e = __builtin_amdgcn_frexp_exp(m) - __builtin_amdgcn_frexp_exp(M);
    const double lq = (double)e + ((lm - lM) + (pm - pM));  // log2 Q <= 0
    const double S = exp2_poly(__builtin_fmax(half_p * lq, -2100.0));
    const double Z = __builtin_fma(S, S, 1.0);  // in [1, 2]
    const double C = pow_z(Z, sq, bc);
    const bool regular = m > 0.0 && M < __builtin_inf();  // also false for a NaN M
    return regular ? M * C : M;
}

// The evaluation part of the p node: p/2 and s, with every table read from LDS.  Device
// functions that are not inlined receive this part only (node_eval).
template <typename T>
struct LpEval;

__device__ __forceinline__ const double *lp_binom_lds() { return lp_ptable() + 3 * LP_TAB_N; }

template <>
struct LpEval<double> {
    using T = double;
    double half_p;  // RN(p/2)
    int sq;         // s: C = (Z^a')^(2^s)
    __device__ double leaf(double a, double b) const
    {
        return lp_core(__builtin_fabs(a), __builtin_fabs(b), half_p, sq, lp_binom_lds());
    }
    __device__ double node(double a, double b) const { return lp_core(a, b, half_p, sq, lp_binom_lds()); }
    __device__ double finish(double r) const { return r; }
};

template <>
struct LpEval<float> {
    using T = float;
    double half_p;  // RN32(p/2)
    int sq;
    __device__ float leaf(float a, float b) const
    {
        return (float)lp_core((double)__builtin_fabsf(a), (double)__builtin_fabsf(b), half_p, sq, lp_binom_lds());
    }
    __device__ float node(float a, float b) const
    {
        return (float)lp_core((double)a, (double)b, half_p, sq, lp_binom_lds());
    }
    __device__ float finish(float r) const { return r; }
};

// The p node as the kernels receive it: the evaluation part, the binomial coefficients
// and the device table of R_j and rho_j (small kernel arguments: a large argument block
// costs several microseconds of host time per launch).  Its own evaluation (inlined into
// the kernel body) takes the coefficients from the kernel arguments, which stay in
// scalar registers.
template <typename T>
struct LpNode : LpEval<T> {
    double b[8];       // binomial coefficients b_1 .. b_7 of a' (b[7] = 0)
    const double *rr;  // device: R_0 .. R_127, then rho_0 .. rho_127
    __device__ T leaf(T a, T b_) const
    {
        return (T)lp_core((double)__builtin_fabs((double)a), (double)__builtin_fabs((double)b_), this->half_p,
                          this->sq, b);
    }
    __device__ T node(T a, T b_) const { return (T)lp_core((double)a, (double)b_, this->half_p, this->sq, b); }
    __device__ T finish(T r) const { return r; }
};

template <typename T>
__host__ __device__ inline LpEval<T> node_eval(const LpNode<T> &nd)
{
    return LpEval<T>{nd.half_p, nd.sq};
}

// Kernel-entry hook of the nodes: the p node fills its tables (the other nodes have
// nothing to set up).
template <typename T>
__device__ __forceinline__ void node_prologue(const LpNode<T> &nd)
{
    lp_table_fill(nd.rr, nd.b);
}

// Per-(device, p) constants of the p node, built on first use and kept until
// release_lp_tables (host side).
struct LpEntry {
    int sq;
    double b[8];
    double *rr;  // device table
};

struct LpCache {
    std::mutex mu;
    std::map<std::pair<int, std::pair<uint64_t, uint64_t>>, LpEntry> map;
};

inline LpCache &lp_cache()
{
    static LpCache c;
    return c;
}

// The node for half_p = RN(p/2) and a = RN(1/p) on the current device.  The first use of
// a (device, p) builds the table in extended precision and uploads it (a synchronous
// copy: outside graph capture); returns 0 or a HIP error code.
template <typename T>
inline int lp_node(double half_p, double a, LpNode<T> *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    uint64_t kh, ka;
    memcpy(&kh, &half_p, 8);
    memcpy(&ka, &a, 8);
    LpCache &c = lp_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    const auto key = std::make_pair(dev, std::make_pair(kh, ka));
    auto it = c.map.find(key);
    if (it == c.map.end()) {
        // a = RN(1/p) must be finite (the entry points reject a smaller p); the halvings
        // below then end after at most 1024 steps
        if (!(a >= 0.0 && a <= 0x1.fffffffffffffp1023)) return (int)hipErrorInvalidValue;
        LpEntry en{};
        double ap = a;
        while (ap > 2.0) {  // exact halvings
            ap = std::ldexp(ap, -1);
            ++en.sq;
        }
        long double bk = 1.0L;
        for (int i = 1; i <= 7; ++i) {
            bk = bk * ((long double)ap - (i - 1)) / i;
            en.b[i - 1] = (double)bk;
        }
        en.b[7] = 0.0;
        double h[2 * LP_TAB_N];
        for (int j = 0; j < LP_TAB_N; ++j) {
            const long double r = std::pow(1.0L / (long double)lp_ptab_host[j], (long double)ap);
            h[j] = (double)r;
            h[LP_TAB_N + j] = (double)(r - 1.0L);
        }
        e = hipMalloc(reinterpret_cast<void **>(&en.rr), sizeof(h));
        if (e != hipSuccess) return (int)e;
        e = hipMemcpy(en.rr, h, sizeof(h), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(en.rr);
            return (int)e;
        }
        it = c.map.emplace(key, en).first;
    }
    out->half_p = half_p;
    out->sq = it->second.sq;
    memcpy(out->b, it->second.b, sizeof(out->b));
    out->rr = it->second.rr;
    return 0;
}

template <typename T>
inline int make_lp_node(T p, LpNode<T> *out);

template <>
inline int make_lp_node<double>(double p, LpNode<double> *out)
{
    return lp_node<double>(p * 0.5, 1.0 / p, out);
}

template <>
inline int make_lp_node<float>(float p, LpNode<float> *out)
{
    const float hp = p * 0.5f, ip = 1.0f / p;
    return lp_node<float>((double)hp, (double)ip, out);
}

// Frees the current device's p-node tables (no work using them may be pending).
inline int release_lp_tables()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    LpCache &c = lp_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto it = c.map.begin(); it != c.map.end();) {
        if (it->first.first == dev) {
            (void)hipFree(it->second.rr);
            it = c.map.erase(it);
        } else {
            ++it;
        }
    }
    return 0;
}

}  // namespace vnp
