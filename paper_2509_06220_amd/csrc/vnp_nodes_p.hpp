// p-norm node (Novakovic, arXiv 2509.06220, Sect. 4).
//
// For partial p-norms a, b >= 0 with M = max, m = min:
//     node(a, b) = M C,  C = Z^(1/p),  Z = fma(S, S, 1),  S = Q^(p/2),  Q = m / M
// (Eq. (sp), (qp); Listing 5 forms 1 + Q^p as fma(S, S, 1) the same way).  p/2 and 1/p
// are rounded once and hoisted out of the recursion (Sect. 4); binary32 uses RN32(p/2)
// and RN32(1/p) and evaluates the node in binary64, rounding the node value to binary32.
//
// The two powers are evaluated as exponentials of logarithms, on the ranges the node
// produces, without the general-purpose library routines:
//   log2 Q = (e_m - e_M) + log2(r),  r = f_m / f_M  (frexp parts; r moved into
//            [sqrt(1/2), sqrt(2)] by a factor 2),
//   S = 2^((p/2) log2 Q),   C = 2^((1/p) log2 Z),  Z in [1, 2].
// log2 near 1 uses the series 2 atanh(s) / ln 2 in s = (r - 1) / (r + 1), |s| <= 0.172
// (terms to s^21); 2^y splits y = k + f, |f| <= 1/2, and sums e^(f ln 2) to the 13th
// power before scaling by 2^k.  Both keep an absolute error of a few ulps of 1 in
// their ranges.  An absolute error d in log2 Q changes C by at most about
// (ln 2 / 2) d relatively, whatever p is (the error of S^2 is weighted by
// S^2 / (p (1 + S^2)) in C), so the node's relative error stays within a few eps.
//
// Special operands: M is taken as the larger bit pattern, so a NaN operand becomes M and
// the node returns NaN; an infinite M (and no NaN) returns +inf; m = 0 returns M.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vnp_internal.hpp"

namespace vnp {

// 1 / r for r in [1/2, 4) (two Newton steps from the hardware reciprocal estimate),
// then q = n / r rounded with one correction step.
__device__ __forceinline__ double div_unit(double n, double r)
{
    double y = __builtin_amdgcn_rcp(r);
    double e = __builtin_fma(-r, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-r, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = n * y;
    return __builtin_fma(__builtin_fma(-r, q, n), y, q);
}

// log2(r) for r in [sqrt(1/2), sqrt(2)].
__device__ __forceinline__ double log2_near1(double r)
{
    constexpr double C1 = 0x1.71547652b82fep+1;  // 2 / ln 2
    const double s = div_unit(r - 1.0, r + 1.0);  // r - 1 is exact here
    const double s2 = s * s;
    double t = C1 / 21.0;
    t = __builtin_fma(t, s2, C1 / 19.0);
    t = __builtin_fma(t, s2, C1 / 17.0);
    t = __builtin_fma(t, s2, C1 / 15.0);
    t = __builtin_fma(t, s2, C1 / 13.0);
    t = __builtin_fma(t, s2, C1 / 11.0);
    t = __builtin_fma(t, s2, C1 / 9.0);
    t = __builtin_fma(t, s2, C1 / 7.0);
    t = __builtin_fma(t, s2, C1 / 5.0);
    t = __builtin_fma(t, s2, C1 / 3.0);
    return __builtin_fma(s * s2, t, s * C1);
}

// 2^y (y clamped to [-2100, 2100]: 0 and +inf beyond the binary64 range).
__device__ __forceinline__ double exp2_any(double y)
{
    constexpr double LN2 = 0x1.62e42fefa39efp-1;
    y = __builtin_fmin(__builtin_fmax(y, -2100.0), 2100.0);
    const double k = __builtin_rint(y);
    const double x = (y - k) * LN2;  // y - k is exact, |x| <= 0.347
    double t = 1.0 / 6227020800.0;   // 1/13!
    t = __builtin_fma(t, x, 1.0 / 479001600.0);
    t = __builtin_fma(t, x, 1.0 / 39916800.0);
    t = __builtin_fma(t, x, 1.0 / 3628800.0);
    t = __builtin_fma(t, x, 1.0 / 362880.0);
    t = __builtin_fma(t, x, 1.0 / 40320.0);
    t = __builtin_fma(t, x, 1.0 / 5040.0);
    t = __builtin_fma(t, x, 1.0 / 720.0);
    t = __builtin_fma(t, x, 1.0 / 120.0);
    t = __builtin_fma(t, x, 1.0 / 24.0);
    t = __builtin_fma(t, x, 1.0 / 6.0);
    t = __builtin_fma(t, x, 0.5);
    t = __builtin_fma(t, x, 1.0);
    t = __builtin_fma(t, x, 1.0);
    return __builtin_amdgcn_ldexp(t, (int)k);
}

__device__ __forceinline__ double lp_core(double a, double b, double half_p, double inv_p)
{
    constexpr double SQRT_HALF = 0x1.6a09e667f3bcdp-1;
    const uint64_t ia = (uint64_t)__double_as_longlong(a), ib = (uint64_t)__double_as_longlong(b);
    const double M = __longlong_as_double((long long)(ia > ib ? ia : ib));
    const double m = __longlong_as_double((long long)(ia > ib ? ib : ia));
    // log2(m / M) = (e_m - e_M) + log2(f_m / f_M), f in [1/2, 1)
    const double fM = __builtin_amdgcn_frexp_mant(M), fm = __builtin_amdgcn_frexp_mant(m);
    int k = __builtin_amdgcn_frexp_exp(m) - __builtin_amdgcn_frexp_exp(M);
    double r = div_unit(fm, fM);  // in (1/2, 2)
    const bool lo = r < SQRT_HALF, hi = r > 2.0 * SQRT_HALF;
    r = lo ? 2.0 * r : (hi ? 0.5 * r : r);
    k += lo ? -1 : (hi ? 1 : 0);
    const double lq = (double)k + log2_near1(r);
    const double S = exp2_any(half_p * lq);
    const double Z = __builtin_fma(S, S, 1.0);  // in [1, 2]
    const bool zh = Z > 2.0 * SQRT_HALF;
    const double lz = (zh ? 1.0 : 0.0) + log2_near1(zh ? 0.5 * Z : Z);
    const double C = exp2_any(inv_p * lz);
    const bool regular = m > 0.0 && M < __builtin_inf();  // also false for a NaN M
    return regular ? M * C : M;
}

template <typename T>
struct LpNode;

template <>
struct LpNode<double> {
    using T = double;
    double half_p, inv_p;
    __device__ double leaf(double a, double b) const
    {
        return lp_core(__builtin_fabs(a), __builtin_fabs(b), half_p, inv_p);
    }
    __device__ double node(double a, double b) const { return lp_core(a, b, half_p, inv_p); }
    __device__ double finish(double r) const { return r; }
};

template <>
struct LpNode<float> {
    using T = float;
    double half_p, inv_p;
    __device__ float leaf(float a, float b) const
    {
        return (float)lp_core((double)__builtin_fabsf(a), (double)__builtin_fabsf(b), half_p, inv_p);
    }
    __device__ float node(float a, float b) const { return (float)lp_core((double)a, (double)b, half_p, inv_p); }
    __device__ float finish(float r) const { return r; }
};

template <typename T>
inline LpNode<T> make_lp_node(T p);

template <>
inline LpNode<double> make_lp_node<double>(double p)
{
    return LpNode<double>{p * 0.5, 1.0 / p};
}

template <>
inline LpNode<float> make_lp_node<float>(float p)
{
    const float hp = p * 0.5f, ip = 1.0f / p;
    return LpNode<float>{(double)hp, (double)ip};
}

}  // namespace vnp
