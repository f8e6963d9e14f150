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
//   log2 Q = (e_m - e_M) + log2(f_m / f_M)  (frexp parts; f_m moved by a factor 2 so
//            the ratio lies in [sqrt(1/2), sqrt(2)]; s = (f_m - f_M) / (f_m + f_M)),
//   S = 2^((p/2) log2 Q),   C = 2^((1/p) log2 Z),  Z in [1, 2].
// log2 near 1 is s g(s^2) with s = (r - 1) / (r + 1), |s| <= 0.172, g a degree-7
// polynomial for 2 atanh(s) / (s ln 2); 2^y splits y = k + f, |f| <= 1/2, and evaluates
// e^(f ln 2) by a degree-11 polynomial before scaling by 2^k (coefficients: Chebyshev
// fits printed by lp_coeffs.py).  Both keep an absolute error of a few ulps of 1 in their
// ranges.  An absolute error d in log2 Q changes C by at most about
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

// q = n / d (d in [1, 4)): two Newton steps from the hardware reciprocal estimate, then one
// correction step.
__device__ __forceinline__ double div_near1(double n, double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-d, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = n * y;
    return __builtin_fma(__builtin_fma(-d, q, n), y, q);
}

// log2(r) = s g(s^2) for s = (r - 1) / (r + 1), r in [sqrt(1/2), sqrt(2)] (|s| <= 0.1716):
// g(u) = 2 atanh(sqrt u) / (sqrt u ln 2), a degree-7 polynomial in u (Chebyshev fit,
// relative error 1.4e-17; lp_coeffs.py prints the coefficients).
__device__ __forceinline__ double log2_of_s(double s)
{
    const double u = s * s;
    double t = 0x1.b592d3c48c41cp-3;
    t = __builtin_fma(t, u, 0x1.c46e1440404d7p-3);
    t = __builtin_fma(t, u, 0x1.0ca160627dbfcp-2);
    t = __builtin_fma(t, u, 0x1.484afb7a67652p-2);
    t = __builtin_fma(t, u, 0x1.a61762d693934p-2);
    t = __builtin_fma(t, u, 0x1.2776c50ee39dcp-1);
    t = __builtin_fma(t, u, 0x1.ec709dc3a047dp-1);
    return __builtin_fma(s * u, t, s * 0x1.71547652b82fep+1);
}

// 2^y (y clamped to [-2100, 2100]: 0 and +inf beyond the binary64 range): y = k + f,
// |f| <= 1/2, e^(f ln 2) by a degree-11 polynomial (Chebyshev fit, relative error
// 1.7e-17), then scaled by 2^k.
__device__ __forceinline__ double exp2_any(double y)
{
    constexpr double LN2 = 0x1.62e42fefa39efp-1;
    y = __builtin_fmin(__builtin_fmax(y, -2100.0), 2100.0);
    const double k = __builtin_rint(y);
    const double x = (y - k) * LN2;  // y - k is exact, |x| <= 0.347
    double t = 0x1.af631d0059becp-26;
    t = __builtin_fma(t, x, 0x1.28b4057f44145p-22);
    t = __builtin_fma(t, x, 0x1.71ddf5749d126p-19);
    t = __builtin_fma(t, x, 0x1.a01991ac8730ap-16);
    t = __builtin_fma(t, x, 0x1.a01a01b14378fp-13);
    t = __builtin_fma(t, x, 0x1.6c16c187fbe02p-10);
    t = __builtin_fma(t, x, 0x1.111111110f225p-7);
    t = __builtin_fma(t, x, 0x1.555555554f0cfp-5);
    t = __builtin_fma(t, x, 0x1.555555555555ap-3);
    t = __builtin_fma(t, x, 0x1.0000000000011p-1);
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
    // log2(m / M) = (e_m - e_M) + log2(f_m / f_M), f in [1/2, 1); f_m is moved by an exact
    // factor 2 so that f_m / f_M lies in [sqrt(1/2), sqrt(2)], where f_m - f_M is exact
    const double fM = __builtin_amdgcn_frexp_mant(M);
    double fm = __builtin_amdgcn_frexp_mant(m);
    int k = __builtin_amdgcn_frexp_exp(m) - __builtin_amdgcn_frexp_exp(M);
    const bool lo = fm < SQRT_HALF * fM, hi = fm > (2.0 * SQRT_HALF) * fM;
    fm = lo ? 2.0 * fm : (hi ? 0.5 * fm : fm);
    k += lo ? -1 : (hi ? 1 : 0);
    const double lq = (double)k + log2_of_s(div_near1(fm - fM, fm + fM));
    const double S = exp2_any(half_p * lq);
    const double Z = __builtin_fma(S, S, 1.0);  // in [1, 2]
    const bool zh = Z > 2.0 * SQRT_HALF;
    const double Zr = zh ? 0.5 * Z : Z;
    const double lz = (zh ? 1.0 : 0.0) + log2_of_s(div_near1(Zr - 1.0, Zr + 1.0));
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
