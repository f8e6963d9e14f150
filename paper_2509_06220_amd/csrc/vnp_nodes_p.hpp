// p-norm node (Novakovic, arXiv 2509.06220, Sect. 4).
//
// For partial p-norms a, b >= 0 with M = max, m = min:
//     node(a, b) = M (1 + Q^p)^(1/p),  Q = max(m / M, 0)          (Eq. (sp))
// with 1 + Q^p formed as Z = fma(S, S, 1), S = Q^(p/2)              (Eq. (qp), Listing 5).
// The powers are evaluated as
//     S = exp((p/2) log Q)                   (Q in [0, 1])
//     C = 1 + expm1((1/p) log1p(Z - 1))      (Z in [1, 2]; Z - 1 is exact)
// with the device math library's log, exp, log1p and expm1 (each within about one ulp),
// so C carries about one ulp of error and S's error reaches C damped by
// 2 S^2 / (p (1 + S^2)).  p/2 and 1/p are rounded once and hoisted (Sect. 4: "defined
// once, at the highest level of the recursion"); binary32 uses RN32(p/2) and RN32(1/p)
// and evaluates the node in binary64, rounding the node value to binary32.
//
// M is taken as the larger bit pattern, so a NaN operand becomes M and the node returns
// NaN; an infinite M (and no NaN) gives Q = 0 and the node returns +inf.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vnp_internal.hpp"

namespace vnp {

__device__ __forceinline__ double lp_core(double a, double b, double half_p, double inv_p)
{
    const uint64_t ia = (uint64_t)__double_as_longlong(a), ib = (uint64_t)__double_as_longlong(b);
    const double M = __longlong_as_double((long long)(ia > ib ? ia : ib));
    const double m = __longlong_as_double((long long)(ia > ib ? ib : ia));
    const double q = m / M;
    const double Q = __builtin_fmax(q, 0.0);  // 0/0 and inf/inf give NaN -> 0
    const double S = exp(half_p * log(Q));
    const double Z = __builtin_fma(S, S, 1.0);
    const double C = 1.0 + expm1(inv_p * log1p(Z - 1.0));
    return M * C;
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
