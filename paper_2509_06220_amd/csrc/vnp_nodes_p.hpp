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
//   log2 Q = (e_m - e_M) + log2 f_m - log2 f_M   (frexp parts f in [1/2, 1), exponents e),
//   S = 2^((p/2) log2 Q),   C = 2^((1/p) log2 Z),  Z in [1, 2].
// log2 f for f in [1/2, 1): the top LP_TAB_BITS fraction bits of f pick c_j ~ 1 / f and
// l_j = log2(2 / c_j) from a table in LDS; then log2 f = (l_j - 1) + log2(1 + t) with
// t = fma(f, c_j, -1), |t| <= 1.01 * 2^-8, and log2(1 + t) = t g(t), g of degree 5.  No
// division is needed.  2^y splits y = k + f, |f| <= 1/2, evaluates 2^f by a degree-11
// polynomial in f and scales by 2^k.  (Coefficients and table: Chebyshev fits and
// 60-digit values written by lp_coeffs.py.)
//
// Errors: the table values carry 2^-54 absolute, the polynomials 2^-61.7 (log2(1 + t),
// absolute) and 2^-55.5 (2^f, relative).  An absolute error d in log2 Q changes C by at
// most (ln 2 / 2) d relatively, whatever p is (the error of S^2 is weighted by
// S^2 / (p (1 + S^2)) in C); one in log2 Z reaches C multiplied by ln 2 / p.
//
// Special operands: M is taken as the larger bit pattern, so a NaN operand becomes M and
// the node returns NaN; an infinite M (and no NaN) returns +inf; m = 0 returns M.  Their
// intermediate values are finite or NaN and are discarded by the final select.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vnp_internal.hpp"
#include "vnp_lp_table.hpp"

namespace vnp {

// The log2 table in LDS: one copy per block, filled by lp_table_fill at kernel entry.
__device__ __forceinline__ double2 *lp_table()
{
    __shared__ double2 tab[1 << LP_TAB_BITS];
    return tab;
}

// Every thread of the block calls this before the first node evaluation.
__device__ __forceinline__ void lp_table_fill()
{
    double2 *tab = lp_table();
    for (int i = threadIdx.x; i < (1 << LP_TAB_BITS); i += blockDim.x)
        tab[i] = make_double2(lp_tab_src[i][0], lp_tab_src[i][1]);
    __syncthreads();
}

// log2 f - (l_j - 1) for f in [1/2, 1), and l_j through `l`.
__device__ __forceinline__ double log2_part(double f, double &l)
{
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(f) >> 32);
    const double2 e = lp_table()[(hi >> (20 - LP_TAB_BITS)) & ((1u << LP_TAB_BITS) - 1)];
    l = e.y;
    const double t = __builtin_fma(f, e.x, -1.0);
    double g = -0x1.ec72d2e6fb6e9p-3;
    g = __builtin_fma(g, t, 0x1.277807fe93552p-2);
    g = __builtin_fma(g, t, -0x1.715476524c17ep-2);
    g = __builtin_fma(g, t, 0x1.ec709dc324b6cp-2);
    g = __builtin_fma(g, t, -0x1.71547652b82fep-1);
    g = __builtin_fma(g, t, 0x1.71547652b82fep+0);
    return t * g;
}

// 2^y for finite y in [-2100, 2100] (0 and +inf beyond the binary64 range).
__device__ __forceinline__ double exp2_poly(double y)
{
    const double k = __builtin_rint(y);
    const double f = y - k;  // exact, |f| <= 1/2
    double t = 0x1.e9ec1fcb69a7fp-32;
    t = __builtin_fma(t, f, 0x1.e6228acd1c6e5p-28);
    t = __builtin_fma(t, f, 0x1.b524ebd13a55fp-24);
    t = __builtin_fma(t, f, 0x1.62bfc2c86d700p-20);
    t = __builtin_fma(t, f, 0x1.ffcbfc6da6ed1p-17);
    t = __builtin_fma(t, f, 0x1.430913112c61bp-13);
    t = __builtin_fma(t, f, 0x1.5d87fe78a3f9cp-10);
    t = __builtin_fma(t, f, 0x1.3b2ab6fb9f1a5p-7);
    t = __builtin_fma(t, f, 0x1.c6b08d704a0c6p-5);
    t = __builtin_fma(t, f, 0x1.ebfbdff82c5aep-3);
    t = __builtin_fma(t, f, 0x1.62e42fefa39efp-1);
    t = __builtin_fma(t, f, 1.0);
    return __builtin_amdgcn_ldexp(t, (int)k);
}

__device__ __forceinline__ double lp_core(double a, double b, double half_p, double inv_p)
{
    const uint64_t ia = (uint64_t)__double_as_longlong(a), ib = (uint64_t)__double_as_longlong(b);
    const double M = __longlong_as_double((long long)(ia > ib ? ia : ib));
    const double m = __longlong_as_double((long long)(ia > ib ? ib : ia));
    double lM, lm;
    const double pM = log2_part(__builtin_amdgcn_frexp_mant(M), lM);
    const double pm = log2_part(__builtin_amdgcn_frexp_mant(m), lm);
    const int k = __builtin_amdgcn_frexp_exp(m) - __builtin_amdgcn_frexp_exp(M);
    const double lq = (double)k + ((lm - lM) + (pm - pM));  // log2 Q <= 0
    const double S = exp2_poly(__builtin_fmax(half_p * lq, -2100.0));
    const double Z = __builtin_fma(S, S, 1.0);  // in [1, 2]
    double lZ;
    const double pZ = log2_part(__builtin_amdgcn_frexp_mant(Z), lZ);
    const double lz = (double)(__builtin_amdgcn_frexp_exp(Z) - 1) + (lZ + pZ);  // log2 Z in [0, 1]
    const double C = exp2_poly(__builtin_fmin(inv_p * lz, 2100.0));
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

// Kernel-entry hook of the nodes: the p node fills its log2 table (the other nodes have
// nothing to set up).
template <typename T>
__device__ __forceinline__ void node_prologue(const LpNode<T> &)
{
    lp_table_fill();
}

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
