// Device node primitives: the hypotenuse that combines two partial norms.
//
// Paper (Novakovic, arXiv 2509.06220), Sect. 1: a node needs no undue overflow or
// underflow, monotonicity and a small relative error |eps_h| <= c eps.  Listing 2 meets
// this with a division and a square root per node; Sect. 3 names the division as the
// cost to remove.  The nodes here use no division:
//
//   hyp_d (binary64): let M be the larger of |a|, |b|, E its biased exponent clamped to
//   [1, 2045] and k = 1023 - E.  With a' = a 2^k, b' = b 2^k (exact),
//       hyp_d(a, b) = 2^-k * RN(sqrt(RN(RN(a'^2) + RN(b'^2)))),
//   i.e. two rounded squares, their rounded sum and a correctly rounded square root, all
//   in a range where nothing over- or underflows.  Relative error <= (1 + eps)^2 - 1:
//   the sum carries at most (1 + eps)^2 - 1, halved by the square root, and the root's
//   own rounding adds eps.  Every operation is commutative, so hyp_d(a, b) = hyp_d(b, a)
//   bitwise, and monotone, so the node is monotone in |a| and |b|.  Inputs may carry a
//   sign (leaves); a NaN input gives NaN, otherwise an infinite input gives +inf.
//   hyp_d(a, 0) = |a| exactly, since RN(sqrt(RN(a'^2))) = |a'| in binary floating point
//   -- zero padding of the tree is therefore exact.
//
//   hyp_s (binary32): a^2 and b^2 are exact in binary64, so
//       hyp_s(a, b) = RN_32(sqrt(RN_64(a^2 + b^2)) (1 + d)),  |d| < 2^-43,
//   with relative error below (1 + 2^-18) eps_S and no scaling needed.
//
// The square root is the Goldschmidt/Newton sequence from v_rsq_f64 that the compiler
// uses for a correctly rounded binary64 sqrt, minus its denormal rescaling: the nodes
// only take square roots of 0, inf, NaN or values in [2^-760, 2^1002], where rescaling
// is never triggered, so the result is the correctly rounded sqrt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vnp {

// Correctly rounded sqrt for s in [2^-767, 2^1023] (no special values).
__device__ __forceinline__ double sqrt_core(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y;
    double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, s);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, s);
    return __builtin_fma(d, h, g);
}

// Correctly rounded sqrt for s in {+0, +inf, NaN} or [2^-767, 2^1023].
__device__ __forceinline__ double sqrt_cr(double s)
{
    const double g = sqrt_core(s);
    // +0 and +inf are their own roots (class mask: +0 | -0 | +inf).
    return __builtin_amdgcn_class(s, 0x260) ? s : g;
}

__device__ __forceinline__ uint32_t hi_word(double v) { return (uint32_t)(__double_as_longlong(v) >> 32); }

// Exponent-scaled evaluation, valid for all inputs (signs allowed).
__device__ __forceinline__ double hyp_d_scaled(double a, double b)
{
    const uint32_t hm = max(hi_word(a) & 0x7fffffffu, hi_word(b) & 0x7fffffffu);
    const int E = min(max((int)(hm >> 20), 1), 2045);
    const int k = 1023 - E;
    const double as = __builtin_amdgcn_ldexp(a, k);
    const double bs = __builtin_amdgcn_ldexp(b, k);
    const double s = as * as + bs * bs;
    return __builtin_amdgcn_ldexp(sqrt_cr(s), -k);
}

// The binary64 node is defined piecewise.  When the larger operand lies in
// [2^-380, 2^500), RN(RN(a^2) + RN(b^2)) neither overflows nor underflows and its square
// root is in the range where sqrt_core is exact, so the node is
// RN(sqrt(RN(RN(a^2) + RN(b^2)))) computed directly; elsewhere (zeros, tiny or huge
// operands, inf, NaN) it is the scaled form above, evaluated only for the lanes that
// need it.  Both forms are symmetric, have relative error at most (1 + eps)^2 - 1 and
// give node(a, 0) = |a|; they differ only where the smaller square underflows in one
// form and not in the other.
__device__ __forceinline__ double hyp_d(double a, double b)
{
    const uint32_t hm = max(hi_word(a) & 0x7fffffffu, hi_word(b) & 0x7fffffffu);
    // exponent field of the larger operand in [1023 - 380, 1023 + 500)
    const bool fast = (hm - 0x28300000u) < (0x5F300000u - 0x28300000u);
    double r = sqrt_core(a * a + b * b);
    // wave-uniform branch (no lane-dependent control flow), per-lane choice
    if (__builtin_amdgcn_ballot_w64(!fast) != 0) {
        const double rs = hyp_d_scaled(a, b);
        r = fast ? r : rs;
    }
    return r;
}

__device__ __forceinline__ double hyp_d_leaf(double a, double b) { return hyp_d(a, b); }

// sqrt(s) to about 2^-44 relative (one Goldschmidt step from v_rsq_f64), for s in
// [2^-767, 2^1023]; NaN for s = +0 and s = +inf (0 * inf), NaN for NaN.  Rounded to
// binary32 this is the correctly rounded single-precision root except within 2^-19 ulp of
// a rounding boundary.
__device__ __forceinline__ double sqrt_for_f32(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    const double g = s * y;
    const double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    return __builtin_fma(g, r, g);
}

// The special cases come from a bound instead of a class test.  s = a^2 + b^2 of binary32
// values is +0 only for a = b = 0, +inf only for an infinite input, and otherwise lies in
// [2^-298, 2^257]; there the rounded root is at most RN32(|a| + |b|) (the hypotenuse is
// below |a| + |b|, and where the root's 2^-44 error could cross that sum, the smaller
// operand is below 2^-42 of the larger and both round to the larger), so the minimum
// picks it.  For +0 and +inf the root is NaN and the minimum picks |a| + |b|: +0 or
// +inf.  A NaN input makes both operands NaN.
__device__ __forceinline__ float hyp_s(float a, float b)
{
    const double A = (double)a, B = (double)b;
    const float g = (float)sqrt_for_f32(__builtin_fma(A, A, B * B));
    return __builtin_fminf(g, __builtin_fabsf(a) + __builtin_fabsf(b));
}

__device__ __forceinline__ float hyp_s_leaf(float a, float b) { return hyp_s(a, b); }

// hyp_s for finite operands, without the guard (10 instructions instead of 12).  The tiny
// addend makes the (0, 0) node exact: b != 0 gives b^2 >= 2^-298, whose last place is
// >= 2^-350, so RN(b^2 + 2^-400) = b^2 and s is hyp_s's; b = 0 and a != 0 likewise give
// s = a^2; a = b = 0 gives s = 2^-400, whose root 2^-200 rounds to +0.  For finite
// operands the minimum in hyp_s always picks the rounded root, so the two nodes agree
// bitwise (an overflow to +inf included).  An infinite operand gives NaN (s = inf: rsq
// gives 0 and g = inf * 0), and so does a NaN operand; a subtree of these nodes therefore
// has a NaN root unless every node in it had finite operands, and then its root is
// hyp_s's bitwise.
__device__ __forceinline__ float hyp_s_fast(float a, float b)
{
    const double A = (double)a, B = (double)b;
    return (float)sqrt_for_f32(__builtin_fma(A, A, __builtin_fma(B, B, 0x1p-400)));
}

// |x| of a single leaf (a one-element subtree).
__device__ __forceinline__ double leaf_abs(double v) { return __builtin_fabs(v); }
__device__ __forceinline__ float leaf_abs(float v) { return __builtin_fabsf(v); }

}  // namespace vnp
