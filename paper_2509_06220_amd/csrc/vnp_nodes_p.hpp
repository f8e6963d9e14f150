// p-norm node (Novakovic, arXiv 2509.06220, Sect. 4).
//
// For partial p-norms a, b >= 0 with M = max, m = min:
//     node(a, b) = M C,  C = Z^(1/p),  Z = fma(S, S, 1),  S = Q^(p/2),  Q = m / M
// (Eq. (sp), (qp); Listing 5 forms 1 + Q^p as fma(S, S, 1) the same way).  p/2 and 1/p
// are rounded once and hoisted out of the recursion (Sect. 4); binary32 uses RN32(p/2)
// and RN32(1/p) and evaluates the node in binary64, rounding the node value to binary32.
//
// The two powers are evaluated on the ranges the node produces, without the
// general-purpose library routines and without a division, from tables in LDS:
//   S = 2^((p/2) log2 Q),  log2 Q = (e_m - e_M) + log2 f_m - log2 f_M  (frexp parts f in
//   [1/2, 1), exponents e).  log2 f: the top LP_LOG_BITS fraction bits of f pick c_j ~ 1/f
//   and l_j = log2(2 / c_j); log2 f + 1 = l_j + t g(t), t = fma(f, c_j, -1), -1.01 * 2^-11
//   <= t <= 1.01 * 2^-10, g of degree 3, evaluated as fma(t, g, l_j).  Entry 0 is the
//   interval's left end (c_0 = 2, l_0 = 0), so that f = 1/2 gives exactly 0.
//   2^(y/N) for y = N (p/2) log2 Q, N = 2^LP_EXP_BITS = 512: y = N k + j + u with integers
//   k, j in [0, N) and |u| <= 1/2 (rounding y to an integer by adding 1.5 * 2^52, whose low
//   word then holds it), 2^(y/N) = 2^k T_j (1 + u H(u)), T_j = RN(2^(j/N)), H of degree 3.
//   C = Z^a, a = RN(1/p), Z in [1, 2]: with a = a' 2^s, a' <= 2, C = (Z^a')^(2^s).  The top
//   LP_POW_BITS fraction bits of Z pick c'_j = RN(512 / (512 + j)) (the reciprocal of the
//   interval's left end), R_j = (1/c'_j)^a' and rho_j = R_j - 1 (both rounded from an
//   extended-precision value; one device table per (device, p), built and uploaded by
//   make_lp_node on first use); with t = fma(Z, c'_j, -1) in [0, 2^-9),
//   Z^a' = R_j (1 + t)^a' and (1 + t)^a' = 1 + u, u = t (b_1 + b_2 t + ... + b_5 t^4)
//   with the binomial coefficients b_k of a'.  Then Z^a' = 1 + w, w = fma(u, R_j, rho_j),
//   so R_j's rounding touches only the small product; each squaring maps w to w (w + 2);
//   and the node is fma(M, w, M), one rounding of M (1 + w).
// (Coefficients and tables: Chebyshev fits and 60-digit values written by lp_coeffs.py.)
//
// Errors: the log2 table values carry 2^-54 absolute and the two fma(t, g, l_j) 2^-54
// each, g 2^-56.4 (absolute), 1 + u H(u) 2^-62.7 and T_j 2^-53 (relative); the binomial
// series omits less than 2^-59.4.  An absolute error d in log2 Q changes C by at most
// (ln 2 / 2) d relatively, whatever p is (the error of S^2 is weighted by
// S^2 / (p (1 + S^2)) in C); each squaring doubles the relative error of Z^a', so p < 1/2
// costs about 2^s ulps more.
//
// Special operands: M and m come from v_max_f64 / v_min_f64 (the non-NaN operand if one
// is NaN); w is finite and positive for every input (a NaN or infinite Z is clamped into
// [1, 2) before the table lookup, and rho_0 = 2^-1074 instead of 0, whose s squarings stay
// below 2^-1074 * 2^(s + 1) < 2^-54 for s <= 1000), so fma(M, w, M) is +inf for an
// infinite M and equals M whenever w < 2^-54; a NaN operand turns w into a quiet NaN.
// m = 0 (Q = 0) clears the high word of S: what is left is below 2^-1042, its square
// vanishes, Z = 1, w = 2^(s - 1074) at most, and node(M, 0) = M exactly.
//
// This value form evaluates every node of binary32 and the levels above the tiles of
// binary64; inside a tile, binary64 carries logarithms instead (LpPair, below).
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

constexpr int LP_LOG_N = 1 << LP_LOG_BITS;
constexpr int LP_EXP_N = 1 << LP_EXP_BITS;
constexpr int LP_POW_N = 1 << LP_POW_BITS;
constexpr int LP_B_N = 8;  // binomial coefficient slots (LP_POW_TERMS used)
constexpr double LP_RHO0 = 0x1p-1074;  // rho_0 (see above)

// The tables in LDS, one copy per block, filled by lp_table_fill at kernel entry, in one
// arena: the log2 table first (1025 entries), then 2^(j/N), the power table and the
// coefficients.  log2_p1 indexes with the exponent's low bit, so the mantissa of a NaN
// (from two NaN operands, whose result is replaced) picks an index in [1024, 2048): the
// arena spans more than 2048 log2 entries, so that read stays inside it.
struct PowEntry {
    double R, rho, c, pad;
};
// Polynomial coefficients: g (4), H (5), then the binomial coefficients b_1 .. b_5 (and
// zeros).  Read at one address in all lanes: as scalar operands they would exhaust the
// scalar registers, and two scalar operands of one fma cost an extra vector move.
constexpr int LP_G_OFF = 0, LP_H_OFF = 4, LP_BC_OFF = LP_H_OFF + LP_EXP_DEG + 1;
constexpr int LP_LOG_BYTES = (LP_LOG_N + 1) * 16;
constexpr int LP_EXP_AT = LP_LOG_BYTES;
constexpr int LP_POW_AT = LP_EXP_AT + LP_EXP_N * 8;
constexpr int LP_COEF_AT = LP_POW_AT + LP_POW_N * (int)sizeof(PowEntry);
constexpr int LP_ARENA_BYTES = LP_COEF_AT + (LP_BC_OFF + LP_B_N) * 8;
static_assert(LP_ARENA_BYTES >= 2 * LP_LOG_N * 16 && LP_POW_AT % 16 == 0 && LP_COEF_AT % 16 == 0,
              "arena layout");
__device__ __forceinline__ unsigned char *lp_arena()
{
    __shared__ __attribute__((aligned(16))) unsigned char arena[LP_ARENA_BYTES];
    return arena;
}
__device__ __forceinline__ double2 *lp_log_lds() { return reinterpret_cast<double2 *>(lp_arena()); }  // {c_j, l_j}
__device__ __forceinline__ double *lp_exp_lds() { return reinterpret_cast<double *>(lp_arena() + LP_EXP_AT); }  // T_j
__device__ __forceinline__ PowEntry *lp_pow_lds()  // {R_j, rho_j, c'_j}
{
    return reinterpret_cast<PowEntry *>(lp_arena() + LP_POW_AT);
}
__device__ __forceinline__ double *lp_coef_lds() { return reinterpret_cast<double *>(lp_arena() + LP_COEF_AT); }

// Every thread of the block calls this before the first node evaluation.  rr: the per-p
// device table (R_0 .. R_511, rho_0 .. rho_511); b: the binomial coefficients.
__device__ __forceinline__ void lp_table_fill(const double *rr, const double *b)
{
    double2 *lt = lp_log_lds();
    double *et = lp_exp_lds();
    PowEntry *pt = lp_pow_lds();
    for (int i = threadIdx.x; i <= LP_LOG_N; i += blockDim.x) lt[i] = make_double2(lp_log_src[i][0], lp_log_src[i][1]);
    for (int i = threadIdx.x; i < LP_EXP_N; i += blockDim.x) et[i] = lp_exp_src[i];
    for (int i = threadIdx.x; i < LP_POW_N; i += blockDim.x)
        pt[i] = PowEntry{rr[i], rr[LP_POW_N + i], lp_pow_src[i], 0.0};
    double *cf = lp_coef_lds();
    if (threadIdx.x < 4) cf[LP_G_OFF + threadIdx.x] = lp_log_g[threadIdx.x];
    if (threadIdx.x <= LP_EXP_DEG) cf[LP_H_OFF + threadIdx.x] = lp_exp_h[threadIdx.x];
    if (threadIdx.x < LP_B_N) cf[LP_BC_OFF + threadIdx.x] = b[threadIdx.x];
    __syncthreads();
}

// log2 f + 1 for f in [1/2, 1] (the exponent's low bit selects entry LP_LOG_N for f = 1).
__device__ __forceinline__ double log2_p1(double f)
{
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(f) >> 32);
    const double2 e = lp_log_lds()[(hi >> (20 - LP_LOG_BITS)) & (2 * LP_LOG_N - 1)];
    const double t = __builtin_fma(f, e.x, -1.0);
    const double *G = lp_coef_lds() + LP_G_OFF;
    double g = G[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) g = __builtin_fma(g, t, G[i]);
    return __builtin_fma(t, g, e.y);
}

// Lower clamp of y (2^(y/N) underflows to +0 well above it; |y| < 2^31 for the rounding).
constexpr double LP_Y_MIN = -2100.0 * LP_EXP_N;

// 2^(y/N), N = 2^LP_EXP_BITS, for y in [LP_Y_MIN, 0] (y = +inf gives NaN, which the caller
// absorbs).
__device__ __forceinline__ double exp2_tab(double y)
{
    // y + 1.5 * 2^52 holds round(y) in its low word (|y| < 2^31)
    const double big = y + 0x1.8p52;
    const int k = (int)(uint32_t)(uint64_t)__double_as_longlong(big);
    const double u = y - (big - 0x1.8p52);  // exact, |u| <= 1/2
    const double T = lp_exp_lds()[k & (LP_EXP_N - 1)];
    const double *Hc = lp_coef_lds() + LP_H_OFF;
    double h = Hc[0];
#pragma unroll
    for (int i = 1; i <= LP_EXP_DEG; ++i) h = __builtin_fma(h, u, Hc[i]);
    return __builtin_amdgcn_ldexp(__builtin_fma(T, u * h, T), k >> LP_EXP_BITS);
}

// w = Z^a - 1 for Z in [1, 2] (a = a' 2^s, see above).
__device__ __forceinline__ double pow_z_m1(double Z, int sq)
{
    const double *b = lp_coef_lds() + LP_BC_OFF;
    const double Zc = __builtin_fmin(Z, 0x1.fffffffffffffp0);  // Z = 2 as its predecessor: within Z's rounding
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(Zc) >> 32);
    const PowEntry &e = lp_pow_lds()[(hi >> (20 - LP_POW_BITS)) & (LP_POW_N - 1)];
    const double t = __builtin_fma(Zc, e.c, -1.0);  // in [0, 2^-9)
    double q = b[4];
    q = __builtin_fma(q, t, b[3]);
    q = __builtin_fma(q, t, b[2]);
    q = __builtin_fma(q, t, b[1]);
    q = __builtin_fma(q, t, b[0]);
    double w = __builtin_fma(t * q, e.R, e.rho);
    for (int i = 0; i < sq; ++i) w = w * (w + 2.0);
    return w;
}

// The node on |a|, |b| (ABS: a leaf, whose operands carry signs; otherwise a, b >= 0),
// NaN and infinities as above; hpy = N RN(p/2) (exact), N = 2^LP_EXP_BITS.
template <bool ABS>
__device__ __forceinline__ double lp_core(double a, double b, double hpy, int sq)
{
    // v_max_f64 / v_min_f64 directly, the absolute values as operand modifiers: as fmax /
    // fmin the compiler first canonicalizes each operand (two more instructions), which only
    // matters for NaN operands, restored below
    double M, m;
    if constexpr (ABS) {
        asm("v_max_f64 %0, |%1|, |%2|" : "=v"(M) : "v"(a), "v"(b));
        asm("v_min_f64 %0, |%1|, |%2|" : "=v"(m) : "v"(a), "v"(b));
    } else {
        asm("v_max_f64 %0, %1, %2" : "=v"(M) : "v"(a), "v"(b));
        asm("v_min_f64 %0, %1, %2" : "=v"(m) : "v"(a), "v"(b));
    }
    const bool nan = __builtin_isunordered(a, b);
    const double hM = log2_p1(__builtin_amdgcn_frexp_mant(M));
    const double hm = log2_p1(__builtin_amdgcn_frexp_mant(m));
    const int e = __builtin_amdgcn_frexp_exp(m) - __builtin_amdgcn_frexp_exp(M);
    const double lq = (double)e + (hm - hM);  // log2 Q <= 0
    const double S = exp2_tab(__builtin_fmax(hpy * lq, LP_Y_MIN));
    const uint64_t sb = (uint64_t)__double_as_longlong(S);
    const uint32_t shi = m > 0.0 ? (uint32_t)(sb >> 32) : 0u;  // m = 0: S below 2^-1042
    const double Sm = __longlong_as_double((long long)(((uint64_t)shi << 32) | (sb & 0xffffffffu)));
    const uint64_t wb = (uint64_t)__double_as_longlong(pow_z_m1(__builtin_fma(Sm, Sm, 1.0), sq));
    const uint32_t whi = nan ? 0x7ff80000u : (uint32_t)(wb >> 32);  // a NaN operand: w is a quiet NaN
    return __builtin_fma(M, __longlong_as_double((long long)(((uint64_t)whi << 32) | (wb & 0xffffffffu))), M);
}

// ---------------------------------------------------------------------------------
// The levels inside a tile of the binary64 p node in the logarithmic domain.
//
// Inside a tile (the per-lane rows with the leaves, the columns and the lanes: 8191 of every
// 8192 nodes) each partial norm v is carried as a pair (l, e) with v = 2^(e + l), l in
// [0, 1) and e an integer.  The node on these levels ("row" node) is
// Sect. 4's node(a, b) = M (1 + Q^p)^(1/p) with the logarithm taken of both sides:
//     log2 node = log2 M + (1/p) log2(1 + 2^(p d)),  d = log2 m - log2 M = -|log2 a - log2 b|,
// with 2^(p d) = S^2 = Q^(2 RN(p/2)) and 1/p = RN(1/p) (the exponents rounded once, Sect. 4).
// An internal row node therefore needs no logarithm of its operands and no power: one 2^y
// (the table above, y = N p d), one log2(1 + S^2) (the log2 table at (1 + S^2)/2, whose
// rounding is that of Z = fma(S, S, 1)), and an fma; a leaf takes the logarithms of its two
// elements first.  The tile root goes back to a value, 2^l scaled by 2^e, and the levels
// above (tiles, runs, blocks) use the value node lp_core.
//
// Exactness and special values:
//   * node(v, 0) = v exactly: a zero operand gives S^2 = 0, (1 + S^2)/2 = 1/2, whose log2
//     table entry (c_0 = 2, l_0 = 0) gives log2 = 0 exactly, and l + 0 keeps l and e; the
//     zero padding of the tree is therefore exact.
//   * +0 is e <= -2^29 (LP_ZERO_E = -2^30, with a finite l), +inf e in [2^27, 2^29)
//     (LP_INF_E), NaN e >= 2^29 (LP_NAN_E), both with l = 0, set by the leaves.  The row
//     node orders such pairs like the values they stand for (NaN above inf above every
//     finite value above +0), and a level moves e by at most 1/p + 1, so the thirteen
//     levels of a tile keep every class apart while 1/p <= 2^20 (for larger 1/p, i.e. p
//     below about 9.5e-7, the node stays in the value domain: the uniform flag `pair`).
//     The conversion to a value maps e beyond the binary64 range to +inf or +0 by ldexp,
//     and NaN pairs to NaN.
//   * Errors per row node: the two table functions (2^-54 each, absolute in log2), the
//     rounding of (1 + S^2)/2, which reaches log2 multiplied by 1/p as in Sect. 4's
//     C = Z^(1/p), and the rounding of l (2^-54 absolute); in the value these are relative
//     errors times ln 2.
struct LpPair {
    double l;  // in [0, 1)
    int e;
};
// exchange of a pair between lanes (the lane levels of a tile)
__device__ __forceinline__ LpPair xshfl(LpPair v, int s) { return LpPair{__shfl_xor(v.l, s), __shfl_xor(v.e, s)}; }
constexpr int LP_ZERO_E = -(1 << 30);
constexpr int LP_INF_E = 1 << 28;
constexpr int LP_NAN_E = 1 << 29;
constexpr double LP_PAIR_MAX_IA = 0x1p20;  // largest 1/p of the logarithmic tile levels

// The common tail of the row node and the leaf: log2 M + (1/p) log2(1 + 2^y) as a pair,
// for y = N p d <= 0 (y = N p d clamped; d <= 0 up to the table's rounding, which
// -|d| absorbs).
__device__ __forceinline__ LpPair lp_pair_tail(double d, double lM, int eM, double py, double ia)
{
    const double y = __builtin_fmax(-py * __builtin_fabs(d), LP_Y_MIN);
    const double S2 = exp2_tab(y);
    // (1 + S^2)/2 in [1/2, 1] (S^2 <= 1 since y <= 0)
    const double lr = __builtin_fma(ia, log2_p1(__builtin_fma(S2, 0.5, 0.5)), lM);  // >= 0
    return LpPair{__builtin_amdgcn_fract(lr), eM + (int)lr};  // (int) truncates: floor
}

// Row node on two pairs.
__device__ __forceinline__ LpPair lp_pair_node(LpPair a, LpPair b, double py, double ia)
{
    const double d = (double)(a.e - b.e) + (a.l - b.l);  // log2 a - log2 b
    const bool ga = d >= 0.0;
    return lp_pair_tail(d, ga ? a.l : b.l, ga ? a.e : b.e, py, ia);
}

// Leaf on two elements (signs allowed): log2 |a|, log2 |b| from the log2 table, then the
// row node.  Zeros and non-finite operands are fixed up afterwards, in a branch that only a
// wave holding one takes (a wave-uniform test, then per-lane choices); the common path
// spends three compares on them.  The fix-ups give what the arithmetic with m's exponent
// taken as that of +0 (S^2 = 0) gives:
//   m = 0 < M: node(M, 0) = M, the pair of log2 M (l and e from lM and eM exactly);
//   M = 0:     +0, e = LP_ZERO_E (with l from the same lM, a finite value);
//   an infinite or NaN operand: l = 0 and the class's e (the logarithm of inf is not
//   finite).
__device__ __forceinline__ LpPair lp_pair_leaf(double a, double b, double py, double ia)
{
    double M, m;
    asm("v_max_f64 %0, |%1|, |%2|" : "=v"(M) : "v"(a), "v"(b));
    asm("v_min_f64 %0, |%1|, |%2|" : "=v"(m) : "v"(a), "v"(b));
    const double lM = log2_p1(__builtin_amdgcn_frexp_mant(M));
    const double lm = log2_p1(__builtin_amdgcn_frexp_mant(m));
    // frexp's exponents are one above those of the mantissa in [1, 2); equal offsets cancel
    const int eM = __builtin_amdgcn_frexp_exp(M);
    const int em = __builtin_amdgcn_frexp_exp(m);
    LpPair r = lp_pair_tail((double)(em - eM) + (lm - lM), lM, eM - 1, py, ia);
    const bool nan = __builtin_isunordered(a, b);
    const bool inf = __builtin_isinf(M);
    const bool zero = !(m > 0.0);
    if (__builtin_amdgcn_ballot_w64(nan || inf || zero) != 0) {
        if (zero) r = LpPair{__builtin_amdgcn_fract(lM), M > 0.0 ? eM - 1 + (int)lM : LP_ZERO_E};
        if (nan || inf) r = LpPair{0.0, nan ? LP_NAN_E : LP_INF_E};
    }
    return r;
}

// The value of a pair: 2^l from the 2^y table (y = N l in [0, N)), scaled by 2^e.
__device__ __forceinline__ double lp_pair_value(LpPair v)
{
    const double y = v.l * (double)LP_EXP_N;
    const double big = y + 0x1.8p52;
    const int k = (int)(uint32_t)(uint64_t)__double_as_longlong(big);
    const double u = y - (big - 0x1.8p52);
    const double T = lp_exp_lds()[k & (LP_EXP_N - 1)];
    const double *Hc = lp_coef_lds() + LP_H_OFF;
    double h = Hc[0];
#pragma unroll
    for (int i = 1; i <= LP_EXP_DEG; ++i) h = __builtin_fma(h, u, Hc[i]);
    const double r = __builtin_amdgcn_ldexp(__builtin_fma(T, u * h, T), (k >> LP_EXP_BITS) + v.e);
    return v.e >= LP_NAN_E ? __builtin_nan("") : r;
}

// The evaluation part of the p node: N RN(p/2), s, RN(1/p) and the log-domain flag, with
// every table read from LDS.  Device functions that are not inlined receive this part only
// (node_eval).  Interface of the tree: leaf(a, b) and row(u, v) on the tile levels' type R,
// row_root(r) back to T, node(a, b) on T above the tiles.
template <typename T>
struct LpEval;

template <>
struct LpEval<double> {
    using T = double;
    using R = LpPair;
    double hpy;  // N RN(p/2), N = 2^LP_EXP_BITS
    double ia;     // RN(1/p)
    int sq;        // s: C = (Z^a')^(2^s)
    int pair;      // tile levels in the logarithmic domain (1/p <= 2^20)
    __device__ LpPair leaf(double a, double b) const
    {
        if (!pair) return LpPair{lp_core<true>(a, b, hpy, sq), 0};
        return lp_pair_leaf(a, b, 2.0 * hpy, ia);
    }
    __device__ LpPair row(LpPair a, LpPair b) const
    {
        if (!pair) return LpPair{lp_core<false>(a.l, b.l, hpy, sq), 0};
        return lp_pair_node(a, b, 2.0 * hpy, ia);
    }
    __device__ double row_root(LpPair r) const { return pair ? lp_pair_value(r) : r.l; }
    __device__ double node(double a, double b) const { return lp_core<false>(a, b, hpy, sq); }
    __device__ double finish(double r) const { return r; }
};

template <>
struct LpEval<float> {
    using T = float;
    using R = float;
    double hpy;  // N RN32(p/2)
    double ia;     // unused (binary32 keeps the value node on every level)
    int sq;
    int pair;
    __device__ float leaf(float a, float b) const
    {
        return (float)lp_core<true>((double)a, (double)b, hpy, sq);
    }
    __device__ float node(float a, float b) const { return (float)lp_core<false>((double)a, (double)b, hpy, sq); }
    __device__ float row(float a, float b) const { return node(a, b); }
    __device__ float row_root(float r) const { return r; }
    __device__ float finish(float r) const { return r; }
};

// The p node as the kernels receive it: the evaluation part, the binomial coefficients
// and the device table of R_j and rho_j (small kernel arguments: a large argument block
// costs several microseconds of host time per launch), which the kernel prologue copies
// to LDS.
template <typename T>
struct LpNode : LpEval<T> {
    double b[LP_B_N];  // binomial coefficients b_1 .. b_5 of a' (the rest 0)
    const double *rr;  // device: R_0 .. R_511, then rho_0 .. rho_511
};

template <typename T>
__host__ __device__ inline LpEval<T> node_eval(const LpNode<T> &nd)
{
    return LpEval<T>{nd.hpy, nd.ia, nd.sq, nd.pair};
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
    double b[LP_B_N];
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
        for (int i = 1; i <= LP_B_N; ++i) {
            bk = bk * ((long double)ap - (i - 1)) / i;
            en.b[i - 1] = i <= LP_POW_TERMS ? (double)bk : 0.0;
        }
        static double h[2 * LP_POW_N];  // under the cache lock
        for (int j = 0; j < LP_POW_N; ++j) {
            const long double r = std::pow(1.0L / (long double)lp_pow_host[j], (long double)ap);
            h[j] = (double)r;
            h[LP_POW_N + j] = j == 0 ? LP_RHO0 : (double)(r - 1.0L);  // R_0 = 1
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
    out->hpy = half_p * (double)LP_EXP_N;
    out->ia = a;
    out->sq = it->second.sq;
    out->pair = sizeof(T) == 8 && a <= LP_PAIR_MAX_IA;
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
