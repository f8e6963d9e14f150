// Node objects evaluated by the tree kernels.  Each provides
//   leaf(a, b):     the node on two raw elements (signs allowed), as the tile levels' type R,
//   row(u, v):      the node on the levels inside a tile (R; here R = T and row = node),
//   row_root(r):    the map from a tile's root to T (the identity here),
//   node(a, b):     the node on two non-negative partial norms above the rows,
//   finish(r):      the map from the tree root to the result (identity for all nodes here).
// Paper (Novakovic, arXiv 2509.06220): Frobenius node = hypot (Sect. 1, Eq. (hr));
// p = 1 node = |a| + |b| (Eq. (vp1)); p = infinity node = max(|a|, |b|) (Eq. (vpI)),
// the absolute values being needed only at the lowest level (Sect. 4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "vnp_node.hpp"
#include "vnp_tree.hpp"

namespace vnp {

template <typename T>
struct HypNode;

template <>
struct HypNode<double> {
    using T = double;
    using R = double;
    __device__ double row(double a, double b) const { return node(a, b); }
    __device__ double row_root(double r) const { return r; }
    __device__ double leaf(double a, double b) const { return hyp_d_leaf(a, b); }
    __device__ double node(double a, double b) const { return hyp_d(a, b); }
    __device__ double finish(double r) const { return r; }
};

template <>
struct HypNode<float> {
    using T = float;
    using R = float;
    __device__ float row(float a, float b) const { return node(a, b); }
    __device__ float row_root(float r) const { return r; }
    __device__ float leaf(float a, float b) const { return hyp_s_leaf(a, b); }
    __device__ float node(float a, float b) const { return hyp_s(a, b); }
    __device__ float finish(float r) const { return r; }
};

// The binary32 hypotenuse for finite operands (hyp_s_fast): the streamed tiles of the
// binary32 Frobenius norm use it, and a wave whose tile root is NaN (an infinite or NaN
// element, or an overflow inside a tile) is evaluated again with hyp_s.
struct HypNodeFinite32 {
    using T = float;
    using R = float;
    __device__ float row(float a, float b) const { return node(a, b); }
    __device__ float row_root(float r) const { return r; }
    __device__ float leaf(float a, float b) const { return hyp_s_fast(a, b); }
    __device__ float node(float a, float b) const { return hyp_s_fast(a, b); }
};
template <>
struct TileNode<HypNode<float>> {
    using type = HypNodeFinite32;
};

template <typename T>
struct SumNode;

template <>
struct SumNode<double> {
    using T = double;
    using R = double;
    __device__ double row(double a, double b) const { return node(a, b); }
    __device__ double row_root(double r) const { return r; }
    __device__ double leaf(double a, double b) const { return __builtin_fabs(a) + __builtin_fabs(b); }
    __device__ double node(double a, double b) const { return a + b; }
    __device__ double finish(double r) const { return r; }
};

template <>
struct SumNode<float> {
    using T = float;
    using R = float;
    __device__ float row(float a, float b) const { return node(a, b); }
    __device__ float row_root(float r) const { return r; }
    __device__ float leaf(float a, float b) const { return __builtin_fabsf(a) + __builtin_fabsf(b); }
    __device__ float node(float a, float b) const { return a + b; }
    __device__ float finish(float r) const { return r; }
};

// max on non-negative values through their bit patterns: the integer order equals the
// numeric order, and NaN patterns (with the sign cleared) sort above +inf, so a NaN
// propagates to the root.
template <typename T>
struct MaxNode;

template <>
struct MaxNode<double> {
    using T = double;
    using R = double;
    __device__ double row(double a, double b) const { return node(a, b); }
    __device__ double row_root(double r) const { return r; }
    __device__ static double mx(double a, double b)
    {
        const uint64_t ia = (uint64_t)__double_as_longlong(a), ib = (uint64_t)__double_as_longlong(b);
        return __longlong_as_double((long long)(ia > ib ? ia : ib));
    }
    __device__ double leaf(double a, double b) const { return mx(__builtin_fabs(a), __builtin_fabs(b)); }
    __device__ double node(double a, double b) const { return mx(a, b); }
    __device__ double finish(double r) const { return r; }
};

template <>
struct MaxNode<float> {
    using T = float;
    using R = float;
    __device__ float row(float a, float b) const { return node(a, b); }
    __device__ float row_root(float r) const { return r; }
    __device__ static float mx(float a, float b)
    {
        const uint32_t ia = __float_as_uint(a), ib = __float_as_uint(b);
        return __uint_as_float(ia > ib ? ia : ib);
    }
    __device__ float leaf(float a, float b) const { return mx(__builtin_fabsf(a), __builtin_fabsf(b)); }
    __device__ float node(float a, float b) const { return mx(a, b); }
    __device__ float finish(float r) const { return r; }
};

// The p values the p-norm calls accept: p > 0 (not NaN) whose reciprocal, rounded once in
// the working precision, is at most 2^1000 in binary64 (the node squares its power of Z at
// most 1000 times) and finite in binary32 (the node is built from RN(1/p), Sect. 4); a p
// below that (about 2^-1000 in binary64, 2^-128 in binary32) is an invalid argument.
template <typename T>
__host__ __device__ inline bool p_ok(T p)
{
    return p > T(0) && T(1) / p <= T(sizeof(T) == 8 ? 0x1p1000 : 0x1.fffffep127);
}

// Compute units of the current device, cached per device (256 when the query fails).
inline int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev >= 0 && dev < 64 && (v = cache[dev].load(std::memory_order_relaxed)) > 0) return v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    if (dev >= 0 && dev < 64) cache[dev].store(v, std::memory_order_relaxed);
    return v;
}

// Rows per load group (one group is in flight per wave while the previous one is
// reduced): 8 KiB per wave for the binary64 hypot node, 4 KiB where the node is heavier
// in registers or arithmetic (measured on MI355X; results never depend on it).
template <class Node>
struct RowsInFlight {
    static constexpr int value = 4;
};
template <>
struct RowsInFlight<HypNode<double>> {
    static constexpr int value = 8;
};
template <>
struct RowsInFlight<SumNode<double>> {
    static constexpr int value = 8;
};
template <>
struct RowsInFlight<MaxNode<double>> {
    static constexpr int value = 8;
};

// Waves per compute unit the single-vector launch aims for (several rounds of resident
// blocks; tiles per wave follow).  The binary32 hypot kernel does twice the node work per
// 64 KiB tile and runs best with half the waves: SNRMF n = 2^30 0.651 ms with 4 tiles per
// wave (64 waves per CU) against 0.669 ms with 2 (128 per CU), n = 636086033 0.404 against
// 0.411 ms (interleaved runs on MI355X); the binary64 and p-node kernels measured flat.
template <class Node>
struct TargetWavesPerCU {
    static constexpr int value = 128;
};
template <>
struct TargetWavesPerCU<HypNode<float>> {
    static constexpr int value = 64;
};

// Kernel-entry hook: every thread of the block calls it before the first node evaluation
// (a node that keeps a table in LDS fills it there).  Nothing to do for these nodes.
template <class Node>
__device__ __forceinline__ void node_prologue(const Node &)
{
}

// The part of a node that device functions outside the kernel body receive (a node
// with large per-launch tables gives a small evaluation part); these nodes are small.
template <class Node>
__host__ __device__ inline Node node_eval(const Node &nd)
{
    return nd;
}

}  // namespace vnp
