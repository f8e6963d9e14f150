// Node objects evaluated by the tree kernels.  Each provides
//   leaf(a, b):  the node on two raw elements (signs allowed),
//   node(a, b):  the node on two non-negative partial norms,
//   finish(r):   the map from the tree root to the result (identity for all nodes here).
// Paper (Novakovic, arXiv 2509.06220): Frobenius node = hypot (Sect. 1, Eq. (hr));
// p = 1 node = |a| + |b| (Eq. (vp1)); p = infinity node = max(|a|, |b|) (Eq. (vpI)),
// the absolute values being needed only at the lowest level (Sect. 4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vnp_node.hpp"
#include "vnp_tree.hpp"

namespace vnp {

template <typename T>
struct HypNode;

template <>
struct HypNode<double> {
    using T = double;
    __device__ double leaf(double a, double b) const { return hyp_d_leaf(a, b); }
    __device__ double node(double a, double b) const { return hyp_d(a, b); }
    __device__ double finish(double r) const { return r; }
};

template <>
struct HypNode<float> {
    using T = float;
    __device__ float leaf(float a, float b) const { return hyp_s_leaf(a, b); }
    __device__ float node(float a, float b) const { return hyp_s(a, b); }
    __device__ float finish(float r) const { return r; }
};

template <typename T>
struct SumNode;

template <>
struct SumNode<double> {
    using T = double;
    __device__ double leaf(double a, double b) const { return __builtin_fabs(a) + __builtin_fabs(b); }
    __device__ double node(double a, double b) const { return a + b; }
    __device__ double finish(double r) const { return r; }
};

template <>
struct SumNode<float> {
    using T = float;
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
    __device__ static float mx(float a, float b)
    {
        const uint32_t ia = __float_as_uint(a), ib = __float_as_uint(b);
        return __uint_as_float(ia > ib ? ia : ib);
    }
    __device__ float leaf(float a, float b) const { return mx(__builtin_fabsf(a), __builtin_fabsf(b)); }
    __device__ float node(float a, float b) const { return mx(a, b); }
    __device__ float finish(float r) const { return r; }
};

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

struct BatchShape {
    int lwt;     // log2(tiles per item)
    int wpb;     // waves per block
    int blocks;  // resident blocks
};

struct BatchWorkspace {
    void *roots = nullptr;
    size_t roots_cap = 0;  // bytes
    int64_t *item_off = nullptr;
    size_t item_cap = 0;  // entries
    unsigned int *seg_cnt = nullptr;
    size_t seg_cap = 0;  // entries
    unsigned long long *ctrs = nullptr;
};

int release_workspaces();
int release_batch_workspaces();
// One class of a request batch: requests [a, a + n) of the batch (sorted by class) share
// dtype and p; items work items at lwt (from request_class_items).
struct RequestClass {
    int dtype;
    double p;
    int64_t a, n;
    int64_t items;
    int lwt;
};
// Item offsets (n + 1 entries) of n requests of one dtype with lengths lens; returns the
// log2(tiles per item) they are computed for.
int request_class_items(int dtype, const int64_t *lens, int64_t n, int64_t *item_off);
// Enqueues one request batch on st: a stage kernel copies the descriptor words from
// h_src (device view of host-mapped memory; ptrs[nreq] | lens[nreq] | incs[nreq] | item
// offsets, class c's n_c + 1 entries at 3 nreq + a_c + c) to d_desc (device, at least
// 4 nreq + ncls words) and clears the class counters; then one batched launch per class
// writes request i of class c to res_d[a_c + i] or res_s[a_c + i].  ptrs are addresses of
// logical element 0 (moved for negative strides); lengths are >= 0.
int enqueue_request_batch(const void *h_src, void *d_desc, int64_t nreq, const RequestClass *cls, int ncls,
                          double *res_d, float *res_s, BatchWorkspace &ws, hipStream_t st);
void release_batch_ws(BatchWorkspace &w);
int set_launch_shape(int wpb, int wt);

}  // namespace vnp
