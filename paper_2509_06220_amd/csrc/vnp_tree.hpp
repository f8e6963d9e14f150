// The canonical reduction tree and the device code that evaluates it.
//
// Paper (Novakovic, arXiv 2509.06220): any split of x into disjoint parts may be
// combined by a hypotenuse node (Eq. (hr)); the vectorized algorithm Z keeps one
// partial norm per vector lane, each reducing the elements in that lane by the
// recursive tree, and reduces the lane vector at the end (Sect. 3, Listing 4 and the
// lane example with p = 4, n = 16).  Results of such a vector algorithm are bitwise
// reproducible for a fixed lane count (Sect. 3); OpenMP-style chunking keeps that
// property only with a fixed reduction order (Sect. 3.1).
//
// The GPU tree fixes one lane layout and one reduction order for all launch shapes:
//
//   * elements are grouped in tiles of TILE = 64 lanes * VEC * ROWS consecutive logical
//     indices (VEC = 2 for binary64, 4 for binary32: one 16-byte load per lane per row);
//     within a tile, logical index i = row * (64 VEC) + lane * VEC + c;
//   * the tree is the perfect binary tree over the zero-padded logical index whose
//     levels consume index bits in this order: the ROWS bits (low to high; this is Z's
//     per-lane recursion over rows), the c bits, the lane bits 0..5, then the tile index
//     bits (low to high);
//   * a node whose right operand is a padding zero returns its left operand exactly, so
//     the result equals the same tree with absent children skipped.
//
// The levels inside a tile (per-lane rows with the leaves, columns, lanes) may carry a
// node-specific representation R of the partial norms (the binary64 p node keeps log2 of
// them); each tile root is mapped back to the element type (row_root) before the tiles are
// combined.  Every path below changes representation at that same level, so the tree and
// its bits stay one.
//
// Any launch evaluates aligned power-of-two subtrees of this one tree (a wave: a tile or
// a run of tiles; a block: a run of waves; the finish: the tree over block results), so
// the value depends on the logical vector only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "vnp_node.hpp"

namespace vnp {

constexpr int WAVE = 64;
constexpr int ROWS = 64;  // rows per tile: depth of the per-lane row tree is 6

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
// The same vectors at the alignment of one element: a contiguous input needs only its
// natural alignment for the 16-byte loads (the target allows dword-aligned vector loads).
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

template <typename T>
struct Vec;
template <>
struct Vec<double> {
    using V = d2v;
    using VU = d2u;
    static constexpr int N = 2;
    __device__ static double get(const V &v, int c) { return v[c]; }
    __device__ static V zero() { return V{0.0, 0.0}; }
};
template <>
struct Vec<float> {
    using V = f4v;
    using VU = f4u;
    static constexpr int N = 4;
    __device__ static float get(const V &v, int c) { return v[c]; }
    __device__ static V zero() { return V{0.f, 0.f, 0.f, 0.f}; }
};

template <typename T>
constexpr int64_t tile_elems() { return (int64_t)WAVE * Vec<T>::N * ROWS; }

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// ---------------------------------------------------------------------------------
// Loaders.  Row `r` of a tile, as seen by `lane`: the VEC consecutive logical elements
// tile_base + r * (64 VEC) + lane * VEC + c.
// ---------------------------------------------------------------------------------
template <typename T>
struct LoadFast {  // contiguous, naturally aligned, full tile
    using V = typename Vec<T>::V;
    using VU = typename Vec<T>::VU;
    const VU *__restrict__ p;  // tile base
    __device__ V operator()(int r, int lane) const { return __builtin_nontemporal_load(p + r * WAVE + lane); }
};

// Address map of a strided input: logical element i is x[(i >> 1) pair + (i & 1) part].
// A real vector with stride inc has pair = 2 inc, part = inc (so element i is x[i inc]);
// the real view (re, im, re, im, ...) of a complex vector with stride inc (in complex
// elements) has pair = 2 inc, part = 1.
struct Stride {
    int64_t pair, part;
};
__host__ __device__ inline Stride real_stride(int64_t inc) { return Stride{2 * inc, inc}; }

template <typename T>
struct LoadGeneric {  // any stride / alignment / partial tile; zero beyond n (n >= 1)
    using V = typename Vec<T>::V;
    const T *x;  // logical element 0
    Stride st;
    int64_t n, base;
    __device__ V operator()(int r, int lane) const
    {
        V v;
        const int64_t i0 = base + (int64_t)r * (WAVE * Vec<T>::N) + lane * Vec<T>::N;
#pragma unroll
        for (int c = 0; c < Vec<T>::N; ++c) {
            // branch-free: lanes past the end read element 0 and keep a zero, so no
            // lane-dependent control flow precedes the wave-wide steps that follow
            const int64_t i = i0 + c;
            const bool in = i < n;
            const int64_t j = in ? i : 0;
            const T e = x[(j >> 1) * st.pair + (j & 1) * st.part];
            v[c] = in ? e : T(0);
        }
        return v;
    }
};

template <typename T>
struct LoadTail {  // contiguous, naturally aligned, the last (partial) tile of the vector
    using V = typename Vec<T>::V;
    using VU = typename Vec<T>::VU;
    const T *x;  // logical element 0
    int64_t n, base;
    __device__ V operator()(int r, int lane) const
    {
        constexpr int RE = WAVE * Vec<T>::N;  // elements per row
        const int64_t r0 = base + (int64_t)r * RE;
        if (r0 + RE <= n)  // a row inside the vector: one vector load per lane (wave-uniform test)
            return __builtin_nontemporal_load(reinterpret_cast<const VU *>(x + r0) + lane);
        V v;
#pragma unroll
        for (int c = 0; c < Vec<T>::N; ++c) {  // the partial row: branch-free, as LoadGeneric
            const int64_t i = r0 + lane * Vec<T>::N + c;
            const bool in = i < n;
            const T e = x[in ? i : 0];
            v[c] = in ? e : T(0);
        }
        return v;
    }
};

// ---------------------------------------------------------------------------------
// Subtree roots in registers.
// ---------------------------------------------------------------------------------

// Butterfly over lane bits 0..5; the lower lane is always the left operand.  On return
// every lane holds the root.
template <class Node, typename T>
__device__ __forceinline__ T lane_tree(const Node &nd, T t, int lane)
{
#pragma unroll
    for (int s = 1; s < WAVE; s <<= 1) {
        const T o = __shfl_xor(t, s);
        const bool upper = (lane & s) != 0;
        t = nd.node(upper ? o : t, upper ? t : o);
    }
    return t;
}

// The same butterfly on a tile's levels in the row representation R (row nodes; the
// exchange of a non-scalar R is an overload of xshfl found with R).  Each lane takes its own
// value as the left operand: lane 0 is the lower lane at every level, so its result is the
// ordered tree's, and the kernels read the tile root from lane 0 (every node here is also
// symmetric bitwise, so the other lanes hold the same value).
__device__ __forceinline__ double xshfl(double v, int s) { return __shfl_xor(v, s); }
__device__ __forceinline__ float xshfl(float v, int s) { return __shfl_xor(v, s); }
template <class Node, typename R>
__device__ __forceinline__ R lane_tree_rows(const Node &nd, R t, int)
{
#pragma unroll
    for (int s = 1; s < WAVE; s <<= 1) t = nd.row(t, xshfl(t, s));
    return t;
}

// Merge a new row subtree root `cur` at level 0 of a binary-counter stack, given that `idx`
// subtrees were pushed before (idx is wave-uniform).  After the push of the last of 2^L
// subtrees, stk[L] holds the root of all of them.
template <class Node, typename R, int L>
__device__ __forceinline__ void push(const Node &nd, R (&stk)[L + 1], R cur, int idx)
{
    bool carry = true;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const bool bit = (idx >> l) & 1;
        if (carry && bit) cur = nd.row(stk[l], cur);
        if (carry && !bit) stk[l] = cur;
        carry = carry && bit;
    }
    if (carry) stk[L] = cur;
}

// Loads U rows (group g of a tile) into buf.
template <int U, class Load>
__device__ __forceinline__ void load_rows(typename Load::V (&buf)[U], const Load &ld, int g, int lane)
{
#pragma unroll
    for (int u = 0; u < U; ++u) buf[u] = ld(g * U + u, lane);
}

// A wave-uniform copy of v (all lanes hold the same value): lets the compiler keep it in
// scalar registers.
__device__ __forceinline__ double uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Root of the partial tail tile of a contiguous, aligned input (kept out of line so the
// vector-load loop keeps its registers): full rows by vector loads, the partial row by
// masked loads.  Row groups past the end of the vector hold only zeros; they are not
// loaded, and the partly filled group stack is combined as the zero-padded tree
// (node(a, 0) = a).
// Not inlined, so it receives the node's evaluation part (node_eval), which is small.
template <class Node, int U>
__device__ __noinline__ typename Node::T tail_tile_root(Node nd, const typename Node::T *x, int64_t n, int64_t t,
                                                        int lane)
{
    using T = typename Node::T;
    using R = typename Node::R;
    using VV = Vec<T>;
    using V = typename VV::V;
    constexpr int C = VV::N;
    constexpr int G = ROWS / U;
    constexpr int LG = ilog2(G);
    const int64_t base = t * tile_elems<T>();
    const LoadTail<T> ld{x, n, base};
    const int64_t rows = (n - base + WAVE * C - 1) / (WAVE * C);  // rows holding elements, >= 1
    const int gn = rows >= G * U ? G : (int)((rows + U - 1) / U);  // wave-uniform
    R rstk[C][LG + 1];
#pragma unroll 1
    for (int g = 0; g < gn; ++g) {
        V v[U];
        load_rows<U>(v, ld, g, lane);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            R w[U / 2];
#pragma unroll
            for (int u = 0; u < U / 2; ++u) w[u] = nd.leaf(VV::get(v[2 * u], c), VV::get(v[2 * u + 1], c));
#pragma unroll
            for (int s = U / 4; s >= 1; s >>= 1) {
#pragma unroll
                for (int u = 0; u < s; ++u) w[u] = nd.row(w[2 * u], w[2 * u + 1]);
            }
            push<Node, R, LG>(nd, rstk[c], w[0], g);
        }
    }
    R col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        R cur = rstk[c][0];  // gn >= 1: some level below is filled
        bool any = false;
#pragma unroll
        for (int l = 0; l <= LG; ++l) {
            if ((gn >> l) & 1) {
                cur = any ? nd.row(rstk[c][l], cur) : rstk[c][l];
                any = true;
            }
        }
        col[c] = cur;
    }
    R r;
    if constexpr (C == 2) {
        r = nd.row(col[0], col[1]);
    } else {
        r = nd.row(nd.row(col[0], col[1]), nd.row(col[2], col[3]));
    }
    return nd.row_root(lane_tree_rows(nd, r, lane));
}

constexpr int MAX_LWT = 12;  // a wave covers at most 2^12 tiles

// A cheaper evaluation of a node inside the streamed tiles: TileNode<Node>::type gives
// Node's values bitwise wherever it is valid and a NaN tile root wherever it is not; a
// wave that meets such a tile is evaluated again with Node.  Nodes without one use
// themselves.
template <class Node>
struct TileNode {
    using type = Node;
};

// Root of the 2^lwt consecutive tiles starting at tile index t0 (tiles at or beyond
// ntiles are padding and are skipped exactly): per-lane row trees (rows in groups of U),
// then columns, then lanes, for each tile; then the tiles, by a binary-counter stack of
// tile roots.  One group of rows is always in flight while the previous one is reduced,
// across tile boundaries.  FAST: contiguous, naturally aligned input.  The streamed
// tiles use the node tn, the tail tile and the tile roots nd; nan_tile is set when a
// streamed tile's root is NaN.
template <class Node, int U, bool FAST, class TN>
__device__ __forceinline__ typename Node::T wave_root_with(const Node &nd, const TN &tn, const typename Node::T *x,
                                                           int64_t n, Stride sd, int64_t t0, int64_t ntiles, int lwt,
                                                           int lane, bool &nan_tile)
{
    using T = typename Node::T;
    using R = typename TN::R;
    using VV = Vec<T>;
    using V = typename VV::V;
    constexpr int C = VV::N;
    constexpr int G = ROWS / U;
    constexpr int LG = ilog2(G);
    constexpr int64_t TE = tile_elems<T>();
    static_assert(U >= 2 && (U & (U - 1)) == 0 && G >= 2, "U must be a power of two in [2, ROWS/2]");

    if (t0 >= ntiles) return T(0);
    const int64_t left = ntiles - t0;
    const int ktiles = left < ((int64_t)1 << lwt) ? (int)left : (1 << lwt);
    const int Q = ktiles * G;  // row groups to reduce (even)

    R rstk[C][LG + 1];
    T tstk[MAX_LWT + 1];

    // binary counter over tile roots; entries stay wave-uniform.  After the last of
    // 2^MAX_LWT pushes the carry reaches the top level.
    auto push_tile = [&](T t, int idx) {
        bool carry = true;
#pragma unroll
        for (int l = 0; l < MAX_LWT; ++l) {
            const bool bit = (idx >> l) & 1;
            if (carry && bit) t = uniform(nd.node(tstk[l], t));
            if (carry && !bit) tstk[l] = t;
            carry = carry && bit;
        }
        if (carry) tstk[MAX_LWT] = t;
    };

    auto step = [&](const V(&v)[U], int q) {
        const int g = q & (G - 1);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            R w[U / 2];
#pragma unroll
            for (int u = 0; u < U / 2; ++u) w[u] = tn.leaf(VV::get(v[2 * u], c), VV::get(v[2 * u + 1], c));
#pragma unroll
            for (int s = U / 4; s >= 1; s >>= 1) {
#pragma unroll
                for (int u = 0; u < s; ++u) w[u] = tn.row(w[2 * u], w[2 * u + 1]);
            }
            push<TN, R, LG>(tn, rstk[c], w[0], g);
        }
        if (g == G - 1) {
            R t;
            if constexpr (C == 2) {
                t = tn.row(rstk[0][LG], rstk[1][LG]);
            } else {
                t = tn.row(tn.row(rstk[0][LG], rstk[1][LG]), tn.row(rstk[2][LG], rstk[3][LG]));
            }
            const T root = uniform(tn.row_root(lane_tree_rows(tn, t, lane)));
            if constexpr (!std::is_same<TN, Node>::value) nan_tile = nan_tile || root != root;
            push_tile(root, q >> LG);
        }
    };

    // Stream row groups [q0, q1) of the run through `ld_of(tile)`, one group in flight.
    // Full tiles of contiguous aligned input use vector loads only, so the loop waits
    // for exactly the previous group; the one partial tail tile goes through the
    // generic loader in a loop of its own.
    auto stream_groups = [&](auto ld_of, int q0, int q1) {
        // q1 - q0 is even.  In the steady-state loop every prefetch is unconditional, so
        // the wait before reducing a buffer covers exactly that buffer's loads; the
        // scheduling barriers keep each group's reduction between its successor's loads
        // and its own wait.
        V a[U], b[U];
        load_rows<U>(a, ld_of(t0 + (q0 >> LG)), q0 & (G - 1), lane);
        int q = q0;
#pragma unroll 1
        for (; q + 2 < q1; q += 2) {
            load_rows<U>(b, ld_of(t0 + ((q + 1) >> LG)), (q + 1) & (G - 1), lane);
            __builtin_amdgcn_sched_barrier(0);
            step(a, q);
            __builtin_amdgcn_sched_barrier(0);
            load_rows<U>(a, ld_of(t0 + ((q + 2) >> LG)), (q + 2) & (G - 1), lane);
            __builtin_amdgcn_sched_barrier(0);
            step(b, q + 1);
            __builtin_amdgcn_sched_barrier(0);
        }
        load_rows<U>(b, ld_of(t0 + ((q + 1) >> LG)), (q + 1) & (G - 1), lane);
        __builtin_amdgcn_sched_barrier(0);
        step(a, q);
        __builtin_amdgcn_sched_barrier(0);
        step(b, q + 1);
    };
    auto generic = [&](int64_t t) { return LoadGeneric<T>{x, sd, n, t * TE}; };
    if constexpr (FAST) {
        const int64_t full = n / TE;  // tiles entirely inside [0, n)
        const int kfull = full <= t0 ? 0 : (full - t0 < ktiles ? (int)(full - t0) : ktiles);
        auto fast = [&](int64_t t) { return LoadFast<T>{reinterpret_cast<const typename VV::VU *>(x + t * TE)}; };
        if (kfull > 0) stream_groups(fast, 0, kfull * G);
        if (kfull < ktiles)
            push_tile(uniform(tail_tile_root<decltype(node_eval(nd)), U>(node_eval(nd), x, n, t0 + kfull, lane)),
                      kfull);
    } else {
        stream_groups(generic, 0, Q);
    }
    // Root of the zero-padded run of 2^lwt tiles: ktiles were pushed; a missing right
    // subtree is zero and node(a, 0) = a, so only the filled levels combine.
    T cur = T(0);
    bool any = false;
#pragma unroll
    for (int l = 0; l <= MAX_LWT; ++l) {
        if (l < lwt + 1 && ((ktiles >> l) & 1)) {
            cur = any ? uniform(nd.node(tstk[l], cur)) : tstk[l];
            any = true;
        }
    }
    return cur;
}

// wave_root_with with Node throughout (kept out of line: waves rarely need it).
template <class Node, int U, bool FAST>
__device__ __noinline__ typename Node::T wave_root_plain(Node nd, const typename Node::T *x, int64_t n, Stride sd,
                                                         int64_t t0, int64_t ntiles, int lwt, int lane)
{
    bool unused = false;
    return wave_root_with<Node, U, FAST>(nd, nd, x, n, sd, t0, ntiles, lwt, lane, unused);
}

template <class Node, int U, bool FAST>
__device__ __forceinline__ typename Node::T wave_root(const Node &nd, const typename Node::T *x, int64_t n,
                                                      Stride sd, int64_t t0, int64_t ntiles, int lwt, int lane)
{
    using TN = typename TileNode<Node>::type;
    bool nan_tile = false;
    if constexpr (std::is_same<TN, Node>::value) {
        return wave_root_with<Node, U, FAST>(nd, nd, x, n, sd, t0, ntiles, lwt, lane, nan_tile);
    } else {
        const typename Node::T r = wave_root_with<Node, U, FAST>(nd, TN{}, x, n, sd, t0, ntiles, lwt, lane, nan_tile);
        // nan_tile is wave-uniform (it follows the tile roots)
        return nan_tile ? wave_root_plain<Node, U, FAST>(nd, x, n, sd, t0, ntiles, lwt, lane) : r;
    }
}

// Root of tile t by a block of TILE_WAVES waves (all waves call; contains a barrier).
// Wave w reduces rows [8w, 8w + 8) of the tile (an aligned subtree of every lane's row
// tree, all its loads in flight at once); the wave roots of each lane and column are
// combined in LDS in row order, then the columns and the lanes.  The root is returned to
// every lane of wave 0 (other waves get an unspecified value).  FAST: contiguous,
// naturally aligned input (sd unused).
constexpr int TILE_WAVES = 8;
constexpr int WAVE_ROWS = ROWS / TILE_WAVES;

template <class Node, bool FAST>
__device__ __forceinline__ typename Node::T tile_root_block(
    const Node &nd, const typename Node::T *x, int64_t n, Stride sd, int64_t t, int lane, int w,
    typename Node::R (&part)[Vec<typename Node::T>::N][TILE_WAVES][WAVE])
{
    using T = typename Node::T;
    using R = typename Node::R;
    using VV = Vec<T>;
    using V = typename VV::V;
    constexpr int C = VV::N;
    constexpr int64_t TE = tile_elems<T>();
    const int64_t base = t * TE;
    V v[WAVE_ROWS];
    if constexpr (FAST) {
        if (base + TE <= n) {  // a full tile (block-uniform test)
            const LoadFast<T> ld{reinterpret_cast<const typename VV::VU *>(x + base)};
#pragma unroll
            for (int r = 0; r < WAVE_ROWS; ++r) v[r] = ld(w * WAVE_ROWS + r, lane);
        } else {
            const LoadTail<T> ld{x, n, base};
#pragma unroll
            for (int r = 0; r < WAVE_ROWS; ++r) v[r] = ld(w * WAVE_ROWS + r, lane);
        }
    } else {
        const LoadGeneric<T> ld{x, sd, n, base};
#pragma unroll
        for (int r = 0; r < WAVE_ROWS; ++r) v[r] = ld(w * WAVE_ROWS + r, lane);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        R a[WAVE_ROWS / 2];
#pragma unroll
        for (int u = 0; u < WAVE_ROWS / 2; ++u) a[u] = nd.leaf(VV::get(v[2 * u], c), VV::get(v[2 * u + 1], c));
        part[c][w][lane] = nd.row(nd.row(a[0], a[1]), nd.row(a[2], a[3]));
    }
    __syncthreads();
    R col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        R b[TILE_WAVES];
#pragma unroll
        for (int j = 0; j < TILE_WAVES; ++j) b[j] = part[c][j][lane];
        col[c] = nd.row(nd.row(nd.row(b[0], b[1]), nd.row(b[2], b[3])), nd.row(nd.row(b[4], b[5]), nd.row(b[6], b[7])));
    }
    R r;
    if constexpr (C == 2) {
        r = nd.row(col[0], col[1]);
    } else {
        r = nd.row(nd.row(col[0], col[1]), nd.row(col[2], col[3]));
    }
    return nd.row_root(lane_tree_rows(nd, r, lane));
}

// Tree over v[0..m) (m a power of two) held in LDS, pairs at growing strides; the root
// ends in v[0].  Call with the whole block; contains barriers.
template <class Node, typename T>
__device__ __forceinline__ void lds_tree(const Node &nd, T *v, int m)
{
    for (int s = 1; s < m; s <<= 1) {
        __syncthreads();
        for (int i = threadIdx.x * 2 * s; i < m; i += blockDim.x * 2 * s) v[i] = nd.node(v[i], v[i + s]);
    }
    __syncthreads();
}

// Fixed tree over r[0..count) (zero-padded to a power of two), by the whole block.
// r is overwritten (chunk roots are compacted to the front between passes).  The root is
// returned to every thread.  sbuf: LDS of blockDim.x elements.
template <class Node, typename T>
__device__ T block_finish(const Node &nd, T *r, int64_t count, T *sbuf)
{
    const int nt = blockDim.x;
    const int64_t chunk = (int64_t)nt * 8;
    while (count > 1) {
        const int64_t nchunks = (count + chunk - 1) / chunk;
        for (int64_t ck = 0; ck < nchunks; ++ck) {
            const int64_t b0 = ck * chunk + (int64_t)threadIdx.x * 8;
            T e[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool in = b0 + j < count;
                const T v = r[in ? b0 + j : 0];
                e[j] = in ? v : T(0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) e[j] = nd.node(e[2 * j], e[2 * j + 1]);
            e[0] = nd.node(e[0], e[1]);
            e[2] = nd.node(e[2], e[3]);
            sbuf[threadIdx.x] = nd.node(e[0], e[2]);
            lds_tree(nd, sbuf, nt);
            if (threadIdx.x == 0) r[ck] = sbuf[0];
            __syncthreads();
        }
        count = nchunks;
    }
    __syncthreads();
    return r[0];
}

}  // namespace vnp
