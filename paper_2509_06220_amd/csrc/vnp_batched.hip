// Batched norms: many segments in one persistent launch (Novakovic, arXiv 2509.06220,
// Sect. 3.1: norms of the columns of a multi-dimensional array).
//
// Work items are (segment, run of 2^lwt tiles of that segment), in a processing order
// (longest segments first when the host knows the lengths).  Wave w of the grid takes
// items w, w + W, w + 2W, ... (W waves, all resident), so the launch needs no atomics.
// Each run's root is an aligned subtree of the segment's canonical tree (the same tree
// the single-vector call uses).  A segment of one run writes its result directly; the
// run roots of longer segments are written to the workspace, and a finish kernel
// launched after the streaming kernel reduces them by the fixed tree.  Waves of the
// streaming kernel never exchange data, so the kernel needs no release or acquire
// (on a multi-XCD device those write back and invalidate the L2).  A setup kernel,
// launched first on the same stream, turns the segment lengths into item offsets
// (prefix sums over the processing order) and writes +0 for empty segments.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <unistd.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vnp.h"
#include "vnp_batch.hpp"
#include "vnp_internal.hpp"
#include "vnp_nodes_p.hpp"

namespace vnp {

// ---------------------------------------------------------------------------------
// Segment descriptors
// ---------------------------------------------------------------------------------
// A descriptor gives, for segment s: len(s), base(x, s) (the address of its logical
// element 0), inc(s) (the stride between logical elements) and ok(s, n_total) (the
// segment lies inside the buffer the caller declared).
struct SegOffsets {  // segment s = x[off[s] .. off[s+1])
    static constexpr bool contiguous = true;  // unit stride, element-aligned when x is
    const int64_t *off;
    __device__ int64_t len(int64_t s) const
    {
        const int64_t l = off[s + 1] - off[s];
        return l > 0 ? l : 0;
    }
    template <typename T>
    __device__ const T *base(const T *x, int64_t s) const { return x + off[s]; }
    __device__ int64_t inc(int64_t) const { return 1; }
    __device__ bool ok(int64_t s, int64_t n_total) const
    {
        const int64_t l = len(s);
        return l == 0 || (off[s] >= 0 && off[s] <= n_total - l);
    }
};

struct SegCols {  // column s of a column-major matrix: x[s * lda .. s * lda + m)
    static constexpr bool contiguous = true;
    int64_t lda, m;
    __device__ int64_t len(int64_t) const { return m; }
    template <typename T>
    __device__ const T *base(const T *x, int64_t s) const { return x + s * lda; }
    __device__ int64_t inc(int64_t) const { return 1; }
    __device__ bool ok(int64_t, int64_t) const { return true; }
};

struct SegList {  // independent requests: len[s] elements at ptr[s] with stride inc[s]
    static constexpr bool contiguous = false;
    const void *const *ptr;  // address of logical element 0 (already moved for inc < 0)
    const int64_t *lens;
    const int64_t *incs;
    __device__ int64_t len(int64_t s) const { return lens[s] > 0 ? lens[s] : 0; }
    template <typename T>
    __device__ const T *base(const T *, int64_t s) const { return static_cast<const T *>(ptr[s]); }
    __device__ int64_t inc(int64_t s) const { return incs[s]; }
    __device__ bool ok(int64_t, int64_t) const { return true; }
};

// Runs of a segment of `tiles` tiles: 2^L tiles each, L the smallest at or above the launch's
// lwt that leaves at most MAX_RUNS runs (so the finish reduces at most 8 chunks of run
// roots per segment; a very long segment is spread over waves in larger runs).  Any run
// size gives the same tree.
constexpr int64_t MAX_RUNS = 4096;
__host__ __device__ inline int seg_lwt(int64_t tiles, int lwt)
{
    while (lwt < MAX_LWT && ((tiles + ((int64_t)1 << lwt) - 1) >> lwt) > MAX_RUNS) ++lwt;
    return lwt;
}

template <typename T>
__device__ __forceinline__ int64_t runs_of(int64_t len, int lwt)
{
    constexpr int64_t TE = tile_elems<T>();
    const int64_t tiles = (len + TE - 1) / TE;
    const int sl = seg_lwt(tiles, lwt);
    return (tiles + ((int64_t)1 << sl) - 1) >> sl;
}

// ---------------------------------------------------------------------------------
// Setup: item_off[k] = number of items before processing position k (exclusive scan of
// the run counts over the order), item_off[nseg] = total; res[s] = +0 for empty s.
// One block of 1024 threads.
// ---------------------------------------------------------------------------------
// Segments reaching outside [0, n_total), or more items than the workspace holds
// (items_cap), make every result NaN and enqueue no work.
template <typename T, class Seg>
__global__ void __launch_bounds__(1024)
    batched_setup_kernel(Seg seg, int64_t nseg, const int32_t *order, int lwt, int64_t n_total, int64_t items_cap,
                         int64_t *item_off, T *res)
{
    // passes of SB positions: coalesced loads (thread t takes positions t, t + 1024, ...),
    // run counts in LDS, each thread scans a contiguous chunk of PER there (an inclusive
    // scan within each wave by shuffles, then the wave totals in order), coalesced stores.
    // With n_total <= VNP_MAX_N a segment has at most 2^15 runs, so counts and offsets
    // within a pass fit 32 bits.
    constexpr int SB = 8192, PER = SB / 1024;
    __shared__ int32_t runs[SB];
    __shared__ int32_t wave_total[1024 / WAVE];
    __shared__ int bad;
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE, nw = blockDim.x / WAVE;
    if (t == 0) bad = 0;
    bool any_bad = false;
    int64_t carry = 0;
    for (int64_t base = 0; base < nseg; base += SB) {
        int64_t sg[PER], len[PER];
        bool ok[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int64_t k = base + t + j * 1024;
            const int64_t kc = k < nseg ? k : nseg - 1;
            sg[j] = order ? order[kc] : kc;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            len[j] = seg.len(sg[j]);
            ok[j] = seg.ok(sg[j], n_total);
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const bool in = base + t + j * 1024 < nseg;
            if (in && len[j] == 0) res[sg[j]] = T(0);
            any_bad = any_bad || (in && !ok[j]);
            // a segment outside the buffer counts no runs (its length is not bounded; the
            // launch is rejected below), so the 32-bit pass sums cannot overflow
            runs[t + j * 1024] = in && ok[j] ? (int32_t)runs_of<T>(len[j], lwt) : 0;
        }
        __syncthreads();
        int32_t c[PER], sum = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            c[j] = runs[t * PER + j];
            sum += c[j];
        }
        int32_t incl = sum;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int32_t v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane == WAVE - 1) wave_total[wv] = incl;
        __syncthreads();
        int32_t run = incl - sum, tot = 0;
        for (int w = 0; w < nw; ++w) {
            const int32_t wt = wave_total[w];
            if (w < wv) run += wt;
            tot += wt;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {  // exclusive offsets within the pass, in place
            runs[t * PER + j] = run;
            run += c[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int64_t k = base + t + j * 1024;
            if (k < nseg) item_off[k] = carry + runs[t + j * 1024];
        }
        carry += tot;
        __syncthreads();  // runs and wave_total are reused by the next pass
    }
    if (any_bad) bad = 1;
    __syncthreads();
    if (bad || carry > items_cap) {
        for (int64_t k = t; k < nseg; k += blockDim.x) res[order ? order[k] : k] = T(__builtin_nan(""));
        if (t == 0) item_off[nseg] = 0;
    } else if (t == 0) {
        item_off[nseg] = carry;
    }
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// Tree over r[0..cnt) (zero-padded to a power of two) by one wave; every lane gets the
// root.  Each pass reduces aligned chunks of 512 (8 per lane, then the lanes) to their
// roots and writes chunk k's root to r[k] (r[k] lies in or before chunk k, whose values
// are already read), until one value is left; with node(a, 0) = a the passes give the
// same value as one perfect tree over the zero-padded r.  r is overwritten.
template <class Node>
__device__ typename Node::T wave_finish(const Node &nd, typename Node::T *r, int64_t cnt, int lane)
{
    using T = typename Node::T;
    cnt = uniform64(cnt);
    while (cnt > 1) {
        const int64_t nck = (cnt + 511) / 512;
        for (int64_t ck = 0; ck < nck; ++ck) {
            const int64_t b0 = ck * 512 + lane * 8;
            T e[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool in = b0 + j < cnt;  // branch-free (see LoadGeneric)
                const T v = r[in ? b0 + j : 0];
                e[j] = in ? v : T(0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) e[j] = nd.node(e[2 * j], e[2 * j + 1]);
            e[0] = nd.node(e[0], e[1]);
            e[2] = nd.node(e[2], e[3]);
            const T t = uniform(lane_tree(nd, nd.node(e[0], e[2]), lane));
            // all lanes have read chunk ck (the cross-lane steps above need every lane's
            // value); every lane stores the same root
            r[ck] = t;
        }
        cnt = nck;
        // the next pass reads this wave's own stores
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    return uniform(r[0]);
}

// ---------------------------------------------------------------------------------
// Streaming kernel: items -> run roots (a segment of one run: its result).
// ---------------------------------------------------------------------------------
constexpr int COARSE_MAX = 4096;  // LDS entries of the item-offset index (32 KiB)

// GEN: segments may be strided or not element-aligned (the generic loader is compiled
// in); without it every segment takes the vector-load path, which needs fewer registers.
// Waves per SIMD the streaming kernel's registers must allow: 4 for the binary64 p node
// (at most 128 VGPRs, which its contiguous variants fit without spilling; uncapped it takes
// 184 and runs 2 waves per SIMD), 1 (no cap beyond the block size) otherwise.  The
// binary32 p node would spill hundreds of registers under the same cap.
template <class Node>
struct BatchedWavesPerEU {
    static constexpr int value = 1;
};
template <>
struct BatchedWavesPerEU<LpNode<double>> {
    static constexpr int value = 4;
};

template <class Node, class Seg, int U, bool GEN>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(BatchedWavesPerEU<Node>::value)))
    batched_kernel(Node nd, Seg seg, const typename Node::T *x, int64_t nseg, const int32_t *order,
                   const int64_t *item_off, int lwt, typename Node::T *roots, typename Node::T *res)
{
    using T = typename Node::T;
    constexpr int64_t TE = tile_elems<T>();
    node_prologue(nd);
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t total = item_off[nseg];
    const int wpb = (int)(blockDim.x / WAVE);
    const int64_t nwaves = (int64_t)gridDim.x * wpb;
    // Coarse index of the item offsets in LDS: every stride-th entry (at most
    // COARSE_MAX), so finding an item's segment takes LDS reads plus log2(stride)
    // global reads.
    extern __shared__ int64_t s_coarse[];
    const int64_t stride = (nseg + COARSE_MAX - 1) / COARSE_MAX;  // >= 1
    const int ncoarse = (int)((nseg + stride - 1) / stride);      // entries k = j * stride < nseg
    for (int j = threadIdx.x; j < ncoarse; j += blockDim.x) s_coarse[j] = item_off[(int64_t)j * stride];
    __syncthreads();
    for (int64_t item = (int64_t)blockIdx.x * wpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
         item < total; item += nwaves) {
        // processing position k: the last k with item_off[k] <= item (item < total)
        int jlo = 0, jhi = ncoarse - 1;
        while (jlo < jhi) {
            const int mid = (jlo + jhi + 1) >> 1;
            if (s_coarse[mid] <= item)
                jlo = mid;
            else
                jhi = mid - 1;
        }
        int64_t lo = (int64_t)jlo * stride;
        int64_t hi = lo + stride - 1 < nseg - 1 ? lo + stride - 1 : nseg - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (item_off[mid] <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t k = lo;
        const int64_t s = order ? order[k] : k;
        const int64_t r = item - item_off[k];
        const int64_t len = seg.len(s), inc = seg.inc(s);
        const int64_t ntiles = (len + TE - 1) / TE;
        const int sl = seg_lwt(ntiles, lwt);
        const int64_t nruns = (ntiles + ((int64_t)1 << sl) - 1) >> sl;
        const T *xs = seg.base(x, s);
        T root;
        if constexpr (GEN) {
            if (inc == 1 && (((uintptr_t)xs) % sizeof(T)) == 0)
                root = wave_root<Node, U, true>(nd, xs, len, real_stride(1), r << sl, ntiles, sl, lane);
            else
                root = wave_root<Node, U, false>(nd, xs, len, real_stride(inc), r << sl, ntiles, sl, lane);
        } else {
            root = wave_root<Node, U, true>(nd, xs, len, real_stride(1), r << sl, ntiles, sl, lane);
        }
        // every lane stores the same value
        if (nruns == 1)
            res[s] = nd.finish(root);
        else
            roots[item] = root;
    }
}

// Small request batches: one block of TILE_WAVES waves per item of one tile (lwt = 0),
// the tile reduced cooperatively (tile_root_block); results and run roots as in the
// streaming kernel.
template <class Node, class Seg>
__global__ void __launch_bounds__(TILE_WAVES * WAVE)
    batched_tile_kernel(Node nd, Seg seg, const typename Node::T *x, int64_t nseg, const int64_t *item_off,
                        typename Node::T *roots, typename Node::T *res)
{
    using T = typename Node::T;
    constexpr int64_t TE = tile_elems<T>();
    __shared__ typename Node::R part[Vec<T>::N][TILE_WAVES][WAVE];
    node_prologue(nd);
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t item = blockIdx.x;  // every thread searches the same item (block-uniform)
    int64_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (item_off[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t k = lo, s = k;
    const int64_t r = item - item_off[k];
    const int64_t len = seg.len(s), inc = seg.inc(s);
    const int64_t ntiles = (len + TE - 1) / TE;
    const T *xs = seg.base(x, s);
    T root;
    if (inc == 1 && (((uintptr_t)xs) % sizeof(T)) == 0)
        root = tile_root_block<Node, true>(nd, xs, len, real_stride(1), r, lane, w, part);
    else
        root = tile_root_block<Node, false>(nd, xs, len, real_stride(inc), r, lane, w, part);
    if (w == 0 && lane == 0) {
        if (ntiles == 1)
            res[s] = nd.finish(root);
        else
            roots[item] = root;
    }
}

// Finish kernel: one wave per segment of several runs reduces its run roots (written by
// the streaming kernel before it on the same stream) by the fixed tree.
template <class Node>
__global__ void __launch_bounds__(256)
    batched_finish_kernel(Node nd, int64_t nseg, const int32_t *order, const int64_t *item_off,
                          typename Node::T *roots, typename Node::T *res)
{
    node_prologue(nd);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = (int)(blockDim.x / WAVE);
    const int64_t nwaves = (int64_t)gridDim.x * wpb;
    const int64_t total = uniform64(item_off[nseg]);  // 0 when the setup rejected the offsets
    for (int64_t k = (int64_t)blockIdx.x * wpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)); k < nseg;
         k += nwaves) {
        const int64_t a = uniform64(item_off[k]), b = uniform64(item_off[k + 1]);
        if (b - a > 1 && b <= total) {
            const int64_t s = order ? order[k] : k;
            res[s] = nd.finish(wave_finish(nd, roots + a, b - a, lane));
        }
    }
}

// Fixed tree over vals[0..count) (the perfect binary tree over the zero-padded index, as
// block_finish evaluates it) by one block; vals is overwritten.
template <class Node>
__global__ void __launch_bounds__(256)
    values_finish_kernel(Node nd, typename Node::T *vals, int64_t count, typename Node::T *res)
{
    __shared__ typename Node::T sbuf[256];
    node_prologue(nd);
    const typename Node::T root = block_finish(nd, vals, count, sbuf);
    if (threadIdx.x == 0) *res = nd.finish(root);
}

// Stage kernel of a request batch: copies the batch's descriptor words from host-mapped
// memory to device memory.
__global__ void __launch_bounds__(1024)
    stage_kernel(const unsigned long long *src, unsigned long long *dst, int64_t nwords)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) dst[i] = src[i];
}

// Admission by copy (the server): copy c moves n_c logical elements of esz_c bytes,
// element k at src_c + k inc_c (src_c: logical element 0, inc_c may be negative), to the
// contiguous pool block dst_c.  tab: {src, dst, n, inc, esz} per copy, then chunk_off
// (ncopy + 1 prefix sums of the copies' COPY_CHUNK-element chunks); one block per chunk.
constexpr int64_t COPY_CHUNK = 4096;

__global__ void __launch_bounds__(256) gather_kernel(const int64_t *tab, int64_t ncopy)
{
    const int64_t *chunk_off = tab + 5 * ncopy;
    const int64_t b = blockIdx.x;
    int64_t lo = 0, hi = ncopy - 1;  // the copy whose chunks hold b (block-uniform search)
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_off[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t *d = tab + 5 * lo;
    const char *src = reinterpret_cast<const char *>(d[0]);
    char *dst = reinterpret_cast<char *>(d[1]);
    const int64_t n = d[2], inc = d[3], esz = d[4];
    const int64_t k0 = (b - chunk_off[lo]) * COPY_CHUNK;
    const int64_t k1 = k0 + COPY_CHUNK < n ? k0 + COPY_CHUNK : n;
    if (esz == 8) {
        for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
            reinterpret_cast<uint64_t *>(dst)[k] = *reinterpret_cast<const uint64_t *>(src + k * inc * 8);
    } else {
        for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
            reinterpret_cast<uint32_t *>(dst)[k] = *reinterpret_cast<const uint32_t *>(src + k * inc * 4);
    }
}

// ---------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------
static int ensure_batch_ws(BatchWorkspace &w, size_t roots_bytes, size_t nseg, hipStream_t st)
{
    hipError_t e;
    const bool grow_roots = w.roots_cap < roots_bytes, grow_items = w.item_cap < nseg + 1;
    if ((grow_roots && w.roots) || (grow_items && w.item_off)) {
        e = hipStreamSynchronize(st);  // old buffers may be in use by queued work
        if (e != hipSuccess) return (int)e;
    }
    if (grow_roots) {
        if (w.roots) (void)hipFree(w.roots);
        w.roots = nullptr;
        const size_t b = std::max<size_t>(std::max<size_t>(roots_bytes, 2 * w.roots_cap), 1 << 16);
        e = hipMalloc(&w.roots, b);
        if (e != hipSuccess) return (int)e;
        w.roots_cap = b;
    }
    if (grow_items) {
        if (w.item_off) (void)hipFree(w.item_off);
        w.item_off = nullptr;
        const size_t c = std::max<size_t>(std::max<size_t>(nseg + 1, 2 * w.item_cap), 4096);
        e = hipMalloc(reinterpret_cast<void **>(&w.item_off), c * sizeof(int64_t));
        if (e != hipSuccess) return (int)e;
        w.item_cap = c;
    }
    return 0;
}

static int ensure_vals(BatchWorkspace &w, size_t bytes, hipStream_t st)
{
    if (w.vals_cap >= bytes) return 0;
    hipError_t e;
    if (w.vals) {
        e = hipStreamSynchronize(st);  // the old buffer may be in use by queued work
        if (e != hipSuccess) return (int)e;
        (void)hipFree(w.vals);
        w.vals = nullptr;
        w.vals_cap = 0;
    }
    const size_t b = std::max<size_t>(bytes, 1 << 16);
    e = hipMalloc(&w.vals, b);
    if (e != hipSuccess) return (int)e;
    w.vals_cap = b;
    return 0;
}

static void free_batch_ws(BatchWorkspace &w)
{
    if (w.roots) (void)hipFree(w.roots);
    if (w.item_off) (void)hipFree(w.item_off);
    if (w.vals) (void)hipFree(w.vals);
    w = BatchWorkspace{};
}

static std::mutex g_bws_mu;
static std::map<std::pair<int, void *>, BatchWorkspace> g_bws;

int release_batch_workspaces()
{
    std::lock_guard<std::mutex> lk(g_bws_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto it = g_bws.begin(); it != g_bws.end();) {
        if (it->first.first == dev) {
            free_batch_ws(it->second);
            it = g_bws.erase(it);
        } else {
            ++it;
        }
    }
    return 0;
}

static int cus() { return device_cus(); }

// One tile per work item, several rounds of resident blocks: the direct calls know no host
// lengths (no longest-first order), and the round-robin items balance best at the finest
// grain with several rounds.  Measured on the 8192 log-uniform FP64 segments, p = 2 (one
// tile per item): 0.85 ms with one round of resident blocks, 0.79-0.80 ms with four,
// 0.787 ms with eight rounds of 4-wave blocks; four tiles per item with one round: 0.92 ms.
// The p node fills its LDS tables in every block, so it keeps four rounds of 8-wave
// blocks: p = 3 took 1.49 ms with those and 1.76 ms with eight rounds of 4-wave blocks.
static BatchShape default_batch_shape(bool table_node)
{
    return table_node ? BatchShape{0, 8, cus() * 8} : BatchShape{0, 4, cus() * 32};
}

template <class Node>
struct TableNode {
    static constexpr bool value = false;
};
template <typename T>
struct TableNode<LpNode<T>> {
    static constexpr bool value = true;
};

static size_t coarse_bytes(int64_t nseg)
{
    const int64_t stride = (nseg + COARSE_MAX - 1) / COARSE_MAX;
    return sizeof(int64_t) * (size_t)((nseg + stride - 1) / stride);
}

// Blocks of wpb waves of kernel k that are resident on one compute unit at once (with
// the largest coarse index).  Items are assigned to waves statically; a grid of several
// rounds of resident blocks lets the hardware give the later blocks to the compute units
// that finish first, which evens out their speeds, so grids are capped at eight rounds.
// Cached per kernel instantiation and block size.
template <typename K>
static int resident_blocks(K k, int wpb)
{
    static int cache[17] = {};
    if (wpb < 1 || wpb > 16) return 1;
    if (!cache[wpb]) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, wpb * WAVE, sizeof(int64_t) * COARSE_MAX) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        cache[wpb] = nb;
    }
    return cache[wpb];
}

template <class Node, class Seg, bool GEN>
static int launch_streaming(const Node &nd, const Seg &seg, const typename Node::T *x, int64_t nseg,
                            const int32_t *order, const int64_t *item_off, int lwt, int wpb, int blocks, void *roots,
                            typename Node::T *res, hipStream_t st)
{
    using T = typename Node::T;
    auto k = batched_kernel<Node, Seg, RowsInFlight<Node>::value, GEN>;
    const int fit = cus() * resident_blocks(k, wpb);
    if (blocks > 8 * fit) blocks = 8 * fit;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(wpb * WAVE), coarse_bytes(nseg), st, nd, seg, x, nseg, order, item_off,
                       lwt, static_cast<T *>(roots), res);
    return blocks;
}

template <class Node>
static void launch_finish(const Node &nd, int64_t nseg, const int32_t *order, const int64_t *item_off, void *roots,
                          typename Node::T *res, hipStream_t st)
{
    using T = typename Node::T;
    // one wave per position up to four rounds of 16 waves per compute unit: each position
    // is a chain of dependent loads, which other waves overlap
    const int64_t waves = std::min<int64_t>(nseg, (int64_t)cus() * 64);
    const int wpb = waves >= 4 ? 4 : 1;
    const int blocks = (int)((waves + wpb - 1) / wpb);
    hipLaunchKernelGGL((batched_finish_kernel<Node>), dim3(blocks), dim3(wpb * WAVE), 0, st, nd, nseg, order, item_off,
                       static_cast<T *>(roots), res);
}

// Whether a segment of the workload can span more than one run of 2^lwt tiles (then the
// finish kernel is needed).
template <typename T>
static bool may_multi(const SegOffsets &, int) { return true; }
template <typename T>
static bool may_multi(const SegCols &c, int lwt)
{
    constexpr int64_t TE = tile_elems<T>();
    const int64_t tiles = (c.m + TE - 1) / TE;
    return tiles > ((int64_t)1 << seg_lwt(tiles, lwt));
}

// Enqueue setup, streaming and (if needed) finish kernels for one batched workload (no
// allocation: ws must hold roots for nseg + total_elems / tile + 1 items).  *used gets
// the shape actually launched (blocks capped to what is resident).
template <class Node, class Seg>
static int enqueue_batched(const Node &nd, const Seg &seg, const typename Node::T *x, int64_t nseg,
                           int64_t n_total, const int32_t *order, const BatchShape &sh, BatchWorkspace &ws,
                           typename Node::T *res, hipStream_t st, BatchShape *used = nullptr)
{
    using T = typename Node::T;
    const int64_t items_cap = (int64_t)(ws.roots_cap / sizeof(T));
    hipLaunchKernelGGL((batched_setup_kernel<T, Seg>), dim3(1), dim3(1024), 0, st, seg, nseg, order, sh.lwt,
                       n_total, items_cap, ws.item_off, res);
    int blocks;
    if (Seg::contiguous && ((uintptr_t)x % sizeof(T)) == 0)
        blocks = launch_streaming<Node, Seg, false>(nd, seg, x, nseg, order, ws.item_off, sh.lwt, sh.wpb, sh.blocks,
                                                    ws.roots, res, st);
    else
        blocks = launch_streaming<Node, Seg, true>(nd, seg, x, nseg, order, ws.item_off, sh.lwt, sh.wpb, sh.blocks,
                                                   ws.roots, res, st);
    if (may_multi<T>(seg, sh.lwt)) launch_finish(nd, nseg, order, ws.item_off, ws.roots, res, st);
    if (used) *used = BatchShape{sh.lwt, sh.wpb, blocks};
    return (int)hipGetLastError();
}

template <class Node, class Seg>
static int run_batched(const Node &nd, const Seg &seg, const typename Node::T *x, int64_t nseg, int64_t total_elems,
                       typename Node::T *res, void *stream)
{
    using T = typename Node::T;
    if (nseg == 0) return 0;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const BatchShape sh = default_batch_shape(TableNode<Node>::value);
    const int64_t items_cap = nseg + (total_elems + tile_elems<T>() - 1) / tile_elems<T>() + 1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    std::lock_guard<std::mutex> lk(g_bws_mu);
    BatchWorkspace &ws = g_bws[std::make_pair(dev, stream)];
    int rc = ensure_batch_ws(ws, sizeof(T) * (size_t)items_cap, (size_t)nseg, st);
    if (rc) return rc;
    return enqueue_batched(nd, seg, x, nseg, total_elems, nullptr, sh, ws, res, st);
}

template <typename T, class Seg>
static int run_batched_p(const Seg &seg, const T *x, int64_t nseg, int64_t total, T p, T *res, void *stream,
                         T cutoff)
{
    if (p == T(2)) return run_batched(HypNode<T>{}, seg, x, nseg, total, res, stream);
    if (p == T(1)) return run_batched(SumNode<T>{}, seg, x, nseg, total, res, stream);
    if (__builtin_isinf(p) || p >= cutoff) return run_batched(MaxNode<T>{}, seg, x, nseg, total, res, stream);
    LpNode<T> nd;
    const int rc = make_lp_node<T>(p, &nd);
    return rc ? rc : run_batched(nd, seg, x, nseg, total, res, stream);
}

// Norm of an m x ncols array with leading dimension lda > m (Sect. 3.1): column norms
// into the workspace, then the fixed tree over them.
template <class Node>
static int run_mat(const Node &nd, int64_t m, int64_t ncols, const typename Node::T *A, int64_t lda,
                   typename Node::T *res, void *stream)
{
    using T = typename Node::T;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const BatchShape sh = default_batch_shape(TableNode<Node>::value);
    const int64_t total = (ncols - 1) * lda + m;
    const int64_t items_cap = ncols + (total + tile_elems<T>() - 1) / tile_elems<T>() + 1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    std::lock_guard<std::mutex> lk(g_bws_mu);
    BatchWorkspace &ws = g_bws[std::make_pair(dev, stream)];
    int rc = ensure_batch_ws(ws, sizeof(T) * (size_t)items_cap, (size_t)ncols, st);
    if (!rc) rc = ensure_vals(ws, sizeof(T) * (size_t)ncols, st);
    if (rc) return rc;
    T *vals = static_cast<T *>(ws.vals);
    rc = enqueue_batched(nd, SegCols{lda, m}, A, ncols, total, nullptr, sh, ws, vals, st);
    if (rc) return rc;
    hipLaunchKernelGGL((values_finish_kernel<Node>), dim3(1), dim3(256), 0, st, nd, vals, ncols, res);
    return (int)hipGetLastError();
}

template <typename T>
static int run_mat_p(int64_t m, int64_t ncols, const T *A, int64_t lda, T p, T *res, void *stream, T cutoff)
{
    if (p == T(2)) return run_mat(HypNode<T>{}, m, ncols, A, lda, res, stream);
    if (p == T(1)) return run_mat(SumNode<T>{}, m, ncols, A, lda, res, stream);
    if (__builtin_isinf(p) || p >= cutoff) return run_mat(MaxNode<T>{}, m, ncols, A, lda, res, stream);
    LpNode<T> nd;
    const int rc = make_lp_node<T>(p, &nd);
    return rc ? rc : run_mat(nd, m, ncols, A, lda, res, stream);
}

// ---------------------------------------------------------------------------------
// Request batches (the server): classes of independent requests, item offsets from the
// host, descriptors staged from host-mapped memory, results written to host-mapped
// memory, one launch per class with a grid sized to its items.
// ---------------------------------------------------------------------------------
template <typename T>
static int64_t host_runs(int64_t len, int lwt)
{
    constexpr int64_t TE = tile_elems<T>();
    const int64_t tiles = len > 0 ? (len + TE - 1) / TE : 0;
    const int sl = seg_lwt(tiles, lwt);
    return (tiles + ((int64_t)1 << sl) - 1) >> sl;
}

template <typename T>
static int class_items(const int64_t *lens, int64_t n, int64_t *item_off)
{
    constexpr int64_t TE = tile_elems<T>();
    int64_t tiles = 0;
    for (int64_t i = 0; i < n; ++i) tiles += lens[i] > 0 ? (lens[i] + TE - 1) / TE : 0;
    // one tile per item while that gives at most 8 items per resident wave, so a small
    // batch spreads over the whole GPU; longer runs per item for large batches
    const int64_t maxw = (int64_t)cus() * 16;
    int lwt = 0;
    while (lwt < 3 && (tiles >> lwt) > 8 * maxw) ++lwt;
    int64_t run = 0;
    for (int64_t i = 0; i < n; ++i) {
        item_off[i] = run;
        run += host_runs<T>(lens[i], lwt);
    }
    item_off[n] = run;
    return lwt;
}

int request_class_items(int dtype, const int64_t *lens, int64_t n, int64_t *item_off)
{
    return dtype == VNP_F32 ? class_items<float>(lens, n, item_off) : class_items<double>(lens, n, item_off);
}

template <class Node>
static void launch_class(const Node &nd, const SegList &seg, const RequestClass &k, const int64_t *item_off,
                         void *roots, typename Node::T *res, hipStream_t st)
{
    using T = typename Node::T;
    if (k.lwt == 0 && k.items <= 4 * (int64_t)cus()) {
        // few tiles: one block of TILE_WAVES waves per tile
        hipLaunchKernelGGL((batched_tile_kernel<Node, SegList>), dim3((unsigned)k.items), dim3(TILE_WAVES * WAVE), 0,
                           st, nd, seg, (const T *)nullptr, k.n, item_off, static_cast<T *>(roots), res);
    } else {
        // one wave per item up to what is resident
        const int64_t waves = std::min<int64_t>(k.items, (int64_t)cus() * 16);
        const int wpb = waves >= 4 * (int64_t)cus() ? 4 : 1;
        const int blocks = (int)((waves + wpb - 1) / wpb);
        (void)launch_streaming<Node, SegList, true>(nd, seg, nullptr, k.n, nullptr, item_off, k.lwt, wpb, blocks,
                                                    roots, res, st);
    }
    if (k.multi) launch_finish(nd, k.n, nullptr, item_off, roots, res, st);
}

template <typename T>
static int launch_class_p(const SegList &seg, const RequestClass &k, const int64_t *item_off, void *roots, T *res,
                          T cutoff, hipStream_t st)
{
    const T pt = (T)k.p;
    if (pt == T(2)) {
        launch_class(HypNode<T>{}, seg, k, item_off, roots, res, st);
    } else if (pt == T(1)) {
        launch_class(SumNode<T>{}, seg, k, item_off, roots, res, st);
    } else if (__builtin_isinf(pt) || pt >= cutoff) {
        launch_class(MaxNode<T>{}, seg, k, item_off, roots, res, st);
    } else {
        LpNode<T> nd;
        const int rc = make_lp_node<T>(pt, &nd);
        if (rc) return rc;
        launch_class(nd, seg, k, item_off, roots, res, st);
    }
    return 0;
}

// One copy, its descriptor in the kernel arguments (a batch of one request).
__global__ void __launch_bounds__(256)
    gather1_kernel(const char *src, char *dst, int64_t n, int64_t inc, int64_t esz)
{
    const int64_t k0 = (int64_t)blockIdx.x * COPY_CHUNK;
    const int64_t k1 = k0 + COPY_CHUNK < n ? k0 + COPY_CHUNK : n;
    if (esz == 8) {
        for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
            reinterpret_cast<uint64_t *>(dst)[k] = *reinterpret_cast<const uint64_t *>(src + k * inc * 8);
    } else {
        for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
            reinterpret_cast<uint32_t *>(dst)[k] = *reinterpret_cast<const uint32_t *>(src + k * inc * 4);
    }
}

int64_t copy_chunks(int64_t n) { return (n + COPY_CHUNK - 1) / COPY_CHUNK; }

int enqueue_copy1(const void *src, void *dst, int64_t n, int64_t inc, int64_t esz, hipStream_t st)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(gather1_kernel, dim3((unsigned)copy_chunks(n)), dim3(256), 0, st,
                       static_cast<const char *>(src), static_cast<char *>(dst), n, inc, esz);
    return (int)hipGetLastError();
}

int enqueue_request_batch(const void *h_src, void *d_desc, int64_t nreq, const RequestClass *cls, int ncls,
                          int64_t ncopy, int64_t nchunks, double *res_d, float *res_s, BatchWorkspace &ws,
                          hipStream_t st)
{
    if (nreq <= 0 || ncls <= 0) return 0;
    int64_t roots = 0;
    for (int c = 0; c < ncls; ++c) roots += cls[c].items;
    int rc = ensure_batch_ws(ws, 8 * (size_t)(roots > 0 ? roots : 1), (size_t)nreq, st);
    if (rc) return rc;
    const int64_t nwords = 3 * nreq + nreq + ncls;
    const int64_t cwords = ncopy > 0 ? 6 * ncopy + 1 : 0;  // copy table after the item offsets
    hipLaunchKernelGGL(stage_kernel, dim3(1), dim3(1024), 0, st, static_cast<const unsigned long long *>(h_src),
                       static_cast<unsigned long long *>(d_desc), nwords + cwords);
    if (ncopy > 0 && nchunks > 0)
        hipLaunchKernelGGL(gather_kernel, dim3((unsigned)nchunks), dim3(256), 0, st,
                           static_cast<const int64_t *>(d_desc) + nwords, ncopy);
    const int64_t *w = static_cast<const int64_t *>(d_desc);
    const void *const *ptrs = reinterpret_cast<const void *const *>(w);
    int64_t roots_off = 0;
    for (int c = 0; c < ncls; ++c) {
        const RequestClass &k = cls[c];
        if (k.items == 0) continue;
        const SegList seg{ptrs + k.a, w + nreq + k.a, w + 2 * nreq + k.a};
        const int64_t *item_off = w + 3 * nreq + k.a + c;
        void *rt = static_cast<char *>(ws.roots) + 8 * roots_off;
        rc = k.dtype == VNP_F32 ? launch_class_p<float>(seg, k, item_off, rt, res_s + k.a, 0x1p24f, st)
                                : launch_class_p<double>(seg, k, item_off, rt, res_d + k.a, 0x1p53, st);
        if (rc) return rc;
        roots_off += k.items;
    }
    return (int)hipGetLastError();
}

void release_batch_ws(BatchWorkspace &w) { free_batch_ws(w); }

// ---------------------------------------------------------------------------------
// Plans: autotuned shape + captured graph
// ---------------------------------------------------------------------------------
struct PlanImpl {
    int dtype = 0;
    double p = 2.0;
    int64_t nseg = 0, n_total = 0;
    const int64_t *offsets = nullptr;
    const void *x = nullptr;
    void *res = nullptr;
    int32_t *order = nullptr;  // device, processing order (longest segments first) or null
    double *lp_rr = nullptr;   // device, the plan's own copy of its p-node table (p-norm plans)
    BatchShape shape{};
    BatchWorkspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

template <class Node>
static int plan_enqueue(const Node &nd, PlanImpl &P, const BatchShape &sh, hipStream_t st, BatchShape *used)
{
    using T = typename Node::T;
    return enqueue_batched(nd, SegOffsets{P.offsets}, static_cast<const T *>(P.x), P.nseg, P.n_total, P.order, sh,
                           P.ws, static_cast<T *>(P.res), st, used);
}

// The p node of a p-norm plan.  The captured graph keeps the table pointer, so the plan
// owns a copy of the table (the shared one is released by vnp_finalize); it is made
// before the capture (plan_prepare).
template <typename T>
static int plan_lp_node(PlanImpl &P, T p, LpNode<T> *nd)
{
    int rc = make_lp_node<T>(p, nd);
    if (rc) return rc;
    if (!P.lp_rr) {
        const size_t bytes = 2 * LP_POW_N * sizeof(double);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&P.lp_rr), bytes);
        if (e == hipSuccess) e = hipMemcpy(P.lp_rr, nd->rr, bytes, hipMemcpyDeviceToDevice);
        if (e != hipSuccess) return (int)e;
    }
    nd->rr = P.lp_rr;
    return 0;
}

template <typename T>
static int plan_prepare_p(PlanImpl &P, T cutoff)
{
    const T p = (T)P.p;
    if (p == T(2) || p == T(1) || __builtin_isinf(p) || p >= cutoff) return 0;
    LpNode<T> nd;
    return plan_lp_node<T>(P, p, &nd);
}

template <typename T>
static int plan_enqueue_p(PlanImpl &P, const BatchShape &sh, hipStream_t st, T cutoff, BatchShape *used)
{
    const T p = (T)P.p;
    if (p == T(2)) return plan_enqueue(HypNode<T>{}, P, sh, st, used);
    if (p == T(1)) return plan_enqueue(SumNode<T>{}, P, sh, st, used);
    if (__builtin_isinf(p) || p >= cutoff) return plan_enqueue(MaxNode<T>{}, P, sh, st, used);
    LpNode<T> nd;
    const int rc = plan_lp_node<T>(P, p, &nd);
    return rc ? rc : plan_enqueue(nd, P, sh, st, used);
}

static int plan_enqueue_any(PlanImpl &P, const BatchShape &sh, hipStream_t st, BatchShape *used = nullptr)
{
    return P.dtype == VNP_F32 ? plan_enqueue_p<float>(P, sh, st, 0x1p24f, used)
                              : plan_enqueue_p<double>(P, sh, st, 0x1p53, used);
}

// ---------------------------------------------------------------------------------
// Autotune cache: the chosen shape per (device, dtype, node kind, size class, alignment,
// tree id), kept for the process and, when VNP_AUTOTUNE_CACHE names a file, in that file
// as JSON (read at the first lookup; after each new choice, merged with the file's current
// entries and written through a temporary file and a rename).  A shape never changes a
// result, so a stale or foreign entry can only cost time.
// ---------------------------------------------------------------------------------
struct TuneEntry {
    int lwt, wpb, blocks;
    double ms;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;
static bool g_tune_loaded = false;

static const char *tune_path()
{
    const char *p = getenv("VNP_AUTOTUNE_CACHE");
    return p && p[0] ? p : nullptr;
}

// Entry lines as tune_write writes them; anything else in the file is ignored, and so is
// an entry whose shape is outside the candidates.
static void tune_read(const char *path, std::map<std::string, TuneEntry> &out)
{
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[1024], key[512];
    while (fgets(line, sizeof line, f)) {
        TuneEntry e{};
        if (sscanf(line, " \"%511[^\"]\": {\"lwt\": %d, \"wpb\": %d, \"blocks\": %d, \"ms\": %lf}", key, &e.lwt,
                   &e.wpb, &e.blocks, &e.ms) == 5 &&
            e.lwt >= 0 && e.lwt <= 3 && (e.wpb == 4 || e.wpb == 8) && e.blocks > 0 && e.blocks <= (1 << 20))
            out[key] = e;
    }
    fclose(f);
}

static void tune_write(const char *path, const std::map<std::string, TuneEntry> &m)
{
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n  \"version\": 1,\n  \"entries\": {\n");
    size_t i = 0;
    for (const auto &kv : m)
        fprintf(f, "    \"%s\": {\"lwt\": %d, \"wpb\": %d, \"blocks\": %d, \"ms\": %.4f}%s\n", kv.first.c_str(),
                kv.second.lwt, kv.second.wpb, kv.second.blocks, kv.second.ms, ++i < m.size() ? "," : "");
    fprintf(f, "  }\n}\n");
    if (fclose(f) == 0 && rename(tmp.c_str(), path) == 0) return;
    remove(tmp.c_str());
}

static std::string tune_key(const PlanImpl &P)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    const bool f32 = P.dtype == VNP_F32;
    const double p = P.p, cutoff = f32 ? 0x1p24 : 0x1p53;
    const char *node = p == 2.0 ? "hypot" : p == 1.0 ? "sum" : (__builtin_isinf(p) || p >= cutoff) ? "max" : "p";
    auto lg = [](int64_t v) { return v > 0 ? 63 - __builtin_clzll((unsigned long long)v) : -1; };
    const bool aligned = ((uintptr_t)P.x % (f32 ? 4 : 8)) == 0;
    char buf[512];
    snprintf(buf, sizeof buf, "%s/%dcu|%s|%s|nseg2^%d|n2^%d|%s|tree%x", prop.gcnArchName, prop.multiProcessorCount,
             f32 ? "f32" : "f64", node, lg(P.nseg), lg(P.n_total), aligned ? "aligned" : "unaligned",
             vnp_tree_id(P.dtype));
    for (char *c = buf; *c; ++c)
        if (*c == '"' || *c == '\\' || *c < ' ') *c = '_';
    return std::string(buf);
}

static bool tune_lookup(const std::string &key, BatchShape *sh)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        if (const char *path = tune_path()) tune_read(path, g_tune);
    }
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *sh = BatchShape{it->second.lwt, it->second.wpb, it->second.blocks};
    return true;
}

static void tune_store(const std::string &key, const BatchShape &sh, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = TuneEntry{sh.lwt, sh.wpb, sh.blocks, ms};
    if (const char *path = tune_path()) {
        std::map<std::string, TuneEntry> merged;
        tune_read(path, merged);  // other processes' entries
        for (const auto &kv : g_tune) merged[kv.first] = kv.second;
        tune_write(path, merged);
    }
}

// Times candidate shapes (median of 5 launches each) and keeps the fastest.  Every shape
// computes the same tree, so the choice never changes a result.  mode 1 takes a cached
// choice when there is one; mode 2 always times and replaces it.
static int autotune(PlanImpl &P, hipStream_t st, int mode)
{
    const std::string key = tune_key(P);
    if (mode == 1 && !key.empty() && tune_lookup(key, &P.shape)) return 0;
    // work item size x block size x waves per CU (the waves that fit at once depend on
    // the kernel's registers; counts above them make later rounds; timing finds the best)
    std::vector<BatchShape> cands;
    for (int lwt : {0, 1, 2, 3})
        for (int wpb : {4, 8})
            for (int wpc : {16, 32, 64, 96, 128}) cands.push_back(BatchShape{lwt, wpb, cus() * wpc / wpb});
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return (int)hipErrorUnknown;
    float best = 1e30f;
    BatchShape best_s = P.shape;
    const char *lg = getenv("VNP_AUTOTUNE_LOG");  // set to 1: print every candidate's time
    const bool log = lg && lg[0] == '1';
    int rc = 0;
    std::vector<BatchShape> seen;
    for (const BatchShape &want : cands) {
        BatchShape c;
        rc = plan_enqueue_any(P, want, st, &c);  // warm-up; c: the shape launched (resident blocks)
        if (rc) break;
        bool dup = false;
        for (const BatchShape &o : seen) dup = dup || (o.lwt == c.lwt && o.wpb == c.wpb && o.blocks == c.blocks);
        if (dup) continue;
        seen.push_back(c);
        float t[5];
        for (int r = 0; r < 5 && !rc; ++r) {
            (void)hipEventRecord(a, st);
            rc = plan_enqueue_any(P, c, st);
            (void)hipEventRecord(b, st);
            if (hipEventSynchronize(b) != hipSuccess) rc = (int)hipErrorUnknown;
            (void)hipEventElapsedTime(&t[r], a, b);
        }
        if (rc) break;
        std::sort(t, t + 5);
        if (log)
            fprintf(stderr, "vnp autotune: tiles/item %d, waves/block %d, blocks %d: %.4f ms\n", 1 << c.lwt, c.wpb,
                    c.blocks, t[2]);
        if (t[2] < best) {
            best = t[2];
            best_s = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    P.shape = best_s;
    if (!rc && best < 1e30f && !key.empty()) tune_store(key, best_s, best);
    return rc;
}

static void plan_free(PlanImpl *P)
{
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->order) (void)hipFree(P->order);
    if (P->lp_rr) (void)hipFree(P->lp_rr);
    free_batch_ws(P->ws);
    delete P;
}

}  // namespace vnp

using namespace vnp;

struct vnp_plan {
    PlanImpl *impl;
};

extern "C" {

int vnp_plan_create(vnp_plan **plan, const vnp_plan_desc *d, void *stream)
{
    if (!plan) return -1;
    *plan = nullptr;
    if (!d || (d->dtype != VNP_F64 && d->dtype != VNP_F32) ||
        !(d->dtype == VNP_F32 ? p_ok((float)d->p) : p_ok(d->p)) || d->nseg < 0 || d->n_total < 0 ||
        (d->nseg > 0 && (!d->offsets || !d->res)) || (d->n_total > 0 && !d->x))
        return -2;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PlanImpl *P = new (std::nothrow) PlanImpl;
    if (!P) return (int)hipErrorOutOfMemory;
    P->dtype = d->dtype;
    P->p = d->p;
    P->nseg = d->nseg;
    P->n_total = d->n_total;
    P->offsets = d->offsets;
    P->x = d->x;
    P->res = d->res;
    {  // the generic-p node, as the plan's enqueue chooses it
        const double pp = d->p, cutoff = d->dtype == VNP_F32 ? 0x1p24 : 0x1p53;
        P->shape = default_batch_shape(!(pp == 2.0 || pp == 1.0 || __builtin_isinf(pp) || pp >= cutoff));
    }
    const int64_t te = d->dtype == VNP_F32 ? tile_elems<float>() : tile_elems<double>();
    const size_t esz = d->dtype == VNP_F32 ? 4 : 8;
    int rc = 0;
    if (d->h_offsets && d->nseg > 1) {  // longest segments first, so no long item starts late
        std::vector<int32_t> ord((size_t)d->nseg);
        std::iota(ord.begin(), ord.end(), 0);
        const int64_t *o = d->h_offsets;
        std::stable_sort(ord.begin(), ord.end(),
                         [o](int32_t u, int32_t v) { return o[u + 1] - o[u] > o[v + 1] - o[v]; });
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&P->order), ord.size() * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemcpy(P->order, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = (int)e;
    }
    const int64_t items_cap = d->nseg + (d->n_total + te - 1) / te + 1;
    if (!rc) rc = ensure_batch_ws(P->ws, esz * (size_t)items_cap, (size_t)(d->nseg > 0 ? d->nseg : 1), st);
    if (!rc) rc = P->dtype == VNP_F32 ? plan_prepare_p<float>(*P, 0x1p24f) : plan_prepare_p<double>(*P, 0x1p53);
    if (!rc && d->autotune && d->nseg > 0) rc = autotune(*P, st, d->autotune == 2 ? 2 : 1);
    if (!rc && d->nseg > 0) {
        // capture on a private stream (the legacy default stream cannot be captured)
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = plan_enqueue_any(*P, P->shape, cs);
            e = hipStreamEndCapture(cs, &P->graph);
            if (!rc && e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
        }
        if (cs) (void)hipStreamDestroy(cs);
        if (!rc && e != hipSuccess) rc = (int)e;
    }
    if (rc) {
        plan_free(P);
        return rc;
    }
    vnp_plan *h = new (std::nothrow) vnp_plan{P};
    if (!h) {
        plan_free(P);
        return (int)hipErrorOutOfMemory;
    }
    *plan = h;
    return 0;
}

int vnp_plan_exec(vnp_plan *plan, void *stream)
{
    if (!plan || !plan->impl) return -1;
    if (!plan->impl->exec) return 0;  // no segments
    return (int)hipGraphLaunch(plan->impl->exec, reinterpret_cast<hipStream_t>(stream));
}

int vnp_plan_destroy(vnp_plan *plan)
{
    if (!plan) return -1;
    plan_free(plan->impl);
    delete plan;
    return 0;
}

int vnp_plan_info(const vnp_plan *plan, int *blocks, int *waves, int *tiles_per_item)
{
    if (!plan || !plan->impl) return -1;
    if (blocks) *blocks = plan->impl->shape.blocks;
    if (waves) *waves = plan->impl->shape.wpb;
    if (tiles_per_item) *tiles_per_item = 1 << plan->impl->shape.lwt;
    return 0;
}

int vnp_autotune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = false;
    return 0;
}

int vnp_dnrmf_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const double *x, double *res,
                      void *stream)
{
    if (nseg < 0) return -1;
    if (nseg > 0 && !offsets) return -2;
    if (n_total < 0 || n_total > VNP_MAX_N) return -3;
    if (nseg > 0 && n_total > 0 && !x) return -4;
    if (nseg > 0 && !res) return -5;
    return run_batched(HypNode<double>{}, SegOffsets{offsets}, x, nseg, n_total, res, stream);
}

int vnp_snrmf_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const float *x, float *res,
                      void *stream)
{
    if (nseg < 0) return -1;
    if (nseg > 0 && !offsets) return -2;
    if (n_total < 0 || n_total > VNP_MAX_N) return -3;
    if (nseg > 0 && n_total > 0 && !x) return -4;
    if (nseg > 0 && !res) return -5;
    return run_batched(HypNode<float>{}, SegOffsets{offsets}, x, nseg, n_total, res, stream);
}

int vnp_dnrmp_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const double *x, double p,
                      double *res, void *stream)
{
    if (nseg < 0) return -1;
    if (nseg > 0 && !offsets) return -2;
    if (n_total < 0 || n_total > VNP_MAX_N) return -3;
    if (nseg > 0 && n_total > 0 && !x) return -4;
    if (!p_ok(p)) return -5;
    if (nseg > 0 && !res) return -6;
    return run_batched_p<double>(SegOffsets{offsets}, x, nseg, n_total, p, res, stream, 0x1p53);
}

int vnp_snrmp_batched(int64_t nseg, const int64_t *offsets, int64_t n_total, const float *x, float p, float *res,
                      void *stream)
{
    if (nseg < 0) return -1;
    if (nseg > 0 && !offsets) return -2;
    if (n_total < 0 || n_total > VNP_MAX_N) return -3;
    if (nseg > 0 && n_total > 0 && !x) return -4;
    if (!p_ok(p)) return -5;
    if (nseg > 0 && !res) return -6;
    return run_batched_p<float>(SegOffsets{offsets}, x, nseg, n_total, p, res, stream, 0x1p24f);
}

int vnp_dnrmf_cols(int64_t m, int64_t ncols, const double *A, int64_t lda, double *res, void *stream)
{
    if (m < 0) return -1;
    if (ncols < 0) return -2;
    if (m > 0 && ncols > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (ncols > 0 && !res) return -5;
    const int64_t total = ncols > 0 ? (ncols - 1) * lda + m : 0;
    return run_batched(HypNode<double>{}, SegCols{lda, m}, A, ncols, total, res, stream);
}

int vnp_snrmf_cols(int64_t m, int64_t ncols, const float *A, int64_t lda, float *res, void *stream)
{
    if (m < 0) return -1;
    if (ncols < 0) return -2;
    if (m > 0 && ncols > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (ncols > 0 && !res) return -5;
    const int64_t total = ncols > 0 ? (ncols - 1) * lda + m : 0;
    return run_batched(HypNode<float>{}, SegCols{lda, m}, A, ncols, total, res, stream);
}


static int mat_args(int64_t m, int64_t ncols, const void *A, int64_t lda)
{
    if (m < 0) return -1;
    if (ncols < 0) return -2;
    if (m > 0 && ncols > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (m > 0 && ncols > 0 && (ncols - 1) > (VNP_MAX_N - m) / lda) return -4;
    return 0;
}

int vnp_dnrmf_mat(int64_t m, int64_t ncols, const double *A, int64_t lda, double *res, void *stream)
{
    const int a = mat_args(m, ncols, A, lda);
    if (a) return a;
    if (!res) return -5;
    if (m == 0 || ncols == 0) return vnp_dnrmf(0, A, 1, res, stream);
    if (lda == m || ncols == 1) return vnp_dnrmf(m * ncols, A, 1, res, stream);
    return run_mat(HypNode<double>{}, m, ncols, A, lda, res, stream);
}

int vnp_snrmf_mat(int64_t m, int64_t ncols, const float *A, int64_t lda, float *res, void *stream)
{
    const int a = mat_args(m, ncols, A, lda);
    if (a) return a;
    if (!res) return -5;
    if (m == 0 || ncols == 0) return vnp_snrmf(0, A, 1, res, stream);
    if (lda == m || ncols == 1) return vnp_snrmf(m * ncols, A, 1, res, stream);
    return run_mat(HypNode<float>{}, m, ncols, A, lda, res, stream);
}

int vnp_dnrmp_mat(int64_t m, int64_t ncols, const double *A, int64_t lda, double p, double *res, void *stream)
{
    const int a = mat_args(m, ncols, A, lda);
    if (a) return a;
    if (!p_ok(p)) return -5;
    if (!res) return -6;
    if (m == 0 || ncols == 0) return vnp_dnrmp(0, A, 1, p, res, stream);
    if (lda == m || ncols == 1) return vnp_dnrmp(m * ncols, A, 1, p, res, stream);
    return run_mat_p<double>(m, ncols, A, lda, p, res, stream, 0x1p53);
}

int vnp_snrmp_mat(int64_t m, int64_t ncols, const float *A, int64_t lda, float p, float *res, void *stream)
{
    const int a = mat_args(m, ncols, A, lda);
    if (a) return a;
    if (!p_ok(p)) return -5;
    if (!res) return -6;
    if (m == 0 || ncols == 0) return vnp_snrmp(0, A, 1, p, res, stream);
    if (lda == m || ncols == 1) return vnp_snrmp(m * ncols, A, 1, p, res, stream);
    return run_mat_p<float>(m, ncols, A, lda, p, res, stream, 0x1p24f);
}

}  // extern "C"
