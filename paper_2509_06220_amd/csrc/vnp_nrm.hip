// Single-vector norms: xNRMF and xNRMP of Novakovic, arXiv 2509.06220 (Sect. 1, 3, 4),
// on the canonical tree of vnp_tree.hpp, in one kernel launch.
//
// Launch: each wave reduces WT consecutive tiles, each block WPB consecutive waves; the
// block root goes to a per-stream workspace, and the last block to finish (atomic
// ticket, agent-scope release/acquire) reduces the block roots by the same fixed tree
// and writes the result.  All launch shapes give bitwise identical results.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include "../../include/vnp.h"
#include "vnp_internal.hpp"
#include "vnp_nodes_p.hpp"

namespace vnp {

// ---------------------------------------------------------------------------------
// Kernel
// ---------------------------------------------------------------------------------
template <class Node, int U, int WT, bool FAST>
__global__ void __launch_bounds__(1024)
    nrm_kernel(Node nd, const typename Node::T *x, int64_t n, int64_t inc, int64_t ntiles,
               typename Node::T *roots, unsigned int *ticket, typename Node::T *res)
{
    using T = typename Node::T;
    __shared__ T sbuf[1024];
    __shared__ unsigned int s_last;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int wpb = blockDim.x / WAVE;
    const int64_t t0 = ((int64_t)blockIdx.x * wpb + wave) * WT;

    const T r = wave_root<Node, U, WT, FAST>(nd, x, n, inc, t0, ntiles, lane);
    if (lane == 0) sbuf[wave] = r;
    lds_tree(nd, sbuf, wpb);
    if (gridDim.x == 1) {
        if (threadIdx.x == 0) *res = nd.finish(sbuf[0]);
        return;
    }
    if (threadIdx.x == 0) {
        roots[blockIdx.x] = sbuf[0];
        s_last = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const T root = block_finish(nd, roots, (int64_t)gridDim.x, sbuf);
    if (threadIdx.x == 0) {
        *res = nd.finish(root);
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T>
__global__ void write_zero_kernel(T *res)
{
    *res = T(0);
}

// ---------------------------------------------------------------------------------
// Launch configuration
// ---------------------------------------------------------------------------------
static int g_force_wpb = 0, g_force_wt = 0;

struct Shape {
    int wpb, wt;
};

static Shape choose_shape(int64_t ntiles)
{
    Shape s;
    if (g_force_wpb > 0 || g_force_wt > 0) {
        s.wpb = g_force_wpb > 0 ? g_force_wpb : 4;
        s.wt = g_force_wt > 0 ? g_force_wt : 1;
    } else if (ntiles >= (int64_t)1 << 16) {
        s = {4, 4};
    } else if (ntiles >= (int64_t)1 << 13) {
        s = {4, 2};
    } else if (ntiles >= 1024) {
        s = {4, 1};
    } else {
        s = {2, 1};
    }
    // keep the number of block roots within what the finish handles comfortably
    while ((ntiles + (int64_t)s.wpb * s.wt - 1) / ((int64_t)s.wpb * s.wt) > ((int64_t)1 << 20)) {
        if (s.wt < 8)
            s.wt *= 2;
        else if (s.wpb < 16)
            s.wpb *= 2;
        else
            break;
    }
    return s;
}

// ---------------------------------------------------------------------------------
// Per-(device, stream) workspace
// ---------------------------------------------------------------------------------
struct Workspace {
    void *roots = nullptr;  // block roots
    size_t roots_bytes = 0;
    unsigned int *ticket = nullptr;
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, void *>, Workspace> g_ws;

static int get_workspace(void *stream, size_t roots_bytes, Workspace **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[std::make_pair(dev, stream)];
    if (!w.ticket) {
        e = hipMalloc(reinterpret_cast<void **>(&w.ticket), 256);
        if (e != hipSuccess) return (int)e;
        e = hipMemset(w.ticket, 0, 256);
        if (e != hipSuccess) return (int)e;
    }
    if (w.roots_bytes < roots_bytes) {
        if (w.roots) {
            // the old buffer may still be in use by work queued on this stream
            e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
            if (e != hipSuccess) return (int)e;
            (void)hipFree(w.roots);
            w.roots = nullptr;
            w.roots_bytes = 0;
        }
        size_t b = roots_bytes < 65536 ? 65536 : roots_bytes;
        e = hipMalloc(&w.roots, b);
        if (e != hipSuccess) return (int)e;
        w.roots_bytes = b;
    }
    *out = &w;
    return 0;
}

int release_workspaces()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first == dev) {
            if (it->second.roots) (void)hipFree(it->second.roots);
            if (it->second.ticket) (void)hipFree(it->second.ticket);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------------
template <class Node, int U, int WT>
static void launch_wt(const Node &nd, bool fast, dim3 grid, dim3 block, hipStream_t st, const typename Node::T *x,
                      int64_t n, int64_t inc, int64_t ntiles, typename Node::T *roots, unsigned *ticket,
                      typename Node::T *res)
{
    if (fast)
        hipLaunchKernelGGL((nrm_kernel<Node, U, WT, true>), grid, block, 0, st, nd, x, n, inc, ntiles, roots, ticket,
                           res);
    else
        hipLaunchKernelGGL((nrm_kernel<Node, U, WT, false>), grid, block, 0, st, nd, x, n, inc, ntiles, roots, ticket,
                           res);
}

template <class Node>
static int run_norm(const Node &nd, int64_t n, const typename Node::T *x, int64_t incx, typename Node::T *res,
                    void *stream)
{
    using T = typename Node::T;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n <= 0) {
        hipLaunchKernelGGL((write_zero_kernel<T>), dim3(1), dim3(1), 0, st, res);
        return (int)hipGetLastError();
    }
    constexpr int64_t TE = tile_elems<T>();
    const int64_t ntiles = (n + TE - 1) / TE;
    const Shape s = choose_shape(ntiles);
    const int64_t per_block = (int64_t)s.wpb * s.wt;
    const int64_t nblocks = (ntiles + per_block - 1) / per_block;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, sizeof(T) * (size_t)nblocks, &ws);
    if (rc) return rc;
    const T *base = incx >= 0 ? x : x + (n - 1) * (-incx);
    const bool fast = incx == 1 && ((uintptr_t)x & 15) == 0;
    const dim3 grid((unsigned)nblocks), block((unsigned)(s.wpb * WAVE));
    T *roots = static_cast<T *>(ws->roots);
    switch (s.wt) {
    case 1: launch_wt<Node, 4, 1>(nd, fast, grid, block, st, base, n, incx, ntiles, roots, ws->ticket, res); break;
    case 2: launch_wt<Node, 4, 2>(nd, fast, grid, block, st, base, n, incx, ntiles, roots, ws->ticket, res); break;
    case 4: launch_wt<Node, 4, 4>(nd, fast, grid, block, st, base, n, incx, ntiles, roots, ws->ticket, res); break;
    default: launch_wt<Node, 4, 8>(nd, fast, grid, block, st, base, n, incx, ntiles, roots, ws->ticket, res); break;
    }
    return (int)hipGetLastError();
}

int set_launch_shape(int wpb, int wt)
{
    auto pow2 = [](int v) { return v == 0 || (v > 0 && (v & (v - 1)) == 0); };
    if (!pow2(wpb) || wpb > 16) return -1;
    if (!pow2(wt) || wt > 8) return -2;
    g_force_wpb = wpb;
    g_force_wt = wt;
    return 0;
}

template <typename T>
static int run_pnorm(int64_t n, const T *x, int64_t incx, T p, T *res, void *stream, T cutoff)
{
    if (p == T(2)) return run_norm(HypNode<T>{}, n, x, incx, res, stream);
    if (p == T(1)) return run_norm(SumNode<T>{}, n, x, incx, res, stream);
    if (__builtin_isinf(p) || p >= cutoff) return run_norm(MaxNode<T>{}, n, x, incx, res, stream);
    return run_norm(make_lp_node<T>(p), n, x, incx, res, stream);
}

}  // namespace vnp

using namespace vnp;

extern "C" {

int vnp_dnrmf(int64_t n, const double *x, int64_t incx, double *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!res) return -4;
    return run_norm(HypNode<double>{}, n, x, incx, res, stream);
}

int vnp_snrmf(int64_t n, const float *x, int64_t incx, float *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!res) return -4;
    return run_norm(HypNode<float>{}, n, x, incx, res, stream);
}

int vnp_dnrmp(int64_t n, const double *x, int64_t incx, double p, double *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!(p > 0)) return -4;
    if (!res) return -5;
    return run_pnorm<double>(n, x, incx, p, res, stream, 0x1p53);
}

int vnp_snrmp(int64_t n, const float *x, int64_t incx, float p, float *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!(p > 0)) return -4;
    if (!res) return -5;
    return run_pnorm<float>(n, x, incx, p, res, stream, 0x1p24f);
}

int vnp_set_launch_shape(int waves_per_block, int tiles_per_wave)
{
    return set_launch_shape(waves_per_block, tiles_per_wave);
}

int64_t vnp_tile_elems(int dtype)
{
    return dtype == VNP_F32 ? tile_elems<float>() : tile_elems<double>();
}

uint32_t vnp_tree_id(int dtype)
{
    // bits 0..7: log2(tile elements); 8..11: rows log2; 12..15: node version; 16: dtype
    const uint32_t te = dtype == VNP_F32 ? 14u : 13u;
    return te | (6u << 8) | (1u << 12) | ((uint32_t)(dtype == VNP_F32) << 16);
}

const char *vnp_version(void) { return "vnp 0.1 (gfx950)"; }

int vnp_finalize(void) { return release_workspaces(); }

}  // extern "C"
