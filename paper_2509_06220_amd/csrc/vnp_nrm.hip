// Single-vector norms: xNRMF and xNRMP of Novakovic, arXiv 2509.06220 (Sect. 1, 3, 4),
// on the canonical tree of vnp_tree.hpp.
//
// Launch: each wave reduces WT consecutive tiles, each block WPB consecutive waves; the
// block roots go to a per-stream workspace and a one-block finish kernel, launched after
// the streaming kernel on the same stream, reduces them by the same fixed tree and
// writes the result (a grid of one block writes it directly).  The streaming kernel's
// blocks never exchange data, so it needs no release or acquire, which on a multi-XCD
// device write back and invalidate the L2.  All launch shapes give bitwise identical
// results.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include "../../include/vnp.h"
#include "vnp_batch.hpp"
#include "vnp_internal.hpp"
#include "vnp_nodes_p.hpp"

namespace vnp {

// ---------------------------------------------------------------------------------
// Kernel
// ---------------------------------------------------------------------------------
template <class Node, int U, bool FAST>
__global__ void __launch_bounds__(1024)
    nrm_kernel(Node nd, const typename Node::T *x, int64_t n, Stride sd, int64_t ntiles, int lwt,
               typename Node::T *roots, typename Node::T *res)
{
    using T = typename Node::T;
    __shared__ T sbuf[16];
    node_prologue(nd);
    const int lane = threadIdx.x & (WAVE - 1);
    // wave index: uniform within the wave (tell the compiler, so the loops stay scalar)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int wpb = blockDim.x / WAVE;
    const int64_t t0 = ((int64_t)blockIdx.x * wpb + wave) << lwt;

    const T r = wave_root<Node, U, FAST>(nd, x, n, sd, t0, ntiles, lwt, lane);
    if (lane == 0) sbuf[wave] = r;
    lds_tree(nd, sbuf, wpb);
    if (threadIdx.x == 0) {
        if (gridDim.x == 1)
            *res = nd.finish(sbuf[0]);
        else
            roots[blockIdx.x] = sbuf[0];
    }
}

// Fixed tree over the block roots of the streaming kernel (one block of at most 1024
// threads; every power-of-two width evaluates the same tree).
template <class Node>
__global__ void __launch_bounds__(1024)
    nrm_finish_kernel(Node nd, typename Node::T *roots, int64_t count, typename Node::T *res)
{
    using T = typename Node::T;
    __shared__ T sbuf[1024];
    node_prologue(nd);
    const T root = block_finish(nd, roots, count, sbuf);
    if (threadIdx.x == 0) *res = nd.finish(root);
}

// Small vectors: one block of TILE_WAVES waves per tile (tile_root_block); the tile roots
// go to the workspace (a grid of one tile writes the result).
template <class Node, bool FAST>
__global__ void __launch_bounds__(TILE_WAVES * WAVE)
    nrm_tile_kernel(Node nd, const typename Node::T *x, int64_t n, Stride sd, typename Node::T *roots,
                    typename Node::T *res)
{
    using T = typename Node::T;
    __shared__ typename Node::R part[Vec<T>::N][TILE_WAVES][WAVE];
    node_prologue(nd);
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const T r = tile_root_block<Node, FAST>(nd, x, n, sd, blockIdx.x, lane, w, part);
    if (w == 0 && lane == 0) {
        if (gridDim.x == 1)
            *res = nd.finish(r);
        else
            roots[blockIdx.x] = r;
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
static int g_force_wpb = 0, g_force_lwt = -1;

struct Shape {
    int wpb, lwt;  // waves per block, log2(tiles per wave)
};

static int cu_count() { return device_cus(); }

// Blocks of 8 waves, about waves_per_cu waves per compute unit in total (128 for most
// nodes: eight rounds of the 16 resident waves of the binary64 kernel; TargetWavesPerCU),
// each wave streaming an aligned run of 2^lwt tiles
// (a run's root is a subtree of the canonical tree, so the shape never changes the
// result).  With several rounds the last, partly filled one is short and the hardware
// gives later blocks to the compute units that finish first; measured on MI355X (FP64):
// n = 2^30 1.267 ms either way, n = 636086033 0.838 -> 0.770 ms and n = 3e8 0.423 -> 0.379 ms
// against two rounds.
static Shape choose_shape(int64_t ntiles, int waves_per_cu)
{
    const int64_t target_waves = (int64_t)cu_count() * waves_per_cu;
    Shape s{8, 0};
    while (((int64_t)1 << s.lwt) * target_waves < ntiles && s.lwt < MAX_LWT) ++s.lwt;
    if (ntiles < (int64_t)cu_count() * 32) s.wpb = 4;
    if (ntiles < (int64_t)cu_count() * 4) s.wpb = 1;
    if (g_force_wpb > 0) s.wpb = g_force_wpb;
    if (g_force_lwt >= 0) s.lwt = g_force_lwt;
    // keep the number of block roots within what one block finishes quickly
    while ((ntiles + ((int64_t)s.wpb << s.lwt) - 1) / ((int64_t)s.wpb << s.lwt) > ((int64_t)1 << 20) &&
           s.lwt < MAX_LWT)
        ++s.lwt;
    return s;
}

// ---------------------------------------------------------------------------------
// Per-(device, stream) workspace
// ---------------------------------------------------------------------------------
struct Workspace {
    void *roots = nullptr;  // block roots
    size_t roots_bytes = 0;
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
template <class Node>
static void launch(const Node &nd, bool fast, dim3 grid, dim3 block, hipStream_t st, const typename Node::T *x,
                   int64_t n, Stride sd, int64_t ntiles, int lwt, typename Node::T *roots, typename Node::T *res)
{
    if (fast)
        hipLaunchKernelGGL((nrm_kernel<Node, RowsInFlight<Node>::value, true>), grid, block, 0, st, nd, x, n, sd,
                           ntiles, lwt, roots, res);
    else
        hipLaunchKernelGGL((nrm_kernel<Node, RowsInFlight<Node>::value, false>), grid, block, 0, st, nd, x, n, sd,
                           ntiles, lwt, roots, res);
    if (grid.x > 1)
        // up to 8192 roots in one pass of 8 per thread (4096 at the automatic shape for large n)
        hipLaunchKernelGGL((nrm_finish_kernel<Node>), dim3(1), dim3(grid.x > 2048 ? 1024 : 256), 0, st, nd, roots,
                           (int64_t)grid.x, res);
}

// The roots buffer of one call: the stream's workspace (fixed == nullptr), or the
// caller's fixed buffer of fixed_cap elements, which must hold every root (else -1).
template <typename T>
static int roots_buffer(void *stream, int64_t count, T *fixed, int64_t fixed_cap, T **out)
{
    if (fixed) {
        if (count > fixed_cap) return -1;
        *out = fixed;
        return 0;
    }
    Workspace *ws = nullptr;
    const int rc = get_workspace(stream, sizeof(T) * (size_t)count, &ws);
    if (rc) return rc;
    *out = static_cast<T *>(ws->roots);
    return 0;
}

// n logical elements, element 0 at base, address map sd; fast: contiguous and naturally
// aligned (vector loads).
template <class Node>
static int run_norm_map(const Node &nd, int64_t n, const typename Node::T *base, Stride sd, bool fast,
                        typename Node::T *res, void *stream, typename Node::T *fixed = nullptr,
                        int64_t fixed_cap = 0)
{
    using T = typename Node::T;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n <= 0) {
        hipLaunchKernelGGL((write_zero_kernel<T>), dim3(1), dim3(1), 0, st, res);
        return (int)hipGetLastError();
    }
    constexpr int64_t TE = tile_elems<T>();
    const int64_t ntiles = (n + TE - 1) / TE;
    if (ntiles < (int64_t)cu_count() * 4 && g_force_wpb == 0 && g_force_lwt < 0) {
        // small vector: eight waves per tile (see nrm_tile_kernel)
        T *roots = nullptr;
        const int rc = roots_buffer<T>(stream, ntiles, fixed, fixed_cap, &roots);
        if (rc) return rc;
        if (fast)
            hipLaunchKernelGGL((nrm_tile_kernel<Node, true>), dim3((unsigned)ntiles), dim3(TILE_WAVES * WAVE), 0, st,
                               nd, base, n, sd, roots, res);
        else
            hipLaunchKernelGGL((nrm_tile_kernel<Node, false>), dim3((unsigned)ntiles), dim3(TILE_WAVES * WAVE), 0, st,
                               nd, base, n, sd, roots, res);
        // the finish: one wave while the roots fit one pass of it (no cross-wave barriers);
        // every power-of-two width evaluates the same tree
        if (ntiles > 1)
            hipLaunchKernelGGL((nrm_finish_kernel<Node>), dim3(1), dim3(ntiles <= 8 * WAVE ? WAVE : 256), 0, st, nd,
                               roots, ntiles, res);
        return (int)hipGetLastError();
    }
    const Shape s = choose_shape(ntiles, TargetWavesPerCU<Node>::value);
    const int64_t per_block = (int64_t)s.wpb << s.lwt;
    const int64_t nblocks = (ntiles + per_block - 1) / per_block;
    T *roots = nullptr;
    const int rc = roots_buffer<T>(stream, nblocks, fixed, fixed_cap, &roots);
    if (rc) return rc;
    launch(nd, fast, dim3((unsigned)nblocks), dim3((unsigned)(s.wpb * WAVE)), st, base, n, sd, ntiles, s.lwt, roots,
           res);
    return (int)hipGetLastError();
}

template <class Node>
static int run_norm(const Node &nd, int64_t n, const typename Node::T *x, int64_t incx, typename Node::T *res,
                    void *stream, typename Node::T *fixed = nullptr, int64_t fixed_cap = 0)
{
    using T = typename Node::T;
    const T *base = incx >= 0 || n <= 0 ? x : x + (n - 1) * (-incx);
    const bool fast = incx == 1 && ((uintptr_t)x % sizeof(T)) == 0;
    return run_norm_map(nd, n, base, real_stride(incx), fast, res, stream, fixed, fixed_cap);
}

// ---------------------------------------------------------------------------------
// Allocation-free DNRMF: the block (or tile) roots of a call live in a fixed device array
// instead of the per-stream workspace.  Host code never passes the array's name (a host
// stand-in) to a kernel: it uses the device address taken once per device.
// ---------------------------------------------------------------------------------
static __device__ __align__(256) double scratch[VNP_NOALLOC_MAX_ROOTS];

constexpr int SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[SCRATCH_DEVICES] = {};

// The current device's copy of `scratch` (looked up on the first call on that device).
static int scratch_ptr(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= SCRATCH_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

// Frobenius norm of n complex elements (interleaved re, im) with stride incz (in complex
// elements): the tree over the 2n-element real view.
template <typename T>
static int run_complex(int64_t n, const T *z, int64_t incz, T *res, void *stream)
{
    if (incz == 1) return run_norm(HypNode<T>{}, n > 0 ? 2 * n : 0, z, 1, res, stream);
    const T *base = incz >= 0 || n <= 0 ? z : z + 2 * (n - 1) * (-incz);
    return run_norm_map(HypNode<T>{}, n > 0 ? 2 * n : 0, base, Stride{2 * incz, 1}, false, res, stream);
}

int set_launch_shape(int wpb, int wt)
{
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    if (wpb != 0 && (!pow2(wpb) || wpb > 16)) return -1;
    if (wt != 0 && (!pow2(wt) || wt > (1 << MAX_LWT))) return -2;
    g_force_wpb = wpb;
    g_force_lwt = wt == 0 ? -1 : ilog2(wt);
    return 0;
}

template <typename T>
static int run_pnorm(int64_t n, const T *x, int64_t incx, T p, T *res, void *stream, T cutoff)
{
    if (p == T(2)) return run_norm(HypNode<T>{}, n, x, incx, res, stream);
    if (p == T(1)) return run_norm(SumNode<T>{}, n, x, incx, res, stream);
    if (__builtin_isinf(p) || p >= cutoff) return run_norm(MaxNode<T>{}, n, x, incx, res, stream);
    LpNode<T> nd;
    const int rc = make_lp_node<T>(p, &nd);
    return rc ? rc : run_norm(nd, n, x, incx, res, stream);
}

}  // namespace vnp

using namespace vnp;

extern "C" {

int vnp_dznrmf(int64_t n, const double *z, int64_t incz, double *res, void *stream)
{
    if (n > VNP_MAX_N / 2) return -1;
    if (n > 0 && !z) return -2;
    if (incz == 0) return -3;
    if (!res) return -4;
    return run_complex<double>(n, z, incz, res, stream);
}

int vnp_scnrmf(int64_t n, const float *z, int64_t incz, float *res, void *stream)
{
    if (n > VNP_MAX_N / 2) return -1;
    if (n > 0 && !z) return -2;
    if (incz == 0) return -3;
    if (!res) return -4;
    return run_complex<float>(n, z, incz, res, stream);
}

int vnp_dnrmf(int64_t n, const double *x, int64_t incx, double *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!res) return -4;
    return run_norm(HypNode<double>{}, n, x, incx, res, stream);
}

int vnp_dnrmf_noalloc(int64_t n, const double *x, int64_t incx, double *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!res) return -4;
    double *roots = nullptr;
    const int rc = scratch_ptr(&roots);
    if (rc) return rc;
    return run_norm(HypNode<double>{}, n, x, incx, res, stream, roots, (int64_t)VNP_NOALLOC_MAX_ROOTS);
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
    if (!p_ok(p)) return -4;
    if (!res) return -5;
    return run_pnorm<double>(n, x, incx, p, res, stream, 0x1p53);
}

int vnp_snrmp(int64_t n, const float *x, int64_t incx, float p, float *res, void *stream)
{
    if (n > VNP_MAX_N) return -1;
    if (n > 0 && !x) return -2;
    if (incx == 0) return -3;
    if (!p_ok(p)) return -4;
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
    // bits 0..7: log2(tile elements); 8..11: rows log2; 12..15: node version (3: the
    // p node's logarithm table exact at 1/2 and, in binary64, its row levels in log2);
    // 16: dtype
    const uint32_t te = dtype == VNP_F32 ? 14u : 13u;
    return te | (6u << 8) | (3u << 12) | ((uint32_t)(dtype == VNP_F32) << 16);
}

const char *vnp_version(void) { return "vnp 0.1 (gfx950)"; }

int vnp_finalize(void)
{
    release_batch_workspaces();
    release_svd_workspaces();
    release_lp_tables();
    return release_workspaces();
}

}  // extern "C"
