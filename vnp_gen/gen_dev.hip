// Seeded synthetic inputs, device side, plus two plain calibration kernels.
//
// Holds no norm arithmetic.  The generator is the same SplitMix64 counter-based
// definition and the same value kinds as gen_host.c (see the header comment there);
// tests compare the two bit for bit.  The calibration kernels (a streaming copy and
// a streaming read) give the empirical HBM ceiling and the scale of the FETCH_SIZE
// and WRITE_SIZE counters.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

__device__ __forceinline__ uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t sm_mix_h(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t key_h(uint64_t seed, uint64_t stream) { return sm_mix_h(seed * SM_GAMMA + sm_mix_h(stream)); }

__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * SM_GAMMA); }

__device__ __forceinline__ int draw_exp(uint64_t rb, int lo, int hi)
{
    return lo + (int)(((rb >> 32) * (uint64_t)(hi - lo + 1)) >> 32);
}

__global__ void fill_d_kernel(double *x, int64_t n, int64_t i0, uint64_t ka, uint64_t kb, int kind, int lo, int hi)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t g = (uint64_t)(i0 + i);
        const uint64_t ra = draw(ka, g);
        double v;
        if (kind == 0) {
            v = 2.0 * ldexp((double)(ra >> 11), -53) - 1.0;
        } else if (kind == 1) {
            double u = 0.5 + ldexp((double)(ra >> 12), -53);
            if ((ra >> 10) & 1) u = -u;
            v = ldexp(u, draw_exp(draw(kb, g), lo, hi));
        } else if (kind == 2) {
            const double w = 2.0 * ldexp((double)(ra >> 11), -53) - 1.0;
            v = ldexp(w, draw_exp(draw(kb, g), lo, hi));
        } else {
            v = ldexp((double)(ra >> 11), -53);
        }
        x[i] = v;
    }
}

__global__ void fill_s_kernel(float *x, int64_t n, int64_t i0, uint64_t ka, uint64_t kb, int kind, int lo, int hi)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t g = (uint64_t)(i0 + i);
        const uint64_t ra = draw(ka, g);
        float v;
        if (kind == 0) {
            v = (float)(2.0 * ldexp((double)(ra >> 11), -53) - 1.0);
        } else if (kind == 1) {
            float u = 0.5f + ldexpf((float)(ra >> 41), -24);
            if ((ra >> 10) & 1) u = -u;
            v = ldexpf(u, draw_exp(draw(kb, g), lo, hi));
        } else if (kind == 2) {
            const float w = (float)(2.0 * ldexp((double)(ra >> 11), -53) - 1.0);
            v = ldexpf(w, draw_exp(draw(kb, g), lo, hi));
        } else {
            v = ldexpf((float)(ra >> 40), -24);
        }
        x[i] = v;
    }
}

// Streaming copy of nvec 16-byte vectors.
__global__ void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t nvec)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
        dst[i] = src[i];
}

// Streaming read of nvec 16-byte vectors: block b reads one contiguous chunk with
// non-temporal loads, 8 in flight per thread; xor-folds them so the loads are live and
// writes one word per block.
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) read_kernel(const u4v *__restrict__ src, int64_t nvec, uint32_t *out)
{
    const int64_t per = (nvec + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = b0 + per < nvec ? b0 + per : nvec;
    uint32_t acc = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256 * 8) {
        u4v v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t j = i + u * 256;
            v[u] = j < b1 ? __builtin_nontemporal_load(src + j) : u4v{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = 0;
        for (int k = 0; k < 256; ++k) r ^= red[k];
        out[blockIdx.x] = r;
    }
}

static int grid_for(int64_t n, int per)
{
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

extern "C" {

int vnpg_dev_fill_d(double *x, int64_t n, int64_t i0, uint64_t seed, uint64_t stream, int kind, int lo, int hi,
                    void *hstream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_d_kernel, dim3(grid_for(n, 256 * 8)), dim3(256), 0, (hipStream_t)hstream, x, n, i0,
                       key_h(seed, 2 * stream), key_h(seed, 2 * stream + 1), kind, lo, hi);
    return (int)hipGetLastError();
}

int vnpg_dev_fill_s(float *x, int64_t n, int64_t i0, uint64_t seed, uint64_t stream, int kind, int lo, int hi,
                    void *hstream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_s_kernel, dim3(grid_for(n, 256 * 8)), dim3(256), 0, (hipStream_t)hstream, x, n, i0,
                       key_h(seed, 2 * stream), key_h(seed, 2 * stream + 1), kind, lo, hi);
    return (int)hipGetLastError();
}

// bytes must be a multiple of 16 and both pointers 16-byte aligned.
int vnpg_dev_copy(void *dst, const void *src, int64_t bytes, int blocks, void *hstream)
{
    if (bytes <= 0 || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15)) return -1;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks > 0 ? blocks : 4096), dim3(256), 0, (hipStream_t)hstream,
                       (const uint4 *)src, (uint4 *)dst, bytes / 16);
    return (int)hipGetLastError();
}

// out must hold `blocks` 32-bit words.
int vnpg_dev_read(const void *src, int64_t bytes, uint32_t *out, int blocks, void *hstream)
{
    if (bytes <= 0 || (bytes & 15) || (((uintptr_t)src) & 15) || blocks <= 0) return -1;
    hipLaunchKernelGGL(read_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)hstream, (const u4v *)src,
                       bytes / 16, out);
    return (int)hipGetLastError();
}

}  // extern "C"
