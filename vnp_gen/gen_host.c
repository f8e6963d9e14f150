/*
 * Seeded synthetic inputs for the norm kernels and for the CPU oracle (host side).
 *
 * This module holds no norm arithmetic.  It only turns (seed, stream, index) into
 * input values, so that the GPU path and the oracle can be fed the same vectors.
 *
 * Random bits: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based generator:
 * the i-th output (0-based) of a SplitMix64 stream started at state K is
 * mix(K + (i+1)*GAMMA).  A (seed, stream) pair selects K.  The device copy in
 * gen_dev.hip implements the same definition; tests check they agree bit for bit.
 *
 * Value kinds (every variate is exact before the final ldexp):
 *   KIND_U11    x = 2*u53 - 1,            u53 = (ra >> 11) * 2^-53      in [-1, 1)
 *   KIND_EXP    x = +-u * 2^e,            u = 1/2 + (ra >> 12) * 2^-53  in [1/2, 1)
 *   KIND_U11EXP x = (2*u53 - 1) * 2^e
 *   KIND_U01    x = u53                                                  in [0, 1)
 * with ra drawn from sub-stream 2*stream and rb from sub-stream 2*stream+1,
 * sign = bit 10 of ra, e = lo + (((rb >> 32) * (hi - lo + 1)) >> 32).
 * binary32 variants: U11 is RN((float)x64); EXP uses u = 1/2 + (ra >> 41) * 2^-24
 * and ldexpf; U11EXP is ldexpf((float)(2*u53-1), e); U01 is (ra >> 40) * 2^-24.
 */
#include <math.h>
#include <stdint.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

enum { KIND_U11 = 0, KIND_EXP = 1, KIND_U11EXP = 2, KIND_U01 = 3 };

static inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t vnpg_key(uint64_t seed, uint64_t stream)
{
    return sm_mix(seed * SM_GAMMA + sm_mix(stream));
}

uint64_t vnpg_draw(uint64_t key, uint64_t i)
{
    return sm_mix(key + (i + 1) * SM_GAMMA);
}

static inline int draw_exp(uint64_t rb, int lo, int hi)
{
    return lo + (int)(((rb >> 32) * (uint64_t)(hi - lo + 1)) >> 32);
}

static inline double gen_d(uint64_t ka, uint64_t kb, uint64_t i, int kind, int lo, int hi)
{
    const uint64_t ra = vnpg_draw(ka, i);
    switch (kind) {
    case KIND_U11:
        return 2.0 * ldexp((double)(ra >> 11), -53) - 1.0;
    case KIND_EXP: {
        const uint64_t rb = vnpg_draw(kb, i);
        double u = 0.5 + ldexp((double)(ra >> 12), -53);
        if ((ra >> 10) & 1) u = -u;
        return ldexp(u, draw_exp(rb, lo, hi));
    }
    case KIND_U11EXP: {
        const uint64_t rb = vnpg_draw(kb, i);
        const double v = 2.0 * ldexp((double)(ra >> 11), -53) - 1.0;
        return ldexp(v, draw_exp(rb, lo, hi));
    }
    default:
        return ldexp((double)(ra >> 11), -53);
    }
}

static inline float gen_s(uint64_t ka, uint64_t kb, uint64_t i, int kind, int lo, int hi)
{
    const uint64_t ra = vnpg_draw(ka, i);
    switch (kind) {
    case KIND_U11:
        return (float)(2.0 * ldexp((double)(ra >> 11), -53) - 1.0);
    case KIND_EXP: {
        const uint64_t rb = vnpg_draw(kb, i);
        float u = 0.5f + ldexpf((float)(ra >> 41), -24);
        if ((ra >> 10) & 1) u = -u;
        return ldexpf(u, draw_exp(rb, lo, hi));
    }
    case KIND_U11EXP: {
        const uint64_t rb = vnpg_draw(kb, i);
        const float v = (float)(2.0 * ldexp((double)(ra >> 11), -53) - 1.0);
        return ldexpf(v, draw_exp(rb, lo, hi));
    }
    default:
        return ldexpf((float)(ra >> 40), -24);
    }
}

/* Fill x[0..n) with elements i0 .. i0+n-1 of the (seed, stream, kind, lo, hi) vector. */
void vnpg_fill_d(double *x, int64_t n, int64_t i0, uint64_t seed, uint64_t stream,
                 int kind, int lo, int hi)
{
    const uint64_t ka = vnpg_key(seed, 2 * stream), kb = vnpg_key(seed, 2 * stream + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        x[i] = gen_d(ka, kb, (uint64_t)(i0 + i), kind, lo, hi);
}

void vnpg_fill_s(float *x, int64_t n, int64_t i0, uint64_t seed, uint64_t stream,
                 int kind, int lo, int hi)
{
    const uint64_t ka = vnpg_key(seed, 2 * stream), kb = vnpg_key(seed, 2 * stream + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        x[i] = gen_s(ka, kb, (uint64_t)(i0 + i), kind, lo, hi);
}

/* Raw 64-bit draws (for tests of the generator itself). */
void vnpg_draws(uint64_t *out, int64_t n, int64_t i0, uint64_t seed, uint64_t stream)
{
    const uint64_t k = vnpg_key(seed, stream);
    for (int64_t i = 0; i < n; ++i)
        out[i] = vnpg_draw(k, (uint64_t)(i0 + i));
}
