// Device-side definitions shared by the libhsb kernels (not by the oracle).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsb {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));

// Counter-based generator: the output mixer of SplitMix64 (Steele, Lea and
// Flood, OOPSLA 2014) chained over (seed, stream, a, b), all modulo 2^64.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t rng_key(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    uint64_t h = mix64(seed + G * (stream + 1));
    h = mix64(h + G * (a + 1));
    return mix64(h + G * (b + 1));
}

// Uniform in the open interval (-1, 1): odd multiples of 2^-24, never 0.
__device__ __forceinline__ float uniform_open(uint64_t h) {
    int m = (int)(h >> 40);
    return (float)(2 * m + 1 - (1 << 24)) * 0x1p-24f;
}

// sgn with sgn(0) = sgn(-0) = +1.
__device__ __forceinline__ float sgnf(float x) { return x >= 0.0f ? 1.0f : -1.0f; }

// One spin of the Methods time step, eqs. (16)-(22), single precision:
//   u = -p x + c0 f, y~ = y + u dt, x~ = x + (a0 dt) y~,
//   walls: |x~| > 1 -> x' = sgn(x~), y~~ = 0 (eqs. (18)-(21)),
//   y' = y~~ + (gamma dt) y_old (eq. (22)).
// p = a0 - a(t_k).  Each operation is rounded once, in this order (the file
// is built with floating-point contraction disabled).
__device__ __forceinline__ void sb_update(float f, float p, float c0, float dt, float a0dt, float gdt,
                                          float &x, float &y) {
    const float c0f = c0 * f;
    const float u = __fmaf_rn(-p, x, c0f);
    const float yt = __fmaf_rn(u, dt, y);
    const float xt = __fmaf_rn(a0dt, yt, x);
    const bool wall = fabsf(xt) > 1.0f;
    // g(x~): x~ inside [-1, 1], else sgn(x~) -- the median of (x~, -1, 1)
    const float xn = __builtin_amdgcn_fmed3f(xt, -1.0f, 1.0f);
    const float ytt = wall ? 0.0f : yt;
    y = __fmaf_rn(gdt, y, ytt);
    x = xn;
}

}  // namespace hsb
