// Device helpers of the persistent FP4 kernels (single runs and batches):
// the tagged exchange words, the FP4 matrix-core products with J held in
// accumulation registers, the sign-operand expansion, the bounded gather of a
// team's sign words, and the update of eqs. (16)-(22) written in place.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hsb_device.h"

namespace hsb {

constexpr uint32_t kNoTag = 0xFFFFFFFFu;
constexpr uint64_t kTimeoutTicks = 400000000ull;  // 4 s of the 100 MHz wall clock

__device__ __forceinline__ uint64_t ld_tagged(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_tagged(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Store for a team whose workgroups all run on one XCD: the word only has to
// reach that XCD's L2, where the readers' device-scope loads find it (about
// half the round trip of a device-scope store, which writes through).
__device__ __forceinline__ void st_tagged_xcd(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Id of the XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20); }

// F tile update on the FP4 matrix cores: acc (VGPRs) += j (J fragment, AGPRs)
// x b (+-1 operand, VGPRs), 32 rows x 32 replicas x 64 spins, unit block
// scales.  Inline assembly keeps the loop-invariant J fragments in the
// accumulation register file for the whole kernel, feeding the MFMA directly
// (the compiler would otherwise copy them to VGPRs before every use).
// Hazards: exactly overlapping srcC/vdst chains are interlocked by the
// hardware; the first product of a step uses an inline zero for srcC; VALU
// reads of the results wait behind mfma_drain().  A VGPR source written by a
// vector instruction needs two wait states before an MFMA reads it, and the
// compiler does not insert them around inline assembly: the B operands here
// come from LDS loads and the scale is loop-invariant, so none arise.
__device__ __forceinline__ void mfma_fp4_first(v16f &acc, const v4i &j, const v4i &b, int one) {
    asm volatile(
        "v_mfma_scale_f32_32x32x64_f8f6f4 %0, %1, %2, 0, %3, %3 op_sel_hi:[0,0,0] cbsz:4 blgp:4"
        : "=&v"(acc)
        : "a"(j), "v"(b), "v"(one));
}
__device__ __forceinline__ void mfma_fp4(v16f &acc, const v4i &j, const v4i &b, int one) {
    asm volatile(
        "v_mfma_scale_f32_32x32x64_f8f6f4 %0, %1, %2, %0, %3, %3 op_sel_hi:[0,0,0] cbsz:4 blgp:4"
        : "+v"(acc)
        : "a"(j), "v"(b), "v"(one));
}

// 21 wait states: more than an XDL write needs before a VALU read of its vdst.
__device__ __forceinline__ void mfma_drain(v16f &acc0, v16f &acc1) {
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 4" : "+v"(acc0), "+v"(acc1));
}
__device__ __forceinline__ void mfma_drain(v16f &acc) {
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 4" : "+v"(acc));
}

// FP4 encoding of the values exact in E2M1.
__device__ __forceinline__ uint32_t fp4_code(float v) {
    const float a = fabsf(v);
    uint32_t m = a == 0.5f ? 1u : a == 1.0f ? 2u : a == 1.5f ? 3u : a == 2.0f ? 4u
               : a == 3.0f ? 5u : a == 4.0f ? 6u : a == 6.0f ? 7u : 0u;
    return m | (v < 0.0f ? 8u : 0u);
}

// Sign words.  The word of (replica, 32-row chunk) holds one bit per row, set
// iff x < 0.  Its bit order follows the accumulator layout of the writer
// (lane l holds rows 8j + 4(l/32) + i, j, i = 0..3, of replica l%32): bit
// b < 16 is row 8(b/4) + b%4, bit b >= 16 is row 8((b-16)/4) + 4 + b%4.
__host__ __device__ constexpr int word_bit_row(int b) {
    return b < 16 ? 8 * (b >> 2) + (b & 3) : 8 * ((b - 16) >> 2) + 4 + (b & 3);
}
__host__ __device__ constexpr int row_word_bit(int t) {
    return (t & 4) ? 16 + 4 * (t >> 3) + (t & 3) : 4 * (t >> 3) + (t & 3);
}

// Packing convention shared by both MFMA operands.  Within a 32-spin chunk,
// nibble n of fragment dword q holds the spin of word bit 4n + 3 - q.  The
// +-1 operand of a chunk is then
//   dword q = ((w << q) & 0x88888888) | 0x22222222
// (0x2 = +1.0, 0xA = -1.0 in E2M1): seven integer operations per chunk.
__device__ __forceinline__ v4i expand_signs(uint32_t w) {
    v4i a;
    a[0] = (int)((w & 0x88888888u) | 0x22222222u);
    a[1] = (int)(((w << 1) & 0x88888888u) | 0x22222222u);
    a[2] = (int)(((w << 2) & 0x88888888u) | 0x22222222u);
    a[3] = (int)(((w << 3) & 0x88888888u) | 0x22222222u);
    return a;
}

// The same expansion at one operation per dword: v_and_or_b32 computes
// (a & b) | c, but its encoding takes no literal, so the two constants come in
// registers (the mask in a scalar one, the +1.0 pattern in a vector one).
__device__ __forceinline__ v4i expand_signs_fast(uint32_t w, uint32_t mask, uint32_t ones) {
    v4i a;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a[0]) : "v"(w), "s"(mask), "v"(ones));
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a[1]) : "v"(w << 1), "s"(mask), "v"(ones));
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a[2]) : "v"(w << 2), "s"(mask), "v"(ones));
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a[3]) : "v"(w << 3), "s"(mask), "v"(ones));
    return a;
}

// Gather, for state m, the tagged sign words of the K blocks this wave
// expands (its share: every 4th block), wv[q] holding block w + 4q.  All
// words are loaded together and every stale one is reloaded together until
// all carry tag m, so the wait costs about one round trip after the last
// writer.  Returns false on timeout (4 s) or when another wave has flagged an
// error.
template <int NQ>
__device__ __forceinline__ bool gather_words(uint64_t (&wv)[NQ], const uint64_t *src,
                                             size_t stride, int nq, uint32_t m, int32_t *err) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q < nq) wv[q] = ld_tagged(src + q * stride);
    uint32_t stale = 0;  // bit q: some lane's word q is stale
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q < nq && __any((uint32_t)(wv[q] >> 32) != m)) stale |= 1u << q;
    if (stale == 0) return true;
    const uint64_t t0 = wall_clock64();
    for (int it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if ((stale >> q) & 1u) wv[q] = ld_tagged(src + q * stride);
        uint32_t still = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (((stale >> q) & 1u) && __any((uint32_t)(wv[q] >> 32) != m)) still |= 1u << q;
        stale = still;
        if (stale == 0) return true;
        if ((it & 31) == 0) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                return false;
            if (wall_clock64() - t0 > kTimeoutTicks) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
}

// sb_update (the same operations and roundings) with the last FMA written
// so that y' lands in the register of y: the compiler would otherwise
// accumulate into the register of y~~ and copy every y back each step.
__device__ __forceinline__ void sb_update_tied(float f, float p, float c0, float dt, float a0dt,
                                               float gdt, float &x, float &y) {
    const float c0f = c0 * f;
    const float u = __fmaf_rn(-p, x, c0f);
    const float yt = __fmaf_rn(u, dt, y);
    const float xt = __fmaf_rn(a0dt, yt, x);
    const bool wall = fabsf(xt) > 1.0f;
    x = __builtin_amdgcn_fmed3f(xt, -1.0f, 1.0f);
    const float ytt = wall ? 0.0f : yt;
    asm("v_fma_f32 %0, %1, %0, %2" : "+v"(y) : "v"(gdt), "v"(ytt));  // y' = (gamma dt) y + y~~
}

}  // namespace hsb
