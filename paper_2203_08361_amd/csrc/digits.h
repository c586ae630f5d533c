// Integer-digit field plan (host interface).
//
// The field of eqs. (4)/(5) is evaluated as an exact integer product on the
// int8 matrix cores (v_mfma_i32_32x32x32_i8):
//   x  -> q = rint(x 2^30), written as balanced base-256 digits
//         q = d0 2^24 + d1 2^16 + d2 2^8 + d3 (d1..d3 in [-128, 127], d0 in
//         [-64, 64]); for |x| >= 2^-6 this is x itself, otherwise x to within
//         2^-31 (|x| <= 1 always holds after a step, eqs. (18)-(21));
//   sgn(x) -> one digit +-1 (dSB);
//   J  -> one digit when every entry is an integer in [-127, 127] (exact), else
//         a per-row power-of-two scale s_i and four digits of rint(J_ij/s_i 2^30).
// The products of digit pairs (a, b) with a + b <= 3 are summed in int32 per
// weight a + b, combined exactly in FP64 and rounded once to FP32.  For
// integer J the field is therefore fl32(sum_j J_ij q_j 2^-30) exactly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace hsb {

struct I8J;  // device J digit store and per-run digit buffers

// Spins are padded to a multiple of this for the digit plan.
constexpr int kI8SpinTile = 256;

// Build the digit store of J (host N x N, row-major).  Returns an hsb_status.
int i8_create(const float *hJ, int N, I8J **out);
void i8_free(I8J *p);
const char *i8_error();
bool i8_exact(const I8J *p);  // J held exactly (one digit)
int i8_max_n();
// Number of result-invariant kernel variants (the autotuner's candidates; 0
// is the default): 0, 1 = the persistent kernel with the default or the
// other wave height (32 or 64 rows), 2, 3 = one launch per step with those
// heights.
int i8_tiles();

struct I8Run {
    int variant;          // HSB_BSB / HSB_DSB
    int N, Nst, Rpad;     // spins, state rows (multiple of 64), padded replicas
    int R;
    int k0, k1, Ns, interval;
    float a0, c0, dt;
    const NHState *nh = nullptr;  // Nose-Hoover thermostat: rate -xi(t_k) per step
    int tile = 0;  // kernel variant, 0 .. i8_tiles(nh != nullptr) - 1
    const int32_t *cancel = nullptr;  // cancel request polled after each sample (b.stop set)
    int local_exchange = 1;  // 0: device-scope exchange in the persistent kernel even for
                             // XCD-local teams
};

// Run steps k0..k1-1 of the digit plan on the state in `b` (X, Y in
// [Nst][Rpad]); samples energies at the sample points (as the FP32 plan).
// The steps between two sample points run in one persistent launch that
// keeps the state on chip (when its teams of workgroups fit one XCD:
// N <= 8192), else one launch per step.
// `fp32J` is the FP32 J store ([Nst][Nst]) used for FP64 energies of real J.
int i8_run(I8J *p, const I8Run &run, StateBufs &b, const float *fp32J, hipStream_t s,
           KernelTimer &timer);

}  // namespace hsb
