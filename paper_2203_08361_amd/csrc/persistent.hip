// Persistent discrete-SB path on FP4 matrix cores.
//
// Field (eq. (5)): f = J sgn(x).  sgn(x) is +-1 and, for this path, every J_ij
// is exactly representable in FP4 (E2M1), so the products are exact and the
// FP32 accumulation of at most 2048 of them is exact: the field -- and hence
// the whole single-precision trajectory -- is bitwise that of any exact
// evaluation of eq. (5).
//
// Work decomposition.  Replicas never interact, so a "team" of waves owns a
// tile of 32 replicas for the whole run, and inside the team wave `rb` owns
// spin rows [32 rb, 32 rb + 32).  Each wave keeps, for the whole launch,
//   - its 32 rows of J as FP4 MFMA operands in registers (32 x Npad x 4 bit),
//   - x and y of its 32 x 32 (row, replica) block in registers.
// One step (Methods, eqs. (16)-(22)) is
//   1. F^T = S^T J  with S = sgn(x(t_k)) of all Npad rows of the team's 32
//      replicas, on v_mfma_scale_f32_32x32x64_f8f6f4 (FP4 x FP4, unit scales);
//   2. the fused update of its 64 x 32 block in registers;
//   3. publishing the new signs: per (32-row chunk, replica) one 32-bit word
//      of sign bits, stored together with the step index as a 64-bit tagged
//      word in a ping-pong exchange buffer (synchronous update, eq. (16):
//      every f_i of step k reads x(t_k) only).
// Readers spin on the tag of each word they need; there is no grid barrier.
// Double buffering by step parity makes a word safe to overwrite: the writer
// of step k+2 has read every word of step k+1, whose writers had finished
// reading step k.
//
// Energy (eq. (1)) needs J sgn(x) of the sampled state -- exactly the field
// already computed for that state -- so each wave stores per-replica partial
// sums sum_i s_i f_i of its rows at every sample point, plus the sign words of
// the sampled state; a small kernel then forms E, keeps the best sample
// (strict improvement, earliest wins) and its spins.
#include "hsb.h"
#include "fp4_device.h"
#include "hsb_device.h"
#include "persistent.h"

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <vector>

namespace hsb {

constexpr int kMaxKB = 32;  // K blocks of 64 spins: N <= 2048

// Scratch of one persistent run (a single instance or a batch of teams).
struct PersistentWork {
    uint64_t *xb = nullptr;      // [2][nchunk][Rpad] tagged sign words
    size_t xb_words = 0;
    uint32_t *snap = nullptr;    // [ns][nchunk][Rpad] sign words of sampled states
    size_t snap_words = 0;
    float *ep = nullptr;         // [ns][nparts][Rpad] energy partials (per row block)
    size_t ep_elems = 0;
    double *es = nullptr;        // [ns][Rpad] sample energies
    size_t es_elems = 0;
    double *tp = nullptr;        // [ns][nparts][Rpad] partial sums of y^2 (traces only)
    size_t tp_elems = 0;
    float *ptab = nullptr;       // p_k = a0 - a(t_k) of the steps of one segment
    size_t ptab_elems = 0;
    int32_t *err = nullptr;      // [1] timeout flag
    uint64_t *xslot = nullptr;   // [grid] (launch epoch, XCD id) per workgroup
    size_t xslot_n = 0;
    uint32_t *epoch = nullptr;   // [1] launch epoch, advanced on the device before each launch
    size_t epoch_n = 0;
    std::vector<FP4Team> teams_up;  // the team table last uploaded to `teams`
    uint64_t gen = 0;            // raised when a buffer is reallocated or the table re-uploaded
    FP4Team *teams = nullptr;    // [nteams] per-team J, N and c0
    size_t teams_n = 0;
    // bSB exchange: digit fragments [2][nkb][8][2 Rpad], chunk exponents
    // [2][2 Rpad][nkb], step flags [nteams][nrb]
    v4i *xd = nullptr;
    size_t xd_n = 0;
    uint8_t *xe = nullptr;
    size_t xe_n = 0;
    uint32_t *flags = nullptr;
    size_t flags_n = 0;
    int32_t *tstop = nullptr;    // [nteams] stop step of each team (-1: running)
    size_t tstop_n = 0;
    uint64_t *ypart = nullptr;   // thermostat: [2][nchunk / 4][Rpad][2] tagged partials of y^2
    size_t ypart_n = 0;
    double *bpart = nullptr;     // bSB thermostat: [2][row blocks][Rpad] partials of y^2
    size_t bpart_n = 0;
};

struct PersistentJ {
    int N = 0, Npad = 0, nkb = 0, nrb = 0;
    v4i *jpk = nullptr;          // [nrb][2][nkb][64] FP4 fragments
    PersistentWork work;         // scratch of this instance's own runs
};

namespace {
thread_local char p_err[256] = "";
int perr(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(p_err, sizeof(p_err), fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace

const char *persistent_error() { return p_err; }
int persistent_tiles(int variant) { return variant == HSB_BSB ? 2 : 3; }
int persistent_max_n() { return kMaxKB * 64; }
bool persistent_supported(int N) { return N >= 1 && N <= kMaxKB * 64; }

// ----------------------------------------------------------------- device

// J fragment for (row block rb, row tile rt, K block kb, lane): lane l holds
// row 64 rb + 32 rt + l%32 and the 32 spins of chunk 2 kb + l/32, in the order
// of the packing convention.
__global__ void k_pack_fp4(const float *__restrict__ J, v4i *__restrict__ jpk, int Npad, int nkb,
                           int nrb) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nrb * 2 * nkb * 64;
    if (e >= total) return;
    const int lane = (int)(e & 63);
    const int kb = (int)((e >> 6) % nkb);
    const int rt = (int)((e >> 6) / nkb % 2);
    const int rb = (int)((e >> 6) / nkb / 2);
    const int row = rb * 64 + rt * 32 + (lane & 31);
    const int base = kb * 64 + (lane >> 5) * 32;
    v4i out;
    for (int q = 0; q < 4; ++q) {
        uint32_t d = 0;
        for (int n = 0; n < 8; ++n)
            d |= fp4_code(J[(size_t)row * Npad + base + word_bit_row(4 * n + 3 - q)]) << (4 * n);
        out[q] = (int)d;
    }
    jpk[e] = out;
}

__global__ void k_zero_i32(int32_t *p) { p[0] = 0; }

__global__ void k_fill_tags(uint64_t *xb, size_t n) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) xb[e] = ((uint64_t)kNoTag << 32);
}

struct SegArgs {
    int seg_k0, seg_k1, final_k, interval, nmult;
};

// The Nose-Hoover thermostat inside the persistent dSB kernel (eqs. (6)-(8)):
// xi per replica ([Rpad], FP64: its value at the segment's first step in, at
// its last out), the per-step partial sums of y^2 of every workgroup's 128
// rows as pairs of tagged words ([2 step parities][nchunk / 4][Rpad][2]:
// (step << 32) | low and high halves of the FP64 partial), c = dt / M and N T.
struct FP4NH {
    double *xi;
    uint64_t *ypart;
    double c, NT;
};

// The sample points of a segment: the run's last step (final_k, if it lies in
// the segment) and every multiple of the interval in (seg_k0, seg_k1]; the
// multiples have indices 0, 1, ... in step order and the last step, if it is
// not one of them, index nmult.  Kept as a running clock, without a division
// per step: `next` is the first multiple after the steps already passed (-1
// once it would exceed the int range, where no step lies) and `index` its
// sample index.  pass(m) is called once each step m, after its own sample and
// before asking about m + 1.
struct SampleClock {
    int next, index;
    __device__ __forceinline__ explicit SampleClock(const SegArgs &g) : index(0) {
        next = step_after((long long)(g.seg_k0 / g.interval) * g.interval, g.interval);
    }
    __device__ static __forceinline__ int step_after(long long mult, int interval) {
        const long long t = mult + interval;
        return t > 0x7FFFFFFFll ? -1 : (int)t;
    }
    __device__ __forceinline__ bool is_sample(const SegArgs &g, int m) const {
        return m == g.final_k || m == next;
    }
    __device__ __forceinline__ int sample_index(const SegArgs &g, int m) const {
        return m == next ? index : g.nmult;
    }
    __device__ __forceinline__ void pass(const SegArgs &g, int m) {
        if (m == next) {
            next = step_after(next, g.interval);
            ++index;
        }
    }
};

// One workgroup = 4 waves = 4 consecutive 32-row blocks of one team, so the
// four waves need the same +-1 operand (the team's signs).  Each step every
// wave gathers and expands a quarter of the K blocks into LDS (ping-pong by
// step parity), one workgroup barrier publishes them, and each wave then runs
// its MFMAs with its J rows from registers and the operand from LDS, followed
// by the fused update of its 32 rows x 32 replicas.
// Two workgroups share a CU (two waves per SIMD): a wave's step is a serial
// chain (products, update, exchange round trip), and the other wave on the
// SIMD -- of another team, which is out of step with it -- fills the matrix
// core while this one waits for its team's signs.  That is why a wave holds
// 32 rows rather than 64: 32 rows of J take 128 of the 256 registers two waves
// per SIMD leave each.
//
// CANCEL: the variant that honours hsb_cancel (below).  It is a separate
// instantiation because its code, though it runs only at sample points,
// changes the schedule the compiler gives the step (measured 6% slower at
// the bench size); the other variant has none of it.
template <int NKB, int KPRE, bool NH, bool CANCEL>
__global__ __launch_bounds__(256, 2) void k_dsb_fp4(
    const FP4Team *__restrict__ teams, float *__restrict__ X, float *__restrict__ Y,
    const float *__restrict__ gamma, uint64_t *xb, uint32_t *__restrict__ snap,
    float *__restrict__ ep, double *__restrict__ tp, const float *__restrict__ ptab,
    int32_t *__restrict__ bad,
    int32_t *__restrict__ status, int32_t *err, uint64_t *xslot, const uint32_t *epoch_p,
    int local_ok, const int32_t *cancel, int32_t *tstop, FP4NH nhp,
    int nkb, int nchunk, int Rpad, int team0, int nteams, SegArgs g, float dt, float a0dt) {
    static_assert(NKB % 4 == 0, "Npad is a multiple of 256");
    constexpr int NQ = NKB / 4;  // K blocks expanded by each wave
    __shared__ v4i a_lds[2][NKB][64];
    __shared__ int wg_abort;
    // thermostat: each wave's y^2 partial of the current state, and the eight
    // half-waves' sums of the team's partials (both by step parity)
    __shared__ double s_yw[NH ? 2 : 1][4][32];
    __shared__ double s_ysum[NH ? 2 : 1][8][32];
    // thermostat: xi(t_k) of the workgroup's 32 replicas (every wave of the
    // team forms the same value; kept here rather than in registers)
    __shared__ double s_xi[NH ? 4 : 1][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD
    // b % 8).  All workgroups of a team are placed on one XCD so that the sign
    // words they exchange every step stay in that XCD's L2: team t uses the
    // blocks b = 8 (wpt (t / 8) + k) + t % 8, k = 0 .. wpt-1.  (Correctness does
    // not depend on the placement; only the exchange latency does.)
    const int wpt = nchunk >> 2;  // workgroups per team
    const int xcd = blockIdx.x & 7, kx = blockIdx.x >> 3;
    const int tl = (kx / wpt) * 8 + xcd;  // team within this launch
    if (tl >= nteams) return;             // whole workgroup
    const int team = team0 + tl;
    // the team's instance: its FP4 J fragments, its N and its c0 (a batch
    // mixes instances of the same padded size in one launch)
    const v4i *__restrict__ jpk = static_cast<const v4i *>(teams[team].jpk);
    const int N = teams[team].N;
    const float c0 = teams[team].c0;
    const int rb = (kx % wpt) * 4 + w;  // 32-row block = chunk
    const int r0 = team * 32;
    const int half = lane >> 5, l32 = lane & 31;
    if (threadIdx.x == 0) wg_abort = 0;
    // a team stopped by a cancel request in an earlier launch of the run keeps
    // its state; a stop step never lies beyond the end of its segment
    if constexpr (CANCEL) {
        const int ts0 = __hip_atomic_load(tstop + team, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ts0 >= 0 && ts0 <= g.seg_k0) return;  // whole workgroup
    }

    // Are all workgroups of this team on one XCD?  Each records (launch epoch,
    // XCD id) in its slot; lane k reads member k's slot.  Only then may the team
    // publish with XCD-scoped stores (readers always load at device scope, and
    // the step tags reject any stale word whatever the placement).
    const int my_xcc = xcc_id();
    // this launch's epoch (advanced on the stream before the launch, so that a
    // replayed launch differs from the previous one too)
    const uint32_t epoch = __hip_atomic_load(epoch_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) st_tagged(xslot + blockIdx.x, ((uint64_t)epoch << 32) | (uint32_t)my_xcc);
    bool xcd_local;
    {
        const int mb = 8 * (wpt * (tl >> 3) + (lane < wpt ? lane : 0)) + (tl & 7);
        uint64_t v = ld_tagged(xslot + mb);
        const uint64_t t0 = wall_clock64();
        bool ok = true;
        while (__any((uint32_t)(v >> 32) != epoch)) {
            __builtin_amdgcn_s_sleep(1);
            v = ld_tagged(xslot + mb);
            if (wall_clock64() - t0 > kTimeoutTicks) {
                ok = false;
                break;
            }
        }
        xcd_local = local_ok && ok && __all((int)(uint32_t)v == my_xcc);
    }

    v4i jr[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) jr[kb] = jpk[((size_t)rb * NKB + kb) * 64 + lane];
    const int one = 127;  // E8M0 block scale 2^0

    // item v: replica r0 + l%32, row 32 rb + 8(v/4) + 4(l/32) + v%4 (vectors
    // rather than arrays: the register allocator then keeps them in place
    // across the step loop instead of copying them every step)
    v16f xs, ys;
    const int rep = r0 + l32;
    const float gdt_heat = gamma[rep] * dt;
    // Nose-Hoover: xi(t_k) of this lane's replica; the heating rate of step k
    // is -xi(t_k) rounded to float, in eq. (22)'s place
    if constexpr (NH) {
        if (half == 0) s_xi[w][l32] = nhp.xi[rep];
    }
    const int rowb = rb * 32 + 4 * half;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = rowb + 8 * (v >> 2) + (v & 3);
        // + 0.0f turns a caller's -0.0 into +0.0, so that the sign bit of x is its
        // sgn (sgn(0) = +1); the update never produces -0.0 from a non-negative zero
        xs[v] = row < N ? X[(size_t)row * Rpad + rep] + 0.0f : 0.0f;
        ys[v] = row < N ? Y[(size_t)row * Rpad + rep] : 0.0f;
    }

    // Cancellation: the team's first wave reads the request at the start of
    // the launch and at each sample point; at the next sample point, if the
    // request was set, it records that sample point as the team's stop step
    // before it publishes the state of that step.  Every wave reads the record
    // at the sample point, once it has gathered that state (so all of them
    // see it), stops after the sample and writes its state back.  The host
    // word's trip is off the step's path: the value is used an interval later.
    const bool decider = CANCEL && cancel && __builtin_amdgcn_readfirstlane(rb) == 0;
    int creq = 0;
    if constexpr (CANCEL)
        if (decider) creq = __hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);

    // publish the sign word of the state x_m (tag m); snapshot at samples.
    // Lane l holds 16 rows of the block for replica l%32, lane l+32 the other
    // 16: the lower half of the wave stores the merged word.
    auto publish = [&](int m, bool sample, int sidx) {
        // b = (b << 1) | sign bit, highest item first: one operation per item
        uint32_t b = 0;
#pragma unroll
        for (int v = 15; v >= 0; --v) b = __builtin_amdgcn_alignbit(b, __float_as_uint(xs[v]), 31);
        const uint32_t got = (uint32_t)__shfl_xor((int)b, 32);
        const uint32_t word = b | (got << 16);
        const size_t slot = (size_t)rb * Rpad + rep;
        if constexpr (CANCEL) {
            if (sample) {
                // cancellation: the team's first wave records this sample point
                // as the team's stop step, before the words of this state, if
                // the request it last read was set
                if (decider && m < g.final_k && __builtin_amdgcn_readfirstlane(creq) != 0) {
                    if (lane == 0)
                        __hip_atomic_store(tstop + team, m, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                }
                if (half == 0) snap[(size_t)sidx * nchunk * Rpad + slot] = word;
            }
        }
        if (half == 0) {
            const uint64_t tagged = ((uint64_t)(uint32_t)m << 32) | word;
            if (xcd_local)
                st_tagged_xcd(xb + (size_t)(m & 1) * nchunk * Rpad + slot, tagged);
            else
                st_tagged(xb + (size_t)(m & 1) * nchunk * Rpad + slot, tagged);
            if constexpr (!CANCEL)
                if (sample) snap[(size_t)sidx * nchunk * Rpad + slot] = word;
        }
    };

    // thermostat: this wave's sum of y_i(t_m)^2 over its 32 rows (exact squares,
    // fixed order) into LDS, for the state about to be published.  A float's
    // square is exact in FP64, so one fused multiply-add per item rounds as
    // the product and the sum would.
    auto y2_partial = [&](int m) {
        if constexpr (NH) {
            double t2 = 0.0;
#pragma unroll
            for (int v = 0; v < 16; ++v) t2 = __fma_rn((double)ys[v], (double)ys[v], t2);
            t2 += __shfl_xor(t2, 32);
            if (half == 0) s_yw[m & 1][w][l32] = t2;
        }
    };
    // sample points: a uniform clock rather than two integer divisions per
    // step (measured 5% faster at the bench size)
    SampleClock clk(g);
    auto is_sample = [&](int m) { return clk.is_sample(g, m); };
    auto sample_index = [&](int m) { return clk.sample_index(g, m); };
    y2_partial(g.seg_k0);
    publish(g.seg_k0, is_sample(g.seg_k0), sample_index(g.seg_k0));
    __syncthreads();
    int stop_at = 0x7FFFFFFF;
    for (int m = g.seg_k0;; ++m) {
        const int buf = m & 1;
        // this wave's share: K block kb = w + 4q is chunk 2 kb + l/32
        const uint64_t *src = xb + ((size_t)buf * nchunk + 2 * w + half) * Rpad + r0 + l32;
        const float p = m < g.seg_k1 ? ptab[m - g.seg_k0] : 0.0f;  // issued early
        // Thermostat: half-wave q = 2 w + half needs the partials of
        // y(t_{m-1})^2 of workgroups q, q + 8 for xi(t_m).  Wave 0 of each
        // workgroup stored them a step ago, as tagged word pairs; they are
        // loaded here with the sign words and polled by their tags, and each
        // half-wave's sum goes to LDS before the barrier below.
        constexpr int WPT = NKB / 2;                 // workgroups of a team
        constexpr int NPL = (WPT + 7) / 8;          // partials per half-wave
        const bool nh_sum = NH && m > g.seg_k0;
        uint64_t pw_lo[NPL], pw_hi[NPL];
        auto part_slot = [&](int par, int wgi) {
            return nhp.ypart + (((size_t)par * (nchunk / 4) + wgi) * Rpad + rep) * 2;
        };
        if constexpr (NH) {
            if (nh_sum) {
#pragma unroll
                for (int q = 0; q < NPL; ++q) {
                    const int src_wg = 2 * w + half + 8 * q;
                    pw_lo[q] = pw_hi[q] = (uint64_t)(uint32_t)(m - 1) << 32;  // absent: zero
                    if (src_wg < nchunk / 4) {
                        const uint64_t *ps = part_slot((m - 1) & 1, src_wg);
                        pw_lo[q] = ld_tagged(ps);
                        pw_hi[q] = ld_tagged(ps + 1);
                    }
                }
            }
        }
        uint64_t wv[NQ];
        bool ok = gather_words<NQ>(wv, src, (size_t)8 * Rpad, NQ, (uint32_t)m, err);
        if constexpr (NH) {
            if (nh_sum && ok) {
                const uint32_t want = (uint32_t)(m - 1);
                const uint64_t t0 = wall_clock64();
                for (int it = 0;; ++it) {
                    bool stale = false;
#pragma unroll
                    for (int q = 0; q < NPL; ++q)
                        stale = stale || (uint32_t)(pw_lo[q] >> 32) != want ||
                                (uint32_t)(pw_hi[q] >> 32) != want;
                    if (!__any(stale)) break;
                    if ((it & 31) == 31 &&
                        (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                         wall_clock64() - t0 > kTimeoutTicks)) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int q = 0; q < NPL; ++q) {
                        const int src_wg = 2 * w + half + 8 * q;
                        if (src_wg < nchunk / 4) {
                            const uint64_t *ps = part_slot((m - 1) & 1, src_wg);
                            pw_lo[q] = ld_tagged(ps);
                            pw_hi[q] = ld_tagged(ps + 1);
                        }
                    }
                }
                double gs = 0.0;
#pragma unroll
                for (int q = 0; q < NPL; ++q)
                    gs += __longlong_as_double(
                        (long long)(((pw_hi[q] & 0xFFFFFFFFull) << 32) | (pw_lo[q] & 0xFFFFFFFFull)));
                s_ysum[m & 1][2 * w + half][l32] = gs;
            }
        }
        if (ok) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                a_lds[buf][w + 4 * q][lane] = expand_signs_fast((uint32_t)wv[q], 0x88888888u, 0x22222222u);
        } else {
            wg_abort = 1;
            __hip_atomic_fetch_or(status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (wg_abort) break;
        // Thermostat: wave 0 stores the workgroup's partial of y(t_m)^2 (the
        // four waves' in a fixed order) as a tagged word pair for step m + 1
        if constexpr (NH) {
            if (w == 0 && half == 0) {
                const double wsum = ((s_yw[m & 1][0][l32] + s_yw[m & 1][1][l32]) +
                                     s_yw[m & 1][2][l32]) + s_yw[m & 1][3][l32];
                const uint64_t bits = (uint64_t)__double_as_longlong(wsum);
                const uint64_t tag = (uint64_t)(uint32_t)m << 32;
                uint64_t *dst = part_slot(m & 1, kx % wpt);
                if (xcd_local) {
                    st_tagged_xcd(dst, tag | (bits & 0xFFFFFFFFull));
                    st_tagged_xcd(dst + 1, tag | (bits >> 32));
                } else {
                    st_tagged(dst, tag | (bits & 0xFFFFFFFFull));
                    st_tagged(dst + 1, tag | (bits >> 32));
                }
            }
        }
        // Thermostat: xi(t_m) = xi(t_{m-1}) + (dt/M)(sum_i y_i(t_{m-1})^2 - N T):
        // the eight half-wave sums (in LDS since the barrier) added pairwise in
        // a fixed order, the same in every wave of the team.  The operations
        // are spread between the products below, where a vector instruction
        // issues while the matrix core works, and xi(t_m) goes to LDS after
        // them (at the segment's first step it is the value read at launch).
        double nva = 0.0, nvb = 0.0, nsa = 0.0, nsb = 0.0, nxi = 0.0;
        if constexpr (NH) {
            nva = s_ysum[m & 1][0][l32];
            nvb = s_ysum[m & 1][1][l32];
            nxi = s_xi[w][l32];
        }
        auto nh_slot = [&](int kb) {
            if constexpr (NH) {
                if (kb == 2) {  // a = v0 + v1
                    nsa = nva + nvb;
                    nva = s_ysum[m & 1][2][l32];
                    nvb = s_ysum[m & 1][3][l32];
                } else if (kb == 4) {  // a = (v0 + v1) + (v2 + v3)
                    nsa = nsa + (nva + nvb);
                    nva = s_ysum[m & 1][4][l32];
                    nvb = s_ysum[m & 1][5][l32];
                } else if (kb == 6) {  // b = v4 + v5
                    nsb = nva + nvb;
                    nva = s_ysum[m & 1][6][l32];
                    nvb = s_ysum[m & 1][7][l32];
                } else if (kb == 8) {  // b = (v4 + v5) + (v6 + v7)
                    nsb = nsb + (nva + nvb);
                } else if (kb == 10) {  // S = a + b, then S - N T
                    nsa = (nsa + nsb) - nhp.NT;
                } else if (kb == 12) {
                    nsa = nhp.c * nsa;
                } else if (kb == 14) {
                    if (m > g.seg_k0) nxi = nxi + nsa;
                }
            }
        };
        v16f acc;
        // The products run at the lowest issue priority and the rest of the
        // step at a raised one: while the other wave on this SIMD is in its
        // products, this wave's update, publish and expansion -- the part of
        // its chain that its team waits for -- issue first.
        __builtin_amdgcn_s_setprio(0);
        // operand reads from LDS run kPre K blocks ahead of the products
        constexpr int kPre = KPRE < NKB ? KPRE : NKB;
        v4i af[kPre];
#pragma unroll
        for (int q = 0; q < kPre; ++q) af[q] = a_lds[buf][q][lane];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            const v4i a = af[kb % kPre];
            if (kb + kPre < NKB) af[kb % kPre] = a_lds[buf][kb + kPre][lane];
            if (kb == 0)
                mfma_fp4_first(acc, jr[0], a, one);
            else
                mfma_fp4(acc, jr[kb], a, one);
            nh_slot(kb);
        }
        if constexpr (NH) {
            if (NKB <= 14) {  // fewer products than slots: the rest of the chain
#pragma unroll
                for (int kb = NKB; kb <= 14; ++kb) nh_slot(kb);
            }
            if (half == 0) s_xi[w][l32] = nxi;
        }
        mfma_drain(acc);
        __builtin_amdgcn_s_setprio(3);
        if (is_sample(m)) {
            // eq. (1) partial over this wave's 32 rows of s_i f_i (exact integers/halves)
            const int j = sample_index(m);
            float part = 0.0f;
            bool fin = true;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                part += sgnf(xs[v]) * acc[v];
                fin = fin && isfinite(xs[v]) && isfinite(ys[v]);
            }
            part += __shfl_xor(part, 32);
            if (half == 0) ep[((size_t)j * nchunk + rb) * Rpad + rep] = part;
            if (tp) {  // sum of y_i^2 over the same rows (eq. (9)), exact squares
                double t = 0.0;
#pragma unroll
                for (int v = 0; v < 16; ++v) t += (double)ys[v] * (double)ys[v];
                t += __shfl_xor(t, 32);
                if (half == 0) tp[((size_t)j * nchunk + rb) * Rpad + rep] = t;
            }
            if (!fin) {
                bad[rep] = 1;
                __hip_atomic_fetch_or(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (CANCEL && cancel && m > g.seg_k0) {
                // the team's stop record (one word: wave-uniform, so the loop's
                // exit stays uniform); every word of x_m is in, and the record
                // was released before them
                if (!xcd_local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const int ts = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(tstop + team, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if (ts == m) stop_at = m;
                if (decider)  // the request, for the next sample point
                    creq = __hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        if (m == g.seg_k1 || (CANCEL && m == stop_at)) break;
        clk.pass(g, m);
        const bool next_sample = is_sample(m + 1);
        float gdt = gdt_heat;
        if constexpr (NH) gdt = (float)(-s_xi[w][l32]) * dt;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            float x = xs[v], y = ys[v];
            sb_update_tied(acc[v], p, c0, dt, a0dt, gdt, x, y);
            xs[v] = x;
            ys[v] = y;
        }
        publish(m + 1, next_sample, sample_index(m + 1));
        // after the publish, off the team's path: wave 0 reads it after the
        // next barrier
        y2_partial(m + 1);
    }
    // write the state back
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = rowb + 8 * (v >> 2) + (v & 3);
        if (row < N) {
            X[(size_t)row * Rpad + rep] = xs[v];
            Y[(size_t)row * Rpad + rep] = ys[v];
        }
    }
    if constexpr (NH) {  // xi after the segment's last step (every wave read it at the start)
        if (rb == 0 && half == 0 && !wg_abort) nhp.xi[rep] = s_xi[w][l32];
    }
}

// --------------------------------------------------- persistent bSB (FP4 digits)
//
// Field (eq. (4)): f = J x.  J is held exactly as FP4, as for dSB.  x is fed
// to the same FP4 x FP4 products as eight base-8 digits: for each 32-row
// chunk of one replica, with E the exponent of the chunk's largest |x|
// (max |x| <= 2^E, E clamped to [-100, 1]),
//   Q_i = rint(x_i 2^(22-E)),  |Q_i| <= 2^22,
//   Q_i + 0x924924 = sum_k u_ik 8^(7-k), u in [0, 7]  (balanced digits d = u - 4),
//   x_i = sum_k d_ik 2^(E-1-3k)  up to 2^(E-23).
// Every digit is an integer in [-4, 3], exact in E2M1, and digit k's weight
// 2^(E-1-3k) is the operand's per-lane E8M0 block scale (lane l's scale
// covers its 32 K values).  So f = sum_k J d_k 2^(E-1-3k) runs on the FP4
// matrix cores with FP32 accumulation: 8 products per K block per tile.
//
// Exchange.  Every step each wave writes, for its two chunks and the team's
// 32 replicas, the digit fragments already in the MFMA operand layout
// (16 bytes per lane per digit) and the chunk exponents, waits until its
// stores are done, then sets its step flag.  Readers poll the flags of the
// team, invalidate their L1 (agent-scope acquire) and stage the fragments
// through LDS in phases of 4 K blocks, double-buffered behind the products.
// Parity buffers by step: the writer of step m+2 has read all of step m+1,
// whose writers had finished reading step m.
// Samples: the sign words of each sampled state go to `snap`; the energies
// are formed after the launch (k_energy_fp4).

constexpr int kXD = 8;   // base-8 digits per x
constexpr int kPB = 4;   // K blocks per staging phase (one per wave)

// The same product with the B operand's block scale taken from byte BYTE of
// sb (four digits' scales packed in one register; op_sel / op_sel_hi bit 1
// give the byte index's low and high bit).  FRESH: sb was just computed by a
// vector instruction (two wait states first, as for mfma_fp4).
#define HSB_MFMA_FP4S(PRE, SEL, SRC_C, CONSTR)                                               \
    asm volatile(PRE "v_mfma_scale_f32_32x32x64_f8f6f4 %0, %1, %2, " SRC_C ", %3, %4 " SEL  \
                 " cbsz:4 blgp:4"                                                            \
                 : CONSTR(acc)                                                               \
                 : "a"(j), "v"(b), "v"(sa), "v"(sb))
#define HSB_MFMA_FP4S_BYTE(PRE, SRC_C, CONSTR)                                                \
    if constexpr (BYTE == 0) HSB_MFMA_FP4S(PRE, "op_sel_hi:[0,0,0]", SRC_C, CONSTR);          \
    else if constexpr (BYTE == 1)                                                            \
        HSB_MFMA_FP4S(PRE, "op_sel:[0,1,0] op_sel_hi:[0,0,0]", SRC_C, CONSTR);                \
    else if constexpr (BYTE == 2) HSB_MFMA_FP4S(PRE, "op_sel_hi:[0,1,0]", SRC_C, CONSTR);     \
    else HSB_MFMA_FP4S(PRE, "op_sel:[0,1,0] op_sel_hi:[0,1,0]", SRC_C, CONSTR)
template <int BYTE, bool FRESH>
__device__ __forceinline__ void mfma_fp4s(v16f &acc, const v4i &j, const v4i &b, int sa, int sb) {
    if constexpr (FRESH) { HSB_MFMA_FP4S_BYTE("s_nop 1\n\t", "%0", "+v"); }
    else { HSB_MFMA_FP4S_BYTE("", "%0", "+v"); }
}
template <int BYTE, bool FRESH>
__device__ __forceinline__ void mfma_fp4s_first(v16f &acc, const v4i &j, const v4i &b, int sa,
                                                int sb) {
    if constexpr (FRESH) { HSB_MFMA_FP4S_BYTE("s_nop 1\n\t", "0", "=&v"); }
    else { HSB_MFMA_FP4S_BYTE("", "0", "=&v"); }
}
#undef HSB_MFMA_FP4S_BYTE
#undef HSB_MFMA_FP4S

__device__ __forceinline__ uint32_t ld_flag(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Direct load of 16 bytes per lane from global memory (wave-uniform base
// plus the lane's 32-bit byte offset) into LDS at lds_base + 16 lane
// (wave-uniform), device scope (the L1 is bypassed).  Written as assembly so
// that the compiler does not track it: it would otherwise make reads of the
// other staging buffers wait for it.  The caller waits for it (vmcnt) and
// synchronises the workgroup before any wave reads the bytes; the compiler's
// own vmcnt waits only get stricter from the extra loads in flight.
__device__ __forceinline__ void lds_load16(const void *base, uint32_t lane_off, uint32_t lds_base) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1 sc1"
                 :
                 : "v"(lane_off), "s"(base), "s"(lds_base)
                 : "memory", "m0");
}

// Digit fragments of one tile.  Lane (h, l%32) holds 16 rows (item v: row
// 8(v/4) + 4h + v%4 of the chunk) of replica l%32.  Returns the biased
// exponent E + 128 of the chunk and fills frag[j][q] (j = 0..3) with the four
// complete 16-byte fragments of digits 4h + j: dword q of digit k holds the
// rows of word bits 4n + 3 - q (n = 0..7), the low half from the lane with
// h = 0, the high half from its partner l^32.
//   Per item, the eight octal digits of U are spread to one byte each (two
// words: digits 7,5,3,1 and 6,4,2,0) and mapped to E2M1 codes by a byte
// table lookup.  Per q, the codes of the four items 3-q, 7-q, 11-q, 15-q
// are merged nibble-wise and regrouped by byte permutes into dwords holding
// the half-words of two digits; one cross-half swap per pair of dwords gives
// each lane its own and its partner's half-words of the digits it keeps.
__device__ __forceinline__ uint32_t make_digits(const float (&xs)[16], int half, v4i (&frag)[4]) {
    float mx = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) mx = fmaxf(mx, fabsf(xs[v]));
    {
        const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(mx), __float_as_uint(mx),
                                                        false, false);
        mx = fmaxf(mx, __uint_as_float(half ? s[0] : s[1]));  // the partner's maximum
    }
    int E = (int)((__float_as_uint(mx) >> 23) & 0xFFu) - 126;  // mx < 2^E for normal mx
    E = E < -100 ? -100 : (E > 1 ? 1 : E);
    const float sc = __uint_as_float((uint32_t)(149 - E) << 23);  // 2^(22 - E)
    // E2M1 codes of d = u - 4 for u = 0..7 (bytes of the lookup table):
    // -4 -3 -2 -1 0 1 2 3
    constexpr uint32_t kLutHi = 0x05040200u, kLutLo = 0x0A0C0D0Eu;
    uint32_t cl[16], ch[16];  // codes of digits 7,5,3,1 / 6,4,2,0, one per byte
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const uint32_t U = (uint32_t)((int)rintf(xs[v] * sc) + 0x924924);
        // octal digit i (bits 3i..3i+2) to bits 0-2 (i even) or 3-5 (i odd) of byte i/2
        const uint32_t w1 = (U & 0xFFFu) | ((U & 0xFFF000u) << 4);
        const uint32_t w2 = (w1 & 0x003F003Fu) | ((w1 & 0x0FC00FC0u) << 2);
        cl[v] = __builtin_amdgcn_perm(kLutHi, kLutLo, w2 & 0x07070707u);
        ch[v] = __builtin_amdgcn_perm(kLutHi, kLutLo, (w2 >> 3) & 0x07070707u);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int a = 3 - q, b = 7 - q, c = 11 - q, d = 15 - q;  // nibbles n = 0..3
        const uint32_t abl = cl[a] | (cl[b] << 4), cdl = cl[c] | (cl[d] << 4);
        const uint32_t abh = ch[a] | (ch[b] << 4), cdh = ch[c] | (ch[d] << 4);
        // half-words of digits (7, 5), (3, 1), (6, 4), (2, 0)
        const uint32_t p75 = __builtin_amdgcn_perm(cdl, abl, 0x05010400u);
        const uint32_t p31 = __builtin_amdgcn_perm(cdl, abl, 0x07030602u);
        const uint32_t p64 = __builtin_amdgcn_perm(cdh, abh, 0x05010400u);
        const uint32_t p20 = __builtin_amdgcn_perm(cdh, abh, 0x07030602u);
        // lanes h = 0 keep digits 0-3, lanes h = 1 digits 4-7; after the swap
        // [0] holds the low-half lane's dword and [1] the high-half lane's
        const auto sa = __builtin_amdgcn_permlane32_swap(p31, p75, false, false);
        const auto sb = __builtin_amdgcn_permlane32_swap(p20, p64, false, false);
        frag[0][q] = (int)__builtin_amdgcn_perm(sb[1], sb[0], 0x07060302u);  // digit 0 / 4
        frag[1][q] = (int)__builtin_amdgcn_perm(sa[1], sa[0], 0x07060302u);  // digit 1 / 5
        frag[2][q] = (int)__builtin_amdgcn_perm(sb[1], sb[0], 0x05040100u);  // digit 2 / 6
        frag[3][q] = (int)__builtin_amdgcn_perm(sa[1], sa[0], 0x05040100u);  // digit 3 / 7
    }
    return (uint32_t)(E + 128);
}

// The Nose-Hoover thermostat inside the persistent bSB kernel (eqs. (6)-(8)):
// xi per replica ([Rpad], FP64: its value at the segment's first step in, at
// the step after its last out), and every wave's partial sum of y_i(t_m)^2
// over its 64 rows ([2 step parities][row blocks][Rpad], FP64), stored with
// the digits of x_{m+1} before the step flag that publishes them.
struct BsbNH {
    double *xi;
    double *part;
    double c, NT;
};

// CANCEL: the variant that honours hsb_cancel, as for the dSB kernel.
// NH: the thermostat (not combined with CANCEL).
template <int NKB, int KPRE, bool CANCEL, bool NH>
__global__ __launch_bounds__(256, 1) void k_bsb_fp4(
    const FP4Team *__restrict__ teams, float *__restrict__ X, float *__restrict__ Y,
    const float *__restrict__ gamma, v4i *xd, uint8_t *xe, uint32_t *flags,
    uint32_t *__restrict__ snap, double *__restrict__ tp, const float *__restrict__ ptab,
    int32_t *__restrict__ bad,
    int32_t *__restrict__ status, int32_t *err, uint64_t *xslot, const uint32_t *epoch_p,
    int local_ok, const int32_t *cancel, int32_t *tstop, BsbNH nhp,
    int nkb, int nrb, int Rpad, int team0, int nteams, SegArgs g, float dt, float a0dt) {
    static_assert(NKB % 4 == 0, "Npad is a multiple of 256");
    static_assert(!(NH && CANCEL), "the thermostat variant takes no cancel requests");
    constexpr int NPH = NKB / kPB;  // staging phases per step
    // thermostat: the eight half-waves' sums of the team's partials, and
    // xi(t_m) of the workgroup's 32 replicas (one copy per wave)
    __shared__ double s_bpart[NH ? 2 : 1][8][32];
    __shared__ double s_bxi[NH ? 4 : 1][32];
    // three staging buffers (phase ph uses buffer ph % 3): separate arrays, so
    // that the compiler sees that reading one does not wait for the direct
    // loads into the others
    __shared__ v4i f_b0[kPB][kXD][64], f_b1[kPB][kXD][64], f_b2[kPB][kXD][64];
    __shared__ int wg_abort;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wu = __builtin_amdgcn_readfirstlane(w);  // the same, known to be wave-uniform
    const int wpt = nrb >> 2;
    const int xcd = blockIdx.x & 7, kx = blockIdx.x >> 3;
    const int tl = (kx / wpt) * 8 + xcd;
    if (tl >= nteams) return;
    const int team = team0 + tl;
    const v4i *__restrict__ jpk = static_cast<const v4i *>(teams[team].jpk);
    const int N = teams[team].N;
    const float c0 = teams[team].c0;
    const int rb = (kx % wpt) * 4 + wu;  // uniform: its addresses stay in scalar registers
    const int r0 = team * 32;
    const int nchunk = 2 * nrb;
    const int half = lane >> 5, l32 = lane & 31;
    const size_t cols = (size_t)2 * Rpad;  // exchange columns: team * 64 + lane
    const int col = team * 64 + lane;
    uint32_t *myflag = flags + (size_t)team * nrb + rb;
    if (threadIdx.x == 0) wg_abort = 0;
    // a team stopped by a cancel request in an earlier launch keeps its state
    if constexpr (CANCEL) {
        const int ts0 = __hip_atomic_load(tstop + team, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ts0 >= 0 && ts0 <= g.seg_k0) return;  // whole workgroup
    }

    const int my_xcc = xcc_id();
    // this launch's epoch (advanced on the stream before the launch, so that a
    // replayed launch differs from the previous one too)
    const uint32_t epoch = __hip_atomic_load(epoch_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) st_tagged(xslot + blockIdx.x, ((uint64_t)epoch << 32) | (uint32_t)my_xcc);
    bool xcd_local;
    {
        const int mb = 8 * (wpt * (tl >> 3) + (lane < wpt ? lane : 0)) + (tl & 7);
        uint64_t v = ld_tagged(xslot + mb);
        const uint64_t t0 = wall_clock64();
        bool ok = true;
        while (__any((uint32_t)(v >> 32) != epoch)) {
            __builtin_amdgcn_s_sleep(1);
            v = ld_tagged(xslot + mb);
            if (wall_clock64() - t0 > kTimeoutTicks) {
                ok = false;
                break;
            }
        }
        xcd_local = local_ok && ok && __all((int)(uint32_t)v == my_xcc);
    }

    v4i jr0[NKB], jr1[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        jr0[kb] = jpk[((size_t)(rb * 2 + 0) * NKB + kb) * 64 + lane];
        jr1[kb] = jpk[((size_t)(rb * 2 + 1) * NKB + kb) * 64 + lane];
    }
    const int one = 127;

    float xs0[16], xs1[16], ys0[16], ys1[16];
    const int rep = r0 + l32;
    const float gdt_heat = gamma[rep] * dt;
    // thermostat: xi(t_k) of this lane's replica; the heating rate of step k
    // is -xi(t_k) rounded to float, in eq. (22)'s place
    if constexpr (NH) {
        if (half == 0) s_bxi[wu][l32] = nhp.xi[rep];
    }
    const int rowb = rb * 64 + 4 * half;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row0 = rowb + 8 * (v >> 2) + (v & 3), row1 = row0 + 32;
        xs0[v] = row0 < N ? X[(size_t)row0 * Rpad + rep] : 0.0f;
        xs1[v] = row1 < N ? X[(size_t)row1 * Rpad + rep] : 0.0f;
        ys0[v] = row0 < N ? Y[(size_t)row0 * Rpad + rep] : 0.0f;
        ys1[v] = row1 < N ? Y[(size_t)row1 * Rpad + rep] : 0.0f;
    }

    // publish the digits of x_m: fragments of chunk 2 rb + t go to K block rb,
    // consumer half t; then the step flag
    // (thermostat: with the partial t2 of y(t_{m-1})^2 over the wave's rows)
    auto publish = [&](int m, double t2) {
        const int par = m & 1;
        if constexpr (NH) {
            if (half == 0) nhp.part[((size_t)((m - 1) & 1) * nrb + rb) * Rpad + rep] = t2;
        }
        v4i fr[4];
        uint32_t eb = make_digits(xs0, half, fr);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            xd[(((size_t)par * nkb + rb) * kXD + 4 * half + j) * cols + team * 64 + l32] = fr[j];
        if (half == 0) xe[((size_t)par * cols + team * 64 + l32) * nkb + rb] = (uint8_t)eb;
        eb = make_digits(xs1, half, fr);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            xd[(((size_t)par * nkb + rb) * kXD + 4 * half + j) * cols + team * 64 + 32 + l32] = fr[j];
        if (half == 0) xe[((size_t)par * cols + team * 64 + 32 + l32) * nkb + rb] = (uint8_t)eb;
        // release: the fragments are in the L2 before the flag
        if (xcd_local) {
            // stores acknowledged by the shared L2 (the memory clobber keeps them
            // above); the flag only has to reach that L2 too
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (lane == 0) __hip_atomic_store(myflag, (uint32_t)m, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) __hip_atomic_store(myflag, (uint32_t)m, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    // sign words of the sampled state x_m (the energy is formed afterwards)
    auto snapshot = [&](int sidx) {
        uint32_t b0 = 0, b1 = 0;
        bool fin = true;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            b0 |= (xs0[v] >= 0.0f ? 0u : 1u) << v;
            b1 |= (xs1[v] >= 0.0f ? 0u : 1u) << v;
            fin = fin && isfinite(xs0[v]) && isfinite(xs1[v]) && isfinite(ys0[v]) && isfinite(ys1[v]);
        }
        const uint32_t got = (uint32_t)__shfl_xor((int)(half ? b0 : b1), 32);
        const uint32_t word = half ? (got | (b1 << 16)) : (b0 | (got << 16));
        const size_t slot = (size_t)(rb * 2 + half) * Rpad + rep;
        snap[(size_t)sidx * nchunk * Rpad + slot] = word;
        if (tp) {  // sum of y_i^2 over the wave's 64 rows (eq. (9)), exact squares
            double t = 0.0;
#pragma unroll
            for (int v = 0; v < 16; ++v)
                t += (double)ys0[v] * (double)ys0[v] + (double)ys1[v] * (double)ys1[v];
            t += __shfl_xor(t, 32);
            if (half == 0) tp[((size_t)sidx * nrb + rb) * Rpad + rep] = t;
        }
        if (!fin) {
            bad[rep] = 1;
            __hip_atomic_fetch_or(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };

    if (g.seg_k0 < g.seg_k1) publish(g.seg_k0, 0.0);
    SampleClock clk(g);  // sample points without a division per step
    for (int m = g.seg_k0;; ++m) {
        // the energy of a sampled state needs only its signs
        const bool sample = clk.is_sample(g, m);
        if (sample) snapshot(clk.sample_index(g, m));
        // (with the thermostat the segment's last step published x_{k1} and its
        // partials too: xi(t_{k1}) is formed below before the loop ends)
        if (!NH && m == g.seg_k1) break;
        if (NH && m == g.seg_k1 && g.seg_k0 == g.seg_k1) break;  // no step: xi as it came
        clk.pass(g, m);
        const int par = m & 1;
        // (the thermostat's last pass, m = k1, takes no step)
        const float p = !NH || m < g.seg_k1 ? ptab[m - g.seg_k0] : 0.0f;
        // wait for every wave of the team to have published x_m
        {
            const uint32_t *fp = flags + (size_t)team * nrb + (lane < nrb ? lane : 0);
            uint32_t f = ld_flag(fp);
            const uint64_t t0 = wall_clock64();
            int it = 0;
            while (__any((uint32_t)(f - (uint32_t)m) > 1u)) {
                __builtin_amdgcn_s_sleep(1);
                f = ld_flag(fp);
                if ((++it & 31) == 0) {
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        wall_clock64() - t0 > kTimeoutTicks) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_or(status, 2, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                        wg_abort = 1;
                        break;
                    }
                }
            }
            // readers on another L2: invalidate for the data written there
            if (!xcd_local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if constexpr (NH) {
            // thermostat: half-wave q = 2 w + h adds the partials of y(t_{m-1})^2
            // of row blocks q, q + 8, ... (stored with x_m before the flags just
            // seen; device-scope loads), into LDS for the barrier below
            if (m > g.seg_k0) {
                const uint64_t *pin =
                    reinterpret_cast<const uint64_t *>(nhp.part + (size_t)((m - 1) & 1) * nrb * Rpad);
                double Ssum = 0.0;
                for (int q = 2 * wu + half; q < nrb; q += 8)
                    Ssum += __longlong_as_double((long long)ld_tagged(pin + (size_t)q * Rpad + rep));
                s_bpart[m & 1][2 * wu + half][l32] = Ssum;
            }
            if (m == g.seg_k1) {
                // the segment's end: xi(t_{k1}) (as every step forms it) out
                __syncthreads();
                if (!wg_abort) {
                    double v8[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) v8[q] = s_bpart[m & 1][q][l32];
                    const double S = ((v8[0] + v8[1]) + (v8[2] + v8[3])) +
                                     ((v8[4] + v8[5]) + (v8[6] + v8[7]));
                    const double xi_k = s_bxi[wu][l32] + nhp.c * (S - nhp.NT);
                    if (rb == 0 && half == 0) nhp.xi[rep] = xi_k;
                }
                break;
            }
        }
        if constexpr (CANCEL) {
            if (cancel) {
                // cancellation: the first wave of the team has recorded this
                // sample point as the stop step before publishing x_m; the
                // state x_m and its sample are kept
                if (m > g.seg_k0 && sample) {
                    const int ts =
                        __hip_atomic_load(tstop + team, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (__builtin_amdgcn_readfirstlane(ts) == m) break;
                }
                // on the step before a sample point the first wave reads the
                // request and records the decision; the release of its publish
                // at the end of this step orders it before the step flag (here,
                // not between the update and the publish, where a branch would
                // split their schedule)
                if (rb == 0 && m + 1 < g.seg_k1 && clk.is_sample(g, m + 1)) {
                    const int c = __hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (__builtin_amdgcn_readfirstlane(c) != 0 && lane == 0)
                        __hip_atomic_store(tstop + team, m + 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        // chunk exponents of this lane's column for every K block (device-scope
        // loads: no stale L1 lines)
        uint32_t ed[NKB / 4];
        {
            const uint32_t *ep4 =
                reinterpret_cast<const uint32_t *>(xe + ((size_t)par * cols + col) * nkb);
#pragma unroll
            for (int q = 0; q < NKB / 4; ++q) ed[q] = ld_flag(ep4 + q);
            // consumed here, before the direct loads below are in flight: a
            // later compiler wait for them would also wait for those loads
#pragma unroll
            for (int q = 0; q < NKB / 4; ++q) asm volatile("" : "+v"(ed[q]));
        }
        // staging: wave w loads the fragments of K block kPB ph + w of phase ph
        // straight into LDS (device scope: no stale L1 lines), two phases
        // ahead of the products.  Every access names its buffer directly (one
        // branch per buffer, resolved when the phase loop is unrolled), so the
        // compiler can tell the buffers apart and does not make the reads of
        // one wait for the loads into another.
        // fragment (kb, k) of this step: row (par nkb + kb) kXD + k of xd, the
        // lane's column col (uniform row base, per-lane byte offset 16 col)
        auto dma_into = [&](v4i(&dst)[kPB][kXD][64], int ph) {
            const int kb = kPB * ph + wu;
#pragma unroll
            for (int k = 0; k < kXD; ++k) {
                const v4i *row = xd + (((size_t)par * nkb + kb) * kXD + k) * cols;
                lds_load16(row, (uint32_t)col * 16u,
                           (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void *)&dst[wu][k][0]);
            }
        };
        auto load_stage = [&](int ph) {
            if (ph % 3 == 0) dma_into(f_b0, ph);
            else if (ph % 3 == 1) dma_into(f_b1, ph);
            else dma_into(f_b2, ph);
        };
        // this wave's loads of phase ph are in LDS when at most the kXD loads of
        // phase ph+1 are outstanding; the barrier then covers all waves'.  (A
        // bare barrier: __syncthreads would also wait for the loads in flight.)
        auto wait_stage = [&](int ph) {
            if (ph + 1 < NPH)
                asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __builtin_amdgcn_s_barrier();
        };
        static_assert(kXD == 8, "the wait above counts kXD loads per phase");
        load_stage(0);
        if (NPH > 1) load_stage(1);
        asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)" ::: "memory");
        if (NPH == 1) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();  // also publishes wg_abort (and the thermostat's sums)
        if (wg_abort) break;
        if constexpr (NH) {
            // xi(t_m) = xi(t_{m-1}) + (dt/M)(sum_i y_i(t_{m-1})^2 - N T): the eight
            // half-wave sums added pairwise, the same in every wave of the team
            if (m > g.seg_k0) {
                double v8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v8[q] = s_bpart[m & 1][q][l32];
                const double S = ((v8[0] + v8[1]) + (v8[2] + v8[3])) +
                                 ((v8[4] + v8[5]) + (v8[6] + v8[7]));
                const double xi_k = s_bxi[wu][l32] + nhp.c * (S - nhp.NT);
                if (half == 0) s_bxi[wu][l32] = xi_k;
            }
        }
        v16f acc0, acc1;
        // the products of phase ph, operands from its buffer
        auto products = [&](const v4i(&src)[kPB][kXD][64], int ph) {
            // operand reads from LDS run kPre fragments ahead of the products
            constexpr int kPre = KPRE, kFr = kPB * kXD;
            v4i af[kPre];
#pragma unroll
            for (int q = 0; q < kPre; ++q) af[q] = src[q / kXD][q % kXD][lane];
            // scale of digit k of K block kb: 127 + (E - 1 - 3k) = e - 2 - 3k (E = e - 128),
            // bytes k = 0..3 in sbp[0] and 4..7 in sbp[1]: the exponent byte of kb
            // copied to all four bytes, less 2 + 3k per byte (e >= 28: no borrows)
            int sbp[2];
#pragma unroll
            for (int fi = 0; fi < kFr; ++fi) {
                const int kl = fi / kXD, k = fi % kXD;
                const int kb = kPB * ph + kl;
                const v4i a = af[fi % kPre];
                if (fi + kPre < kFr) af[fi % kPre] = src[(fi + kPre) / kXD][(fi + kPre) % kXD][lane];
                if (k == 0) {
                    const uint32_t rep = __builtin_amdgcn_perm(0u, ed[kb >> 2], 0x01010101u * (kb & 3));
                    sbp[0] = (int)(rep - 0x0B080502u);
                    sbp[1] = (int)(rep - 0x1714110Eu);
                }
                const int sb = sbp[k >> 2];
                auto pair = [&](auto byte) {
                    constexpr int B = decltype(byte)::value;
                    // sb is new at k = 0 and k = 4 (computed by vector
                    // instructions just before): wait states before its first use
                    if (kb == 0 && k == 0) {
                        mfma_fp4s_first<B, true>(acc0, jr0[0], a, one, sb);
                        mfma_fp4s_first<B, false>(acc1, jr1[0], a, one, sb);
                    } else if ((k & 3) == 0) {
                        mfma_fp4s<B, true>(acc0, jr0[kb], a, one, sb);
                        mfma_fp4s<B, false>(acc1, jr1[kb], a, one, sb);
                    } else {
                        mfma_fp4s<B, false>(acc0, jr0[kb], a, one, sb);
                        mfma_fp4s<B, false>(acc1, jr1[kb], a, one, sb);
                    }
                };
                switch (k & 3) {
                case 0: pair(std::integral_constant<int, 0>{}); break;
                case 1: pair(std::integral_constant<int, 1>{}); break;
                case 2: pair(std::integral_constant<int, 2>{}); break;
                default: pair(std::integral_constant<int, 3>{}); break;
                }
            }
        };
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
            if (ph + 2 < NPH) load_stage(ph + 2);
            if (ph % 3 == 0) products(f_b0, ph);
            else if (ph % 3 == 1) products(f_b1, ph);
            else products(f_b2, ph);
            if (ph + 1 < NPH) wait_stage(ph + 1);
        }
        mfma_drain(acc0, acc1);
        float gdt = gdt_heat;
        double t2 = 0.0;  // thermostat: this wave's sum of y_i(t_m)^2 (exact squares)
        if constexpr (NH) {
            gdt = (float)(-s_bxi[wu][l32]) * dt;
#pragma unroll
            for (int v = 0; v < 16; ++v) t2 = __fma_rn((double)ys0[v], (double)ys0[v], t2);
#pragma unroll
            for (int v = 0; v < 16; ++v) t2 = __fma_rn((double)ys1[v], (double)ys1[v], t2);
            t2 += __shfl_xor(t2, 32);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            sb_update(acc0[v], p, c0, dt, a0dt, gdt, xs0[v], ys0[v]);
            sb_update(acc1[v], p, c0, dt, a0dt, gdt, xs1[v], ys1[v]);
        }
        // with the thermostat the last step publishes too: its partials give
        // xi(t_{k1}) at the segment's end
        if (m + 1 < g.seg_k1 || NH) publish(m + 1, t2);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row0 = rowb + 8 * (v >> 2) + (v & 3), row1 = row0 + 32;
        if (row0 < N) {
            X[(size_t)row0 * Rpad + rep] = xs0[v];
            Y[(size_t)row0 * Rpad + rep] = ys0[v];
        }
        if (row1 < N) {
            X[(size_t)row1 * Rpad + rep] = xs1[v];
            Y[(size_t)row1 * Rpad + rep] = ys1[v];
        }
    }
}

// Energy partials of sampled states from their sign words (eq. (1)):
// F = J sgn(x) on the FP4 matrix cores, then per wave sum_i s_i F_i of its 64
// rows.  Grid (teams x row-block groups, samples), 256 threads.
template <int NKB>
__global__ __launch_bounds__(256) void k_energy_fp4(const FP4Team *__restrict__ teams,
                                                    const uint32_t *__restrict__ snap,
                                                    float *__restrict__ ep, int nrb, int Rpad,
                                                    int team0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wpt = nrb >> 2;
    const int team = team0 + blockIdx.x / wpt;
    const int rb = (blockIdx.x % wpt) * 4 + w;
    const int j = blockIdx.y;
    const int nchunk = 2 * nrb;
    const int half = lane >> 5, l32 = lane & 31;
    const int rep = team * 32 + l32;
    const v4i *__restrict__ jpk = static_cast<const v4i *>(teams[team].jpk);
    const uint32_t *sw = snap + (size_t)j * nchunk * Rpad;
    v16f acc0 = {}, acc1 = {};
#pragma unroll 4
    for (int kb = 0; kb < NKB; ++kb) {
        const v4i a = expand_signs(sw[(size_t)(2 * kb + half) * Rpad + rep]);
        const v4i j0 = jpk[((size_t)(rb * 2 + 0) * NKB + kb) * 64 + lane];
        const v4i j1 = jpk[((size_t)(rb * 2 + 1) * NKB + kb) * 64 + lane];
        v8i a8 = {a[0], a[1], a[2], a[3], 0, 0, 0, 0};
        v8i b0 = {j0[0], j0[1], j0[2], j0[3], 0, 0, 0, 0};
        v8i b1 = {j1[0], j1[1], j1[2], j1[3], 0, 0, 0, 0};
        acc0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b0, a8, acc0, 4, 4, 0, 127, 0, 127);
        acc1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b1, a8, acc1, 4, 4, 0, 127, 0, 127);
    }
    // signs of this wave's rows: word bit of row t in chunk 2 rb + tile
    const uint32_t w0 = sw[(size_t)(2 * rb) * Rpad + rep];
    const uint32_t w1 = sw[(size_t)(2 * rb + 1) * Rpad + rep];
    float part = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int t = 8 * (v >> 2) + 4 * half + (v & 3);
        const float s0 = ((w0 >> row_word_bit(t)) & 1u) ? -1.0f : 1.0f;
        const float s1 = ((w1 >> row_word_bit(t)) & 1u) ? -1.0f : 1.0f;
        part += s0 * acc0[v] + s1 * acc1[v];
    }
    part += __shfl_xor(part, 32);
    if (half == 0) ep[((size_t)j * nrb + rb) * Rpad + rep] = part;
}

// Energy of sample j of replica r (eq. (1)): -1/2 times the sum of its nparts
// partials (one per row block of the kernel that formed them).  Every partial
// is a multiple of 1/2 below 2^23 in magnitude, so the FP64 totals are exact
// in any order.  Grid (Rpad/256, samples), one thread per (replica, sample).
__global__ __launch_bounds__(256) void k_fp4_energies(const float *__restrict__ ep,
                                                      double *__restrict__ es, int nparts,
                                                      int Rpad) {
    const int r = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (r >= Rpad) return;
    const float *p = ep + (size_t)j * nparts * Rpad + r;
    double e = 0.0;
    for (int b = 0; b < nparts; ++b) e += (double)p[(size_t)b * Rpad];
    es[(size_t)j * Rpad + r] = -0.5 * e;
}

// Traces of the segment's samples: row row0 + j of trace_e / trace_t ([.][R])
// receives sample j's energy and T_inst = (1/N) sum_i y_i^2 (eq. (9)), the
// latter from the nparts FP64 partial sums, added in a fixed order.  Grid
// (R/256, samples), one thread per (replica, sample).
__global__ __launch_bounds__(256) void k_fp4_trace(const double *__restrict__ es,
                                                   const double *__restrict__ tp, int nparts,
                                                   int N, int R, int Rpad, int row0,
                                                   double *__restrict__ trace_e,
                                                   double *__restrict__ trace_t) {
    const int r = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (r >= R) return;
    const size_t o = (size_t)(row0 + j) * R + r;
    if (trace_e) trace_e[o] = es[(size_t)j * Rpad + r];
    if (trace_t) {
        const double *q = tp + (size_t)j * nparts * Rpad + r;
        double t = 0.0;
        for (int b = 0; b < nparts; ++b) t += q[(size_t)b * Rpad];
        trace_t[o] = t / N;
    }
}

// Best-sample update of the segment's samples and its spins.  Grid Rpad/32,
// 256 threads: lane group g = threadIdx.x / 32 scans samples j = g, g + 8, ...
// of 32 replicas; the groups' minima are merged with the earliest sample
// winning ties, then the winning sample's sign words are decoded into best_s.
__global__ __launch_bounds__(256) void k_fp4_best(
    const double *__restrict__ es, const uint32_t *__restrict__ snap, int ns, int nchunk,
    int N, int R, int Rpad, SegArgs g, double *__restrict__ best_e, double *__restrict__ last_e,
    int32_t *__restrict__ best_step, const int32_t *__restrict__ bad, int8_t *__restrict__ best_s,
    const int32_t *__restrict__ tstop) {
    __shared__ double s_e[8][32];
    __shared__ int s_j[8][32];
    const int rl = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int r = blockIdx.x * 32 + rl;
    double emin = __builtin_huge_val();
    int jmin = -1;
    // a team stopped by a cancel request: only its samples up to the stop step
    // exist, and the one at the stop step is its last
    const int ts = tstop[blockIdx.x];  // 32 replicas = one team
    auto step_of = [&](int j) {
        return j < g.nmult ? (g.seg_k0 / g.interval + 1 + j) * g.interval : g.final_k;
    };
    if (r < R) {
        for (int j = grp; j < ns; j += 8) {
            if (ts >= 0 && step_of(j) > ts) continue;
            const double e = es[(size_t)j * Rpad + r];
            if (ts >= 0 ? step_of(j) == ts : j == ns - 1) last_e[r] = bad[r] ? __builtin_nan("") : e;
            if (e < emin) {
                emin = e;
                jmin = j;
            }
        }
    }
    s_e[grp][rl] = emin;
    s_j[grp][rl] = jmin;
    __syncthreads();
    if (grp == 0) {
        for (int q = 1; q < 8; ++q) {
            const double e = s_e[q][rl];
            const int j = s_j[q][rl];
            if (j >= 0 && (e < emin || (e == emin && j < jmin))) {
                emin = e;
                jmin = j;
            }
        }
        const bool take = r < R && jmin >= 0 && !bad[r] && emin < best_e[r];
        if (take) {
            best_e[r] = emin;
            best_step[r] = jmin < g.nmult ? (g.seg_k0 / g.interval + 1 + jmin) * g.interval
                                          : g.final_k;
        }
        s_j[0][rl] = take ? jmin : -1;
    }
    __syncthreads();
    const int bj = s_j[0][rl];
    if (r >= R || bj < 0) return;
    for (int i = grp; i < N; i += 8) {
        const uint32_t w = snap[((size_t)bj * nchunk + (i >> 5)) * Rpad + r];
        best_s[(size_t)i * Rpad + r] = ((w >> row_word_bit(i & 31)) & 1u) ? -1 : 1;
    }
}

// ------------------------------------------------------------------- host

namespace {

// Result-invariant variants of the persistent kernels (the autotuner's
// candidates): how many K blocks (dSB) or digit fragments (bSB) ahead of the
// products the operand is read from LDS.  Candidate 0 is the default.
constexpr int kDsbPre[] = {2, 1, 4};
constexpr int kBsbPre[] = {4, 2};

// tile -1: the thermostat's kernel (operand read one K block ahead: the
// registers of a further prefetch hold the thermostat's partials)
template <int NKB>
const void *dsb_ptr(int tile, bool cancel) {
    if (cancel) switch (tile) {
        case -1: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, 2, true, true>);
        case 1: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, kDsbPre[1], false, true>);
        case 2: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, kDsbPre[2], false, true>);
        default: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, kDsbPre[0], false, true>);
        }
    switch (tile) {
    case -1: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, 2, true, true>);
    case 1: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, kDsbPre[1], false, false>);
    case 2: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, kDsbPre[2], false, false>);
    default: return reinterpret_cast<const void *>(&k_dsb_fp4<NKB, kDsbPre[0], false, false>);
    }
}

const void *pick_kernel(int nkb, int tile, bool cancel) {
    switch (nkb) {
    case 4: return dsb_ptr<4>(tile, cancel);
    case 8: return dsb_ptr<8>(tile, cancel);
    case 12: return dsb_ptr<12>(tile, cancel);
    case 16: return dsb_ptr<16>(tile, cancel);
    case 20: return dsb_ptr<20>(tile, cancel);
    case 24: return dsb_ptr<24>(tile, cancel);
    case 28: return dsb_ptr<28>(tile, cancel);
    default: return dsb_ptr<32>(tile, cancel);
    }
}

template <int NKB>
const void *bsb_ptr(int tile, bool cancel, bool nh) {
    if (nh) return reinterpret_cast<const void *>(&k_bsb_fp4<NKB, kBsbPre[0], false, true>);
    if (cancel)
        return tile == 1 ? reinterpret_cast<const void *>(&k_bsb_fp4<NKB, kBsbPre[1], true, false>)
                         : reinterpret_cast<const void *>(&k_bsb_fp4<NKB, kBsbPre[0], true, false>);
    return tile == 1 ? reinterpret_cast<const void *>(&k_bsb_fp4<NKB, kBsbPre[1], false, false>)
                     : reinterpret_cast<const void *>(&k_bsb_fp4<NKB, kBsbPre[0], false, false>);
}

const void *pick_bsb_kernel(int nkb, int tile, bool cancel, bool nh) {
    switch (nkb) {
    case 4: return bsb_ptr<4>(tile, cancel, nh);
    case 8: return bsb_ptr<8>(tile, cancel, nh);
    case 12: return bsb_ptr<12>(tile, cancel, nh);
    case 16: return bsb_ptr<16>(tile, cancel, nh);
    case 20: return bsb_ptr<20>(tile, cancel, nh);
    case 24: return bsb_ptr<24>(tile, cancel, nh);
    case 28: return bsb_ptr<28>(tile, cancel, nh);
    default: return bsb_ptr<32>(tile, cancel, nh);
    }
}

hipError_t launch_energy_fp4(int nkb, dim3 grid, const FP4Team *teams, const uint32_t *snap,
                             float *ep, int nrb, int Rpad, int team0, hipStream_t s) {
#define HSB_ENERGY_CASE(K)                                                                  \
    case K:                                                                                 \
        hipLaunchKernelGGL(k_energy_fp4<K>, grid, dim3(256), 0, s, teams, snap, ep, nrb, Rpad, \
                           team0);                                                          \
        break;
    switch (nkb) {
        HSB_ENERGY_CASE(4)
        HSB_ENERGY_CASE(8)
        HSB_ENERGY_CASE(12)
        HSB_ENERGY_CASE(16)
        HSB_ENERGY_CASE(20)
        HSB_ENERGY_CASE(24)
        HSB_ENERGY_CASE(28)
        default: HSB_ENERGY_CASE(32)
    }
#undef HSB_ENERGY_CASE
    return hipGetLastError();
}

// p_k = a0 - a(t_k) with a(t_k) = a0 k / Ns, for k = k0 .. k0 + n - 1: the
// same single-precision operations, in the same order and rounding, as the
// host's table of the other plans.
__global__ void k_fill_ptab(float *ptab, int k0, int n, float a0, float Ns_f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float ak = __fdiv_rn(__fmul_rn(a0, (float)(k0 + i)), Ns_f);
    ptab[i] = __fsub_rn(a0, ak);
}

// Next launch epoch: never 0xFFFFFFFF, the value the slots are filled with.
__global__ void k_next_epoch(uint32_t *epoch) {
    uint32_t e = epoch[0] + 1u;
    if (e == 0xFFFFFFFFu) e = 1u;
    epoch[0] = e;
}

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

template <typename T>
int grow(T **p, size_t *cap, size_t n) {
    if (n <= *cap) return HSB_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess)
        return perr(e == hipErrorOutOfMemory ? HSB_ENOMEM : HSB_EDEVICE, "persistent scratch: %s",
                    hipGetErrorString(e));
    *cap = n;
    return HSB_OK;
}

}  // namespace

int persistent_create(const float *J, int N, PersistentJ **out) {
    *out = nullptr;
    if (!persistent_supported(N)) return perr(HSB_EUNSUPPORTED, "N=%d too large for FP4 path", N);
    PersistentJ *pj = new PersistentJ;
    pj->N = N;
    pj->Npad = (N + 255) / 256 * 256;  // four row blocks of 64 per workgroup
    pj->nkb = pj->Npad / 64;
    pj->nrb = pj->Npad / 64;
    const size_t np = (size_t)pj->Npad;
    std::vector<float> padded(np * np, 0.0f);
    for (int i = 0; i < N; ++i)
        std::memcpy(&padded[(size_t)i * np], J + (size_t)i * N, sizeof(float) * N);
    float *dJ = nullptr;
    const size_t frags = (size_t)pj->nrb * 2 * pj->nkb * 64;
    hipError_t e = hipMalloc((void **)&dJ, np * np * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&pj->jpk, frags * sizeof(v4i));
    if (e == hipSuccess)
        e = hipMemcpy(dJ, padded.data(), np * np * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pack_fp4, dim3((unsigned)((frags + 255) / 256)), dim3(256), 0, 0, dJ,
                           pj->jpk, pj->Npad, pj->nkb, pj->nrb);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (dJ) (void)hipFree(dJ);
    if (e != hipSuccess) {
        persistent_free(pj);
        return perr(e == hipErrorOutOfMemory ? HSB_ENOMEM : HSB_EDEVICE, "FP4 J store: %s",
                    hipGetErrorString(e));
    }
    *out = pj;
    return HSB_OK;
}

int persistent_nkb(const PersistentJ *pj) { return pj->nkb; }
uint64_t persistent_gen(const PersistentJ *pj) { return pj->work.gen; }
const void *persistent_jpk(const PersistentJ *pj) { return pj->jpk; }

int persistent_work_create(PersistentWork **out) {
    *out = new (std::nothrow) PersistentWork;
    return *out ? HSB_OK : perr(HSB_ENOMEM, "persistent scratch: host allocation");
}

void persistent_work_free(PersistentWork *w) {
    if (!w) return;
    void *ptrs[] = {w->xb, w->snap, w->ep, w->es, w->tp, w->ptab, w->err, w->xslot, w->epoch,
                    w->teams, w->xd, w->xe, w->flags, w->tstop, w->ypart, w->bpart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete w;
}

void persistent_free(PersistentJ *pj) {
    if (!pj) return;
    PersistentWork &w = pj->work;
    void *ptrs[] = {pj->jpk, w.xb, w.snap, w.ep, w.es, w.tp, w.ptab, w.err, w.xslot, w.epoch,
                    w.teams, w.xd, w.xe, w.flags, w.tstop, w.ypart, w.bpart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete pj;
}

int persistent_run(PersistentJ *pj, int variant, const PersistentRun &run, StateBufs &b, int N,
                   hipStream_t s, KernelTimer &timer) {
    std::vector<FP4Team> teams((size_t)run.Rpad / 32);
    for (FP4Team &t : teams) {
        t.jpk = pj->jpk;
        t.N = N;
        t.c0 = run.c0;
    }
    return persistent_run_teams(&pj->work, variant, pj->nkb, teams.data(), (int)teams.size(), run,
                                b, N, s, timer);
}

namespace {

// Teams per launch and workgroups per team of a persistent launch: a multiple
// of 8 teams (one slot per XCD) whose workgroups all fit on the device at once.
// Waves hold 64 rows (bSB) or 32 rows (dSB); so do the energy partials.
int launch_shape(bool bsb, int nkb, int tile, bool cancel, int *teams_per_launch, int *wpt,
                 int *wg_capacity) {
    int dev = 0, ncu = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, bsb ? pick_bsb_kernel(nkb, tile, cancel, tile < 0) : pick_kernel(nkb, tile, cancel),
            256, 0);
    if (e != hipSuccess) return perr(HSB_EDEVICE, "FP4 path: %s", hipGetErrorString(e));
    const int nparts = bsb ? nkb : 2 * nkb;
    *wg_capacity = nb * ncu;
    *wpt = nparts / 4;
    *teams_per_launch = 8 * (*wg_capacity / (8 * *wpt));
    if (*teams_per_launch < 8)
        return perr(HSB_EUNSUPPORTED, "FP4 path: %d resident workgroups < 8 teams of %d",
                    *wg_capacity, *wpt);
    return HSB_OK;
}

// The launch sequence of a run whose buffers in pw are in place (sized for
// nteams_total teams over run.Rpad columns and seg_samples samples per
// segment) and whose team table is on the device: per segment of at most
// seg_samples sample points, the persistent launches of all teams, then the
// sample energies, the best-sample update and the traces.
int run_segments(PersistentWork *pw, int variant, int nkb, int nteams_total, int teams_per_launch,
                 int wpt, size_t seg_samples, const PersistentRun &run, StateBufs &b, int Nrows,
                 hipStream_t s, KernelTimer &timer) {
    const bool bsb = variant == HSB_BSB;
    const int Rpad = run.Rpad, nrb = nkb, nchunk = 2 * nrb;
    const int nparts = bsb ? nrb : nchunk;
    const int interval = run.interval;
    const bool traces = b.trace_e || b.trace_t;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, pw->err);
    // no team has stopped (cancellation), for the whole run
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nteams_total + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<uint32_t *>(pw->tstop), (size_t)nteams_total, kNoTag);
    b.tstop = pw->tstop;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return perr(HSB_EDEVICE, "%s", hipGetErrorString(e));
    const float a0dt = run.a0 * run.dt;
    const bool nh = run.nh != nullptr;
    const void *kfn = bsb ? pick_bsb_kernel(nkb, run.tile, run.cancel != nullptr, nh)
                          : pick_kernel(nkb, nh ? -1 : run.tile, run.cancel != nullptr);
    FP4NH nhp{};
    BsbNH bnh{};
    if (nh && !bsb) nhp = FP4NH{run.nh->xi, pw->ypart, run.nh->c, run.nh->NT};
    if (nh && bsb) bnh = BsbNH{run.nh->xi, pw->bpart, run.nh->c, run.nh->NT};
    int a = run.k0;
    for (;;) {
        // segment [a, e]: at most seg_samples multiples of interval in (a, e]
        long long e_ll = ((long long)a / interval + (long long)seg_samples) * interval;
        const int e_k = e_ll < run.k1 ? (int)e_ll : run.k1;
        SegArgs g;
        g.seg_k0 = a;
        g.seg_k1 = e_k;
        g.final_k = run.k1;
        g.interval = interval;
        g.nmult = e_k / interval - a / interval;
        const int ns = g.nmult + ((e_k == run.k1 && (e_k % interval != 0 || e_k == a)) ? 1 : 0);
        if (e_k > a) {  // p_k of the segment's steps, on the device (no host round trip)
            hipLaunchKernelGGL(k_fill_ptab, dim3((unsigned)((e_k - a + 255) / 256)), dim3(256), 0,
                               s, pw->ptab, a, e_k - a, run.a0, (float)run.Ns);
            e = hipGetLastError();
            if (e != hipSuccess) return perr(HSB_EDEVICE, "%s", hipGetErrorString(e));
        }
        for (int t0 = 0; t0 < nteams_total; t0 += teams_per_launch) {
            int nt = nteams_total - t0 < teams_per_launch ? nteams_total - t0 : teams_per_launch;
            if (bsb) {  // no wave of this launch has published yet
                const size_t nf = (size_t)nteams_total * nrb;
                hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s,
                                   pw->flags, nf, kNoTag);
            } else {
                const size_t nxb = (size_t)2 * nchunk * Rpad;
                hipLaunchKernelGGL(k_fill_tags, dim3((unsigned)((nxb + 255) / 256)), dim3(256), 0,
                                   s, pw->xb, nxb);
                if (nh) {  // no thermostat partial of an earlier launch carries a live tag
                    const size_t np = (size_t)4 * (nchunk / 4) * Rpad;
                    hipLaunchKernelGGL(k_fill_tags, dim3((unsigned)((np + 255) / 256)), dim3(256), 0,
                                       s, pw->ypart, np);
                }
            }
            // block b -> team (b/8)/wpt*8 + b%8: round the team count up to 8
            const dim3 grid((unsigned)(8 * ((nt + 7) / 8) * wpt)), block(256);
            float dt = run.dt, a0dtv = a0dt;
            int nkb_v = nkb, nrb_v = nrb, nchunk_v = nchunk, Rpad_v = Rpad, t0_v = t0, nt_v = nt;
            hipLaunchKernelGGL(k_next_epoch, dim3(1), dim3(1), 0, s, pw->epoch);
            int local_ok = run.local_exchange ? 1 : 0;
            const int32_t *cancel = run.cancel;
            const float *gam = run.gamma;
            double *tpv = traces ? pw->tp : nullptr;
            void *args_d[] = {(void *)&pw->teams, (void *)&run.X,    (void *)&run.Y,
                              (void *)&gam,       (void *)&pw->xb,   (void *)&pw->snap,
                              (void *)&pw->ep,    (void *)&tpv,      (void *)&pw->ptab,
                              (void *)&b.bad,
                              (void *)&b.status,  (void *)&pw->err,  (void *)&pw->xslot,
                              (void *)&pw->epoch, (void *)&local_ok, (void *)&cancel,
                              (void *)&pw->tstop, (void *)&nhp,   (void *)&nkb_v,
                              (void *)&nchunk_v,  (void *)&Rpad_v,   (void *)&t0_v,
                              (void *)&nt_v,      (void *)&g,        (void *)&dt,
                              (void *)&a0dtv};
            void *args_b[] = {(void *)&pw->teams, (void *)&run.X,     (void *)&run.Y,
                              (void *)&gam,       (void *)&pw->xd,    (void *)&pw->xe,
                              (void *)&pw->flags, (void *)&pw->snap,  (void *)&tpv,
                              (void *)&pw->ptab,
                              (void *)&b.bad,     (void *)&b.status,  (void *)&pw->err,
                              (void *)&pw->xslot, (void *)&pw->epoch, (void *)&local_ok,
                              (void *)&cancel,    (void *)&pw->tstop, (void *)&bnh,
                              (void *)&nkb_v,     (void *)&nrb_v,     (void *)&Rpad_v,
                              (void *)&t0_v,      (void *)&nt_v,      (void *)&g,
                              (void *)&dt,        (void *)&a0dtv};
            void **args = bsb ? args_b : args_d;
            // every workgroup of the grid is resident at once: the grid never exceeds
            // the occupancy-derived capacity, and every wait inside the kernel is
            // bounded, so a wave that cannot make progress ends the launch cleanly
            e = timer.begin(s);
            if (e == hipSuccess) e = hipLaunchKernel(kfn, grid, block, args, 0, s);
            if (e == hipSuccess) e = timer.end(s);
            if (e != hipSuccess)
                return perr(HSB_EDEVICE, "FP4 persistent launch: %s", hipGetErrorString(e));
        }
        if (bsb && ns > 0) {  // energies of the segment's samples from their sign words
            e = launch_energy_fp4(nkb, dim3((unsigned)(nteams_total * wpt), (unsigned)ns),
                                  pw->teams, pw->snap, pw->ep, nrb, Rpad, 0, s);
            if (e != hipSuccess) return perr(HSB_EDEVICE, "%s", hipGetErrorString(e));
        }
        if (ns > 0)
            hipLaunchKernelGGL(k_fp4_energies, dim3((unsigned)((Rpad + 255) / 256), (unsigned)ns),
                               dim3(256), 0, s, pw->ep, pw->es, nparts, Rpad);
        hipLaunchKernelGGL(k_fp4_best, dim3((unsigned)((run.R + 31) / 32)), dim3(256), 0, s,
                           pw->es, pw->snap, ns, nchunk, Nrows, run.R, Rpad, g, b.best_e, b.last_e,
                           b.best_step, b.bad, b.best_s, pw->tstop);
        if (traces && ns > 0)  // rows of the segment's samples: after those of (k0, a]
            hipLaunchKernelGGL(k_fp4_trace, dim3((unsigned)((run.R + 255) / 256), (unsigned)ns),
                               dim3(256), 0, s, pw->es, pw->tp, nparts, Nrows, run.R, Rpad,
                               a / interval - run.k0 / interval, b.trace_e, b.trace_t);
        e = hipGetLastError();
        if (e != hipSuccess) return perr(HSB_EDEVICE, "%s", hipGetErrorString(e));
        if (e_k >= run.k1) break;
        a = e_k;
    }
    // an exchange wait that timed out sets bit 1 of the run's status word,
    // which the caller reads with the rest of the status after its output
    return HSB_OK;
}

// Every entry of the team table: the same instance (J fragments, N, c0).
__global__ void k_fill_teams(FP4Team *teams, int n, const void *jpk, int N, float c0) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) teams[t] = FP4Team{jpk, N, c0};
}

}  // namespace

int persistent_run_teams(PersistentWork *pw, int variant, int nkb, const FP4Team *host_teams,
                         int nteams_total, const PersistentRun &run, StateBufs &b, int Nrows,
                         hipStream_t s, KernelTimer &timer) {
    const bool bsb = variant == HSB_BSB;
    const int Rpad = run.Rpad, nrb = nkb, nchunk = 2 * nrb;
    if (nteams_total * 32 > Rpad) return perr(HSB_EINVAL, "FP4 path: teams exceed the columns");
    int teams_per_launch = 0, wpt = 0, wg_capacity = 0;
    if (run.nh && bsb && run.cancel)
        return perr(HSB_EUNSUPPORTED, "FP4 path: no cancellable thermostat run for bSB");
    int rc = launch_shape(bsb, nkb, run.nh ? -1 : run.tile, run.cancel != nullptr, &teams_per_launch,
                          &wpt, &wg_capacity);
    if (rc) return rc;
    const int nparts = bsb ? nrb : nchunk;
    const int interval = run.interval;
    // samples per launch bounded by a 512 MiB snapshot budget (and 4096)
    const size_t snap_per_sample = (size_t)nchunk * Rpad;
    size_t seg_samples = ((size_t)512 << 20) / (snap_per_sample * 4);
    if (seg_samples > 4096) seg_samples = 4096;
    if (seg_samples < 1) seg_samples = 1;
    const bool traces = b.trace_e || b.trace_t;
    const void *const before[] = {pw->xb, pw->snap, pw->ep, pw->es, pw->tp, pw->ptab, pw->err,
                                  pw->teams, pw->xd, pw->xe, pw->flags, pw->xslot, pw->epoch,
                                  pw->tstop, pw->ypart, pw->bpart};
    rc = grow(&pw->xb, &pw->xb_words, (size_t)2 * nchunk * Rpad);
    if (!rc) rc = grow(&pw->snap, &pw->snap_words, (seg_samples + 1) * snap_per_sample);
    if (!rc) rc = grow(&pw->ep, &pw->ep_elems, (seg_samples + 1) * (size_t)nparts * Rpad);
    if (!rc) rc = grow(&pw->es, &pw->es_elems, (seg_samples + 1) * (size_t)Rpad);
    if (!rc && traces) {  // partials of at most the run's own samples per segment
        const size_t run_samples = (size_t)(run.k1 / interval - run.k0 / interval) + 1;
        const size_t tps = run_samples < seg_samples + 1 ? run_samples : seg_samples + 1;
        rc = grow(&pw->tp, &pw->tp_elems, tps * (size_t)nparts * Rpad);
    }
    const long long max_seg_steps = (long long)seg_samples * interval;
    const int ptab_need = (int)((long long)(run.k1 - run.k0) < max_seg_steps
                                    ? (run.k1 - run.k0)
                                    : max_seg_steps);
    if (!rc) rc = grow(&pw->ptab, &pw->ptab_elems, (size_t)(ptab_need > 0 ? ptab_need : 1));
    size_t one = 0;
    if (!rc && !pw->err) rc = grow(&pw->err, &one, 1);
    if (!rc) {
        const FP4Team *before = pw->teams;
        rc = grow(&pw->teams, &pw->teams_n, (size_t)nteams_total);
        if (pw->teams != before) pw->teams_up.clear();  // a new buffer holds no table yet
    }
    if (!rc && bsb) rc = grow(&pw->xd, &pw->xd_n, (size_t)2 * nkb * 8 * 2 * Rpad);
    if (!rc && bsb) rc = grow(&pw->xe, &pw->xe_n, (size_t)2 * 2 * Rpad * nkb);
    if (!rc && bsb) rc = grow(&pw->flags, &pw->flags_n, (size_t)nteams_total * nrb);
    if (!rc) rc = grow(&pw->tstop, &pw->tstop_n, (size_t)nteams_total);
    if (!rc && run.nh && !bsb) rc = grow(&pw->ypart, &pw->ypart_n, (size_t)4 * (nchunk / 4) * Rpad);
    if (!rc && run.nh && bsb) rc = grow(&pw->bpart, &pw->bpart_n, (size_t)2 * nrb * Rpad);
    if (!rc && !pw->epoch) {
        rc = grow(&pw->epoch, &pw->epoch_n, 1);
        if (!rc) {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, pw->epoch, (size_t)1, 0u);
            if (hipGetLastError() != hipSuccess) rc = perr(HSB_EDEVICE, "epoch fill failed");
        }
    }
    if (!rc && pw->xslot_n < (size_t)wg_capacity + 8 * (size_t)wpt) {
        rc = grow(&pw->xslot, &pw->xslot_n, (size_t)wg_capacity + 8 * (size_t)wpt);
        if (!rc) {  // epoch 0xFFFFFFFF in every slot: never a launch's epoch
            hipLaunchKernelGGL(k_fill_tags, dim3((unsigned)((pw->xslot_n + 255) / 256)), dim3(256), 0,
                               s, pw->xslot, pw->xslot_n);
            if (hipGetLastError() != hipSuccess) rc = perr(HSB_EDEVICE, "xslot fill failed");
        }
    }
    if (rc) return rc;
    {
        const void *const after[] = {pw->xb, pw->snap, pw->ep, pw->es, pw->tp, pw->ptab, pw->err,
                                     pw->teams, pw->xd, pw->xe, pw->flags, pw->xslot, pw->epoch,
                                     pw->tstop, pw->ypart, pw->bpart};
        if (std::memcmp(before, after, sizeof(before)) != 0) ++pw->gen;
    }
    // the team table, uploaded only when it differs from the last upload (a
    // repeated run then queues no host-to-device copy)
    if (pw->teams_up.size() != (size_t)nteams_total ||
        std::memcmp(pw->teams_up.data(), host_teams, sizeof(FP4Team) * (size_t)nteams_total) != 0) {
        hipError_t e = hipMemcpyAsync(pw->teams, host_teams, sizeof(FP4Team) * (size_t)nteams_total,
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // host_teams may go away after return
        if (e != hipSuccess) return perr(HSB_EDEVICE, "%s", hipGetErrorString(e));
        pw->teams_up.assign(host_teams, host_teams + nteams_total);
        ++pw->gen;
    }
    return run_segments(pw, variant, nkb, nteams_total, teams_per_launch, wpt, seg_samples, run, b,
                        Nrows, s, timer);
}

// Scratch layout of a dSB run of the FP4 plan in caller-given memory: every
// buffer of the run's work, 256-byte aligned, carved in order from `base`.
// With base == nullptr only the size is computed.
namespace {
struct Carver {
    uint8_t *base;
    size_t used = 0;
    template <typename T>
    T *take(size_t n) {
        used = (used + 255) / 256 * 256;
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += n * sizeof(T);
        return p;
    }
};
void carve_dsb_work(Carver &c, PersistentWork &w, int nkb, int nteams, int Rpad, size_t seg,
                    size_t ptab_n, size_t nslots) {
    const size_t nchunk = 2 * (size_t)nkb;
    w.xb = c.take<uint64_t>(2 * nchunk * Rpad);
    w.snap = c.take<uint32_t>((seg + 1) * nchunk * Rpad);
    w.ep = c.take<float>((seg + 1) * nchunk * Rpad);
    w.es = c.take<double>((seg + 1) * (size_t)Rpad);
    w.ptab = c.take<float>(ptab_n);
    w.err = c.take<int32_t>(1);
    w.epoch = c.take<uint32_t>(1);
    w.xslot = c.take<uint64_t>(nslots);
    w.teams = c.take<FP4Team>((size_t)nteams);
    w.tstop = c.take<int32_t>((size_t)nteams);
}
}  // namespace

int persistent_run_in(void *scratch, size_t bytes, const PersistentJ *pj, const PersistentRun &run,
                      StateBufs &b, int Nrows, hipStream_t s) {
    const int nkb = pj->nkb, Rpad = run.Rpad, nteams = Rpad / 32;
    int teams_per_launch = 0, wpt = 0, wg_capacity = 0;
    int rc = launch_shape(false, nkb, run.tile, run.cancel != nullptr, &teams_per_launch, &wpt,
                          &wg_capacity);
    if (rc) return rc;
    const size_t nslots = (size_t)wg_capacity + 8 * (size_t)wpt;
    const int interval = run.interval;
    // the most samples per segment that fit (at most the run's own, and 4096)
    const size_t run_samples = (size_t)(run.k1 / interval - run.k0 / interval) + 1;
    size_t seg = run_samples < 4096 ? run_samples : 4096;
    auto need = [&](size_t sg) {
        const long long steps = (long long)sg * interval;
        const size_t ptab_n = (size_t)((long long)(run.k1 - run.k0) < steps ? (run.k1 - run.k0)
                                                                            : steps) + 1;
        Carver c{nullptr};
        PersistentWork w;
        carve_dsb_work(c, w, nkb, nteams, Rpad, sg, ptab_n, nslots);
        return std::pair<size_t, size_t>(c.used, ptab_n);
    };
    while (seg > 1 && need(seg).first > bytes) seg /= 2;
    const auto nd = need(seg);
    if (nd.first > bytes)
        return perr(HSB_EINVAL, "the run needs %zu bytes of work space, %zu are left in the "
                                "fixed scratch", nd.first, bytes);
    Carver c{static_cast<uint8_t *>(scratch)};
    PersistentWork w;
    carve_dsb_work(c, w, nkb, nteams, Rpad, seg, nd.second, nslots);
    // the buffers sit wherever this call's sizes put them, so the placement
    // slots and the launch epoch start afresh (slot tag 0xFFFFFFFF is never an
    // epoch), and the team table is written on the device
    hipLaunchKernelGGL(k_fill_tags, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s,
                       w.xslot, nslots);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, w.epoch, (size_t)1, 0u);
    hipLaunchKernelGGL(k_fill_teams, dim3((unsigned)((nteams + 255) / 256)), dim3(256), 0, s,
                       w.teams, nteams, (const void *)pj->jpk, pj->N, run.c0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return perr(HSB_EDEVICE, "%s", hipGetErrorString(e));
    KernelTimer off;
    rc = run_segments(&w, HSB_DSB, nkb, nteams, teams_per_launch, wpt, seg, run, b, Nrows, s, off);
    // w points into the caller's scratch: nothing of it is freed
    w = PersistentWork{};
    return rc;
}

}  // namespace hsb
