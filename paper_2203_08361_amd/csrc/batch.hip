// Batched discrete SB on the FP4 plan: every job of a batch in one persistent
// launch.
//
// A batch mixes instances of different sizes N_i <= 2048 (the uneven instance
// sets and parameter sweeps of the Results section), each run by many
// replicas at its own c0 and heating rate.  Its unit of work is a team: 32
// replicas of one job, run for all steps by Npad_i / 128 workgroups that
// exchange their sign words every step, exactly as a single run's teams do
// (field eq. (5), update eqs. (16)-(22), exact FP4 products).  Here one
// persistent grid, as large as the device holds at once, serves all teams:
//
//   * eight job queues, one per XCD slot (workgroup b serves queue b % 8, and
//     the dispatcher places block b on XCD b % 8, so a team's workgroups share
//     one L2).  A queue lists, for every team given to it, one entry per
//     workgroup of the team, teams one after another.  A workgroup takes the
//     next entry (an atomic counter), runs that part of its team to the end
//     of the run, and takes the next.  A team's entries are consecutive, so at
//     most one team of a queue is partly taken at any time and the others
//     finish: with at least 16 workgroups per queue no team waits for ever.
//   * the host fills the queues longest-first, each team to the queue with
//     the least estimated work (workgroups x step time), so the queues end
//     together and large instances do not start last.
//   * the team's instance (its FP4 J fragments, N, the K-block count, c0,
//     gamma, seed) comes from a per-team table: one compiled kernel serves
//     every size, looping over the team's own K blocks.
//   * the initial state is drawn inside the kernel from the counter-based
//     generator; no state array exists.
//   * energies (eq. (1)) and the best sample are tracked inside the kernel: at
//     a sample point each wave writes sum_i s_i f_i of its 32 rows (the field
//     of that state is the one it just formed), and at the next step -- once
//     every wave of the team has published the following state, which it does
//     only after that partial is stored -- every wave adds the team's partials
//     in FP64 (multiples of 1/2: exact in any order) and keeps the best (strict
//     improvement, earliest wins) with its own chunk's sign word.  The last
//     sample gets one extra exchange round.  Each wave finally writes the best
//     (or final) spins of its rows into the job's output.
// Nothing waits on the host between the start of the launch and its end.
#include "batch.h"
#include "fp4_device.h"
#include "hsb.h"
#include "hsb_device.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>

namespace hsb {

namespace {

constexpr int kQKB = 32;                         // K blocks of the largest instance
constexpr int kQChunks = 2 * kQKB;               // 32-row chunks of the largest instance
constexpr size_t kTeamWords = 2 * kQChunks * 32;  // per-team exchange entries (two parities)
constexpr int kMaxWpt = kQChunks / 4;            // workgroups of the largest team

thread_local char q_err[256] = "";
int qerr(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(q_err, sizeof(q_err), fmt, ap);
    va_end(ap);
    return code;
}

__device__ __forceinline__ uint32_t ld_word(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

const char *queue_error() { return q_err; }

// ----------------------------------------------------------------- device

// Shared memory of a workgroup of the queue kernel.
struct QShared {
    v4i a_lds[2][kQKB][64];  // the +-1 operand of the current step, ping-pong
    // best-sample tracking of each wave's replicas, touched only at sample
    // points: best energy, and the sign words of this wave's chunk at the best
    // and at the pending (not yet evaluated) sample
    double beste[4][32];
    uint32_t wbest[4][64], wpend[4][64];
    int unit, entry, abort;
};

struct QArgs {
    uint64_t *xb;
    uint32_t *ep;
    const float *ptab;
    double *best_e, *last_e;
    int32_t *bad, *status, *err;
    int steps, interval, return_best;
    int nteams;  // teams of the batch: the stride of the exchange layout
    float dt, a0dt, amp;
};

// One workgroup's part of a team whose instance has NKB K blocks: waves
// rb = 4 member + w, all steps of the run, then the outputs of its rows.
// Returns false if an exchange wait ended the run (err or timeout).
template <int NKB>
__device__ __forceinline__ bool run_unit(QShared &sh, const QTeam &tm, int team, int rb,
                                         bool xcd_local, const QArgs &g) {
    constexpr int NQ = NKB / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int one = 127;  // E8M0 block scale 2^0
    const int N = tm.N, steps = g.steps;
    // sample points m = interval, 2 interval, ... and the last step, as a
    // running clock (no division per step)
    int next_mult = g.interval;
    auto is_sample = [&](int m) { return m == steps || m == next_mult; };

    // the wave's 32 rows of J (FP4 fragments, accumulation registers)
    const v4i *__restrict__ jpk = static_cast<const v4i *>(tm.jpk);
    v4i jr[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) jr[kb] = jpk[((size_t)rb * NKB + kb) * 64 + lane];

    // the seeded initial state of the team's replicas (zero in padding)
    const int rep = tm.rep0 + l32;
    const bool live = l32 < tm.nrep;
    const float c0 = tm.c0;
    const float gdt = live ? tm.gamma * g.dt : 0.0f;
    const int rowb = rb * 32 + 4 * half;
    v16f xs, ys;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = rowb + 8 * (v >> 2) + (v & 3);
        const bool ok = live && row < N;
        xs[v] = ok ? g.amp * uniform_open(rng_key(tm.seed, 0, (uint64_t)rep, (uint64_t)row)) : 0.0f;
        ys[v] = ok ? g.amp * uniform_open(rng_key(tm.seed, 1, (uint64_t)rep, (uint64_t)row)) : 0.0f;
    }

    // Exchange entries (sign words, energy partials) of parity p and chunk c:
    // the 32 replicas of a team side by side, the teams of the batch side by
    // side, then chunks, then parities -- one chunk's entries of all teams
    // form one row, as a single run's columns of replicas do.
    const size_t tstride = (size_t)g.nteams * 32;  // one chunk of every team
    uint64_t *xbt = g.xb + (size_t)team * 32;
    uint32_t *ept = g.ep + (size_t)team * 32;
    // sign word of the current state's chunk for this lane's replica (bit b
    // < 16 from the lower half of the wave, b >= 16 from the upper half)
    auto cur_word = [&]() -> uint32_t {
        uint32_t bsig = 0;
#pragma unroll
        for (int v = 15; v >= 0; --v)
            bsig = __builtin_amdgcn_alignbit(bsig, __float_as_uint(xs[v]), 31);
        const uint32_t got = (uint32_t)__shfl_xor((int)bsig, 32);
        return half ? (got | (bsig << 16)) : (bsig | (got << 16));
    };
    // the lower half of the wave stores the word, tagged with the step
    auto publish = [&](int m) {
        const uint32_t word = cur_word();
        if (half == 0) {
            uint64_t *dst = xbt + ((size_t)(m & 1) * kQChunks + rb) * tstride + l32;
            const uint64_t tagged = ((uint64_t)(uint32_t)m << 32) | word;
            if (xcd_local)
                st_tagged_xcd(dst, tagged);
            else
                st_tagged(dst, tagged);
        }
    };
    // The partials of a sample are stored before the next published word:
    // acknowledged by the shared L2 (team on one XCD) or released to the device
    // (team spread over XCDs).
    auto release_partial = [&]() {
        if (xcd_local)
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        else
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    };
    // eq. (1) of the sample whose partials are in parity sp: -1/2 the sum of
    // the team's 2 NKB partials (each a multiple of 1/2 below 2^23, so the FP64
    // sum is exact and the same in every wave)
    auto team_energy = [&](int sp) -> double {
        if (!xcd_local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint32_t *src = ept + (size_t)sp * kQChunks * tstride + l32;
        double S = 0.0;
#pragma unroll 8
        for (int c = 0; c < 2 * NKB; ++c) S += (double)__uint_as_float(ld_word(src + c * tstride));
        return -0.5 * S;
    };
    // the best of the samples evaluated so far (strict improvement: the
    // earliest of equal energies stays)
    auto consider = [&](double E) {
        if (E < sh.beste[w][l32]) {
            sh.wbest[w][lane] = sh.wpend[w][lane];
            if (half == 0) sh.beste[w][l32] = E;
        }
    };
    if (half == 0) sh.beste[w][l32] = __builtin_huge_val();
    sh.wbest[w][lane] = 0;
    bool pend = false;  // a sample whose energy is not formed yet
    int sp = 0;         // parity of the next sample's partials

    publish(0);
    for (int m = 0;; ++m) {
        const int buf = m & 1;
        // this wave's share of the operand: K block kb = w + 4q is chunk 2 kb + l/32
        const uint64_t *src = xbt + ((size_t)buf * kQChunks + 2 * w + half) * tstride + l32;
        const float p = m < steps ? g.ptab[m] : 0.0f;
        uint64_t wv[NQ];
        if (gather_words<NQ>(wv, src, 8 * tstride, NQ, (uint32_t)m, g.err)) {
#pragma unroll
            for (int qq = 0; qq < NQ; ++qq)
                sh.a_lds[buf][w + 4 * qq][lane] =
                    expand_signs_fast((uint32_t)wv[qq], 0x88888888u, 0x22222222u);
        } else {
            sh.abort = 1;
            __hip_atomic_fetch_or(g.status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (sh.abort) return false;
        if (pend) {  // the sample of the previous step: all its partials are in
            consider(team_energy(sp ^ 1));
            pend = false;
        }
        v16f acc;
        __builtin_amdgcn_s_setprio(0);
        constexpr int kPre = 2;
        v4i af[kPre];
#pragma unroll
        for (int qq = 0; qq < kPre; ++qq) af[qq] = sh.a_lds[buf][qq][lane];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            const v4i a = af[kb % kPre];
            if (kb + kPre < NKB) af[kb % kPre] = sh.a_lds[buf][kb + kPre][lane];
            if (kb == 0)
                mfma_fp4_first(acc, jr[0], a, one);
            else
                mfma_fp4(acc, jr[kb], a, one);
        }
        mfma_drain(acc);
        __builtin_amdgcn_s_setprio(3);
        if (is_sample(m)) {
            float part = 0.0f;
            bool fin = true;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                part += sgnf(xs[v]) * acc[v];
                fin = fin && isfinite(xs[v]) && isfinite(ys[v]);
            }
            part += __shfl_xor(part, 32);
            if (half == 0) {
                uint32_t *dst = ept + ((size_t)sp * kQChunks + rb) * tstride + l32;
                if (xcd_local)
                    __hip_atomic_store(dst, __float_as_uint(part), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                else
                    __hip_atomic_store(dst, __float_as_uint(part), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            // the partial is in before the next published word (here, at the
            // sample step, rather than in a branch of every step between the
            // update and the publish, which would split their schedule)
            release_partial();
            if (!fin && live) {
                g.bad[team * 32 + l32] = 1;
                __hip_atomic_fetch_or(g.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            sh.wpend[w][lane] = cur_word();
            pend = true;
            sp ^= 1;
        }
        if (m == steps) break;
        if (m == next_mult) next_mult = g.interval <= steps - m ? m + g.interval : -1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            float x = xs[v], y = ys[v];
            sb_update_tied(acc[v], p, c0, g.dt, g.a0dt, gdt, x, y);
            xs[v] = x;
            ys[v] = y;
        }
        publish(m + 1);
    }
    // the last sample: one more round, so that every partial is in
    release_partial();
    publish(steps + 1);
    {
        const uint64_t *src =
            xbt + ((size_t)((steps + 1) & 1) * kQChunks + 2 * w + half) * tstride + l32;
        uint64_t wv[NQ];
        if (!gather_words<NQ>(wv, src, 8 * tstride, NQ, (uint32_t)(steps + 1), g.err)) {
            sh.abort = 1;
            __hip_atomic_fetch_or(g.status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (sh.abort) return false;
    }
    const double lastE = team_energy(sp ^ 1);
    consider(lastE);
    // outputs: spins of this wave's rows (best or final sample), and the
    // replica's energies from the first wave of the team
    if (live) {
        const uint32_t wsel = g.return_best ? sh.wbest[w][lane] : sh.wpend[w][lane];
        int8_t *out = tm.spins + (size_t)rep * N;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int t = 8 * (v >> 2) + 4 * half + (v & 3);
            const int row = rb * 32 + t;
            if (row < N) out[row] = ((wsel >> row_word_bit(t)) & 1u) ? -1 : 1;
        }
        if (rb == 0 && half == 0) {
            g.best_e[team * 32 + l32] = sh.beste[w][l32];
            g.last_e[team * 32 + l32] = lastE;
        }
    }
    return true;
}

// Grid: a multiple of 8 workgroups, all resident at once.  See the file
// comment for the scheme; the per-step body is that of the single-run kernel,
// compiled once per padded size (K blocks 4, 8, ..., 32) and chosen per team.
__global__ __launch_bounds__(256, 2) void k_dsb_fp4_queue(
    const QTeam *__restrict__ teams, const uint32_t *__restrict__ units,
    const int *__restrict__ qoff, int *head, uint64_t *mslot, const uint32_t *epoch_p,
    int local_ok, QArgs g) {
    __shared__ QShared sh;
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x & 7;
    const int qbeg = qoff[q], qlen = qoff[q + 1] - qbeg;
    const uint32_t epoch = __hip_atomic_load(epoch_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int my_xcc = xcc_id();
    // The first unit of workgroup j of a queue is entry j: block 8 j + q runs
    // part j % wpt of the queue's team j / wpt when all teams have wpt parts,
    // the placement of the single-run kernel (the two workgroups a CU holds,
    // blocks b and b + 256, then belong to different teams, out of step with
    // each other).  Later entries go to whichever workgroup is free first.
    int first = (int)(blockIdx.x >> 3);
    for (;;) {
        __syncthreads();  // nothing of the previous unit is read any more
        if (threadIdx.x == 0) {
            int u = -1, k = -1;
            if (__hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                k = first >= 0 ? first : atomicAdd(head + q, 1);
                if (k < qlen) u = (int)units[qbeg + k];
            }
            sh.unit = u;
            sh.entry = k;
            sh.abort = 0;
        }
        first = -1;
        __syncthreads();
        // wave-uniform values (scalar registers): the unit, the team record
        const int unit = __builtin_amdgcn_readfirstlane(sh.unit);
        if (unit < 0) return;
        const int team = unit >> 4, member = unit & 15;
        const QTeam tm = teams[team];
        const int nkb = __builtin_amdgcn_readfirstlane(tm.nkb);
        const int wpt = nkb >> 1;
        const int rb = member * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

        // Are all workgroups of the team on this XCD?  Each member records
        // (launch epoch, XCD id); lane k reads member k's record.  A member
        // may wait here for as long as other teams run: the team's last entry
        // is handed out only when a workgroup of the queue becomes free (the
        // first grid/8 entries are taken at the start, then one by one from
        // the counter).  So the time limit runs only once every entry of the
        // team has been handed out.
        const int entry = __builtin_amdgcn_readfirstlane(sh.entry);
        const int last_entry = entry - member + wpt - 1;
        const int nstatic = (int)(gridDim.x >> 3);
        auto all_taken = [&]() {
            return last_entry < nstatic ||
                   __hip_atomic_load(head + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > last_entry;
        };
        if (threadIdx.x == 0)
            st_tagged(mslot + (size_t)team * kMaxWpt + member,
                      ((uint64_t)epoch << 32) | (uint32_t)my_xcc);
        bool xcd_local;
        {
            const uint64_t *ms = mslot + (size_t)team * kMaxWpt + (lane < wpt ? lane : 0);
            uint64_t v = ld_tagged(ms);
            uint64_t t0 = wall_clock64();
            bool taken = all_taken();
            bool ok = true;
            while (__any((uint32_t)(v >> 32) != epoch)) {
                __builtin_amdgcn_s_sleep(1);
                v = ld_tagged(ms);
                if (!taken) {  // the clock starts when the last member is handed out
                    taken = all_taken();
                    t0 = wall_clock64();
                }
                if (wall_clock64() - t0 > kTimeoutTicks ||
                    __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = false;
                    break;
                }
            }
            if (!ok) {
                __hip_atomic_store(g.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or(g.status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;  // every other workgroup sees err and ends too
            }
            xcd_local = local_ok && __all((int)(uint32_t)v == my_xcc);
        }
        bool done = false;
        switch (nkb) {
        case 4: done = run_unit<4>(sh, tm, team, rb, xcd_local, g); break;
        case 8: done = run_unit<8>(sh, tm, team, rb, xcd_local, g); break;
        case 12: done = run_unit<12>(sh, tm, team, rb, xcd_local, g); break;
        case 16: done = run_unit<16>(sh, tm, team, rb, xcd_local, g); break;
        case 20: done = run_unit<20>(sh, tm, team, rb, xcd_local, g); break;
        case 24: done = run_unit<24>(sh, tm, team, rb, xcd_local, g); break;
        case 28: done = run_unit<28>(sh, tm, team, rb, xcd_local, g); break;
        default: done = run_unit<32>(sh, tm, team, rb, xcd_local, g); break;
        }
        (void)done;  // an ended run has set err: the next take ends the workgroup
    }
}

// energy of every job replica: eq. (1) of the returned spins, NaN for a
// replica whose state became non-finite.  One thread per team column.
__global__ void k_queue_energy(const QTeam *__restrict__ teams, int nteams,
                               const double *__restrict__ best_e, const double *__restrict__ last_e,
                               const int32_t *__restrict__ bad, int return_best) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nteams * 32) return;
    const QTeam tm = teams[c >> 5];
    const int l = c & 31;
    if (l >= tm.nrep) return;
    tm.energy[tm.rep0 + l] = bad[c] ? __builtin_nan("") : (return_best ? best_e[c] : last_e[c]);
}

namespace {

__global__ void k_q_fill_u64(uint64_t *p, size_t n, uint64_t v) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}
__global__ void k_q_fill_i32(int32_t *p, size_t n, int32_t v) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}
// next launch epoch: never 0xFFFFFFFF (the fill of unused records) nor 0
__global__ void k_q_next_epoch(uint32_t *epoch) {
    uint32_t e = epoch[0] + 1u;
    if (e == 0xFFFFFFFFu || e == 0u) e = 1u;
    epoch[0] = e;
}
// p_k = a0 - a(t_k), a(t_k) = a0 k / Ns, in the host table's single-precision
// operations and rounding
__global__ void k_q_ptab(float *ptab, int n, float a0, float Ns_f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ptab[i] = __fsub_rn(a0, __fdiv_rn(__fmul_rn(a0, (float)i), Ns_f));
}

}  // namespace

// ------------------------------------------------------------------- host

struct QueueWork {
    QTeam *teams = nullptr;
    size_t teams_n = 0;
    uint32_t *units = nullptr;
    size_t units_n = 0;
    int *qoff = nullptr;
    int *head = nullptr;
    uint64_t *xb = nullptr;      // [nteams][2][64][32] tagged sign words
    size_t xb_n = 0;
    uint32_t *ep = nullptr;      // [nteams][2][64][32] sample energy partials
    size_t ep_n = 0;
    uint64_t *mslot = nullptr;   // [nteams][16] member placement records
    size_t mslot_n = 0;
    float *ptab = nullptr;
    size_t ptab_n = 0;
    double *best_e = nullptr, *last_e = nullptr;
    int32_t *bad = nullptr;
    size_t cols_n = 0;
    int32_t *status = nullptr, *err = nullptr;
    uint32_t *epoch = nullptr;
    // what was last uploaded (a repeated batch queues no host copy)
    std::vector<QTeam> teams_up;
    std::vector<uint32_t> units_up;
    std::vector<int> qoff_up;
    uint64_t gen = 0;
};

namespace {

template <typename T>
int grow(T **p, size_t *cap, size_t n, QueueWork *w) {
    if (n <= *cap) return HSB_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess)
        return qerr(e == hipErrorOutOfMemory ? HSB_ENOMEM : HSB_EDEVICE, "batch queue buffers: %s",
                    hipGetErrorString(e));
    *cap = n;
    ++w->gen;
    return HSB_OK;
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// Estimated time of one step of a team, in cycles: the latency of the exchange
// round trip, expansion, update and publish, plus the products of its K blocks
// (measured on the single-run kernel; only the ratios matter).
double team_step_cost(int nkb) { return 2300.0 + 64.0 * nkb; }

}  // namespace

int queue_work_create(QueueWork **out) {
    *out = new (std::nothrow) QueueWork;
    return *out ? HSB_OK : qerr(HSB_ENOMEM, "batch queue: host allocation");
}

void queue_work_free(QueueWork *w) {
    if (!w) return;
    void *ptrs[] = {w->teams, w->units, w->qoff, w->head, w->xb, w->ep, w->mslot, w->ptab,
                    w->best_e, w->last_e, w->bad, w->status, w->err, w->epoch};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete w;
}

uint64_t queue_gen(const QueueWork *w) { return w->gen; }
const int32_t *queue_status(const QueueWork *w) { return w->status; }

double queue_schedule(const std::vector<QTeam> &teams, int policy, std::vector<uint32_t> &units,
                      std::vector<int> &qoff) {
    const int nt = (int)teams.size();
    std::vector<std::vector<int>> qs(8);
    std::vector<double> load(8, 0.0);
    if (policy == 1) {
        for (int t = 0; t < nt; ++t) {
            qs[t % 8].push_back(t);
            load[t % 8] += (teams[t].nkb / 2) * team_step_cost(teams[t].nkb);
        }
    } else {
        std::vector<int> order(nt);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return team_step_cost(teams[a].nkb) > team_step_cost(teams[b].nkb);
        });
        for (int t : order) {
            const int qmin = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            qs[qmin].push_back(t);
            load[qmin] += (teams[t].nkb / 2) * team_step_cost(teams[t].nkb);
        }
    }
    units.clear();
    qoff.assign(9, 0);
    for (int q = 0; q < 8; ++q) {
        qoff[q] = (int)units.size();
        for (int t : qs[q])
            for (int k = 0; k < teams[t].nkb / 2; ++k) units.push_back(((uint32_t)t << 4) | (uint32_t)k);
    }
    qoff[8] = (int)units.size();
    return *std::max_element(load.begin(), load.end());
}

int queue_run(QueueWork *w, const std::vector<QTeam> &teams, const QRun &run, int policy,
              hipStream_t s, KernelTimer &timer) {
    const size_t nt = teams.size();
    if (nt == 0) return HSB_OK;
    if (nt > (size_t)(1 << 27)) return qerr(HSB_EINVAL, "batch queue: too many teams");
    for (const QTeam &t : teams)
        if (t.nkb < 4 || t.nkb > kQKB || t.nkb % 4 != 0 || t.N > t.nkb * 64 || t.nrep < 1 ||
            t.nrep > 32)
            return qerr(HSB_EINVAL, "batch queue: invalid team (N %d, %d K blocks)", t.N, t.nkb);
    int dev = 0, ncu = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_dsb_fp4_queue), 256, 0);
    if (e != hipSuccess) return qerr(HSB_EDEVICE, "batch queue: %s", hipGetErrorString(e));
    const int grid = 8 * ((nb * ncu) / 8);
    if (grid / 8 < kMaxWpt)
        return qerr(HSB_EUNSUPPORTED, "batch queue: %d resident workgroups per queue < %d", grid / 8,
                    kMaxWpt);
    std::vector<uint32_t> units;
    std::vector<int> qoff;
    queue_schedule(teams, policy, units, qoff);

    int rc = grow(&w->teams, &w->teams_n, nt, w);
    if (!rc) rc = grow(&w->units, &w->units_n, units.size(), w);
    size_t nine = w->qoff ? 9 : 0, eight = w->head ? 8 : 0;
    if (!rc) rc = grow(&w->qoff, &nine, 9, w);
    if (!rc) rc = grow(&w->head, &eight, 8, w);
    if (!rc) rc = grow(&w->xb, &w->xb_n, nt * kTeamWords, w);
    if (!rc) rc = grow(&w->ep, &w->ep_n, nt * kTeamWords, w);
    if (!rc) rc = grow(&w->mslot, &w->mslot_n, nt * kMaxWpt, w);
    if (!rc) rc = grow(&w->ptab, &w->ptab_n, (size_t)std::max(run.steps, 1), w);
    if (!rc && w->cols_n < nt * 32) {
        size_t c1 = w->cols_n, c2 = w->cols_n, c3 = w->cols_n;
        rc = grow(&w->best_e, &c1, nt * 32, w);
        if (!rc) rc = grow(&w->last_e, &c2, nt * 32, w);
        if (!rc) rc = grow(&w->bad, &c3, nt * 32, w);
        if (!rc) w->cols_n = nt * 32;
    }
    if (!rc && !w->status) {
        size_t one = 0, one2 = 0, one3 = 0;
        rc = grow(&w->status, &one, 1, w);
        if (!rc) rc = grow(&w->err, &one2, 1, w);
        if (!rc) rc = grow(&w->epoch, &one3, 1, w);
        if (!rc) {
            hipLaunchKernelGGL(k_q_fill_i32, dim3(1), dim3(1), 0, s, (int32_t *)w->epoch, (size_t)1, 0);
            if (hipGetLastError() != hipSuccess) rc = qerr(HSB_EDEVICE, "epoch fill failed");
        }
    }
    if (rc) return rc;
    // the tables, uploaded only when they differ from the last upload
    const bool same = w->teams_up.size() == nt && w->units_up == units && w->qoff_up == qoff &&
                      std::memcmp(w->teams_up.data(), teams.data(), nt * sizeof(QTeam)) == 0;
    if (!same) {
        e = hipMemcpyAsync(w->teams, teams.data(), nt * sizeof(QTeam), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w->units, units.data(), units.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w->qoff, qoff.data(), 9 * sizeof(int), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors go away on return
        if (e != hipSuccess) return qerr(HSB_EDEVICE, "batch queue tables: %s", hipGetErrorString(e));
        w->teams_up = teams;
        w->units_up = units;
        w->qoff_up = qoff;
        ++w->gen;
    }
    // per launch: empty queues' counters, no stale word of an earlier launch,
    // the epoch, the flags, the pump table
    const size_t nxb = nt * kTeamWords;
    hipLaunchKernelGGL(k_q_fill_u64, dim3(cdiv(nxb, 256)), dim3(256), 0, s, w->xb, nxb,
                       (uint64_t)kNoTag << 32);
    // the queues' counters start past the entries taken statically (one per workgroup)
    hipLaunchKernelGGL(k_q_fill_i32, dim3(1), dim3(64), 0, s, (int32_t *)w->head, (size_t)8,
                       grid / 8);
    hipLaunchKernelGGL(k_q_fill_i32, dim3(cdiv(nt * 32, 256)), dim3(256), 0, s, w->bad, nt * 32, 0);
    hipLaunchKernelGGL(k_q_fill_i32, dim3(1), dim3(64), 0, s, w->status, (size_t)1, 0);
    hipLaunchKernelGGL(k_q_fill_i32, dim3(1), dim3(64), 0, s, w->err, (size_t)1, 0);
    hipLaunchKernelGGL(k_q_next_epoch, dim3(1), dim3(1), 0, s, w->epoch);
    if (run.steps > 0)
        hipLaunchKernelGGL(k_q_ptab, dim3(cdiv(run.steps, 256)), dim3(256), 0, s, w->ptab,
                           run.steps, run.a0, (float)run.steps);
    e = hipGetLastError();
    if (e != hipSuccess) return qerr(HSB_EDEVICE, "batch queue set-up: %s", hipGetErrorString(e));
    const float a0dt = run.a0 * run.dt;
    e = timer.begin(s);
    if (e == hipSuccess) {
        QArgs g;
        g.xb = w->xb;
        g.ep = w->ep;
        g.ptab = w->ptab;
        g.best_e = w->best_e;
        g.last_e = w->last_e;
        g.bad = w->bad;
        g.status = w->status;
        g.err = w->err;
        g.steps = run.steps;
        g.interval = run.interval;
        g.return_best = run.return_best;
        g.nteams = (int)nt;
        g.dt = run.dt;
        g.a0dt = a0dt;
        g.amp = run.amp;
        hipLaunchKernelGGL(k_dsb_fp4_queue, dim3((unsigned)grid), dim3(256), 0, s, w->teams,
                           w->units, w->qoff, w->head, w->mslot, w->epoch,
                           run.local_exchange ? 1 : 0, g);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = timer.end(s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_queue_energy, dim3(cdiv(nt * 32, 256)), dim3(256), 0, s, w->teams,
                           (int)nt, w->best_e, w->last_e, w->bad, run.return_best);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return qerr(HSB_EDEVICE, "batch queue launch: %s", hipGetErrorString(e));
    return HSB_OK;
}

}  // namespace hsb
