// Integer-digit field plan: the field of eqs. (4)/(5) as an exact integer
// product on the int8 matrix cores with the update of eqs. (16)-(22) fused
// into its epilogue: one persistent launch per segment of steps between two
// sample points (k_i8_persist), or one launch per step (k_i8_field).
//
// Digits (see digits.h): x -> four balanced base-256 digits of rint(x 2^30),
// sgn(x) -> one digit, J -> one digit (integer J) or four digits of a per-row
// power-of-two scaled rint(J_ij / s_i 2^30).  Digit pairs (a, b) with
// a + b <= 3 are multiplied; each weight w = a + b has its own int32
// accumulator (exact), and the weights are combined exactly in FP64:
//   T = sum_w 2^(8 (NW-1-w)) U_w,   f = fl32(T * rowscale_i * xscale).
//
// Layouts (16-spin K blocks, 16 bytes per record):
//   J digits  jd[a][Npad/16][Npad][16]   record (kb, row) = J[row][16 kb .. 16 kb + 15]
//   x digits  xd[b][Npad/16][Rpad][16]   record (kb, r)   = digit b of x[16 kb ..][r]
// so every MFMA operand fragment (16 consecutive K of one row or one replica)
// is one 16-byte load, and 32 lanes read 512 contiguous bytes.
//
// Work decomposition of one step: a workgroup (4 waves) computes the field of
// 256 spins x 32 replicas; wave w owns spins [64 w, 64 w + 64) of the tile as
// two 32 x 32 MFMA tiles.  The x digits of the 32 replicas are shared by the
// four waves and staged through LDS (double-buffered, one barrier per stage);
// each wave streams its own J rows from L2 straight into registers, one stage
// ahead.  v_mfma_i32_32x32x32_i8 operand layout (lane l, half h = l / 32):
//   A: A[l % 32][16 h .. 16 h + 15]   B: B[16 h .. 16 h + 15][l % 32]
//   D: item v of lane l is D[8 (v / 4) + 4 h + v % 4][l % 32]
#include "digits.h"
#include "hsb.h"
#include "hsb_device.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

namespace hsb {

typedef int v16i __attribute__((ext_vector_type(16)));

struct I8J {
    int N = 0, Npad = 0, njd = 1;
    v4i *jd = nullptr;           // [njd][Npad/16][Npad] records
    double *rowscale = nullptr;  // [Npad]: 1 (one digit) or s_i 2^-30
    int8_t *xd = nullptr;        // [2][4][Npad/16][Rpad][16] digit ping-pong
    size_t xd_bytes = 0;
    int8_t *sd = nullptr;        // [Npad/16][Rpad][16] sign digits of sampled states
    size_t sd_bytes = 0;
    // persistent kernel: placement slots and step flags, p_k of a segment, error word
    uint32_t *sync = nullptr;
    size_t sync_n = 0;
    float *ptab = nullptr;
    size_t ptab_n = 0;
    int32_t *err = nullptr;
    size_t err_n = 0;
};

namespace {
thread_local char d_err[256] = "";
int derr(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(d_err, sizeof(d_err), fmt, ap);
    va_end(ap);
    return code;
}
constexpr int kMaxN = 16384;  // int32 digit sums stay below 2^31 for four-digit J
}  // namespace

const char *i8_error() { return d_err; }
bool i8_exact(const I8J *p) { return p->njd == 1; }
int i8_max_n() { return kMaxN; }

// ----------------------------------------------------------------- device

// Balanced base-256 digits of |q| <= 2^30: d3, d2, d1 in [-128, 127], d0 in [-64, 64].
__device__ __forceinline__ void split4(int q, int (&d)[4]) {
#pragma unroll
    for (int b = 3; b > 0; --b) {
        const int lo = (int)(int8_t)(q & 0xFF);
        d[b] = lo;
        q = (q - lo) >> 8;
    }
    d[0] = q;
}

__device__ __forceinline__ int x_fixed(float x) { return (int)rintf(x * 0x1p30f); }

// Digits of the state X ([Nst][Rpad] FP32) into `nsets` consecutive digit
// buffers.  Grid (Rpad / 64, Npad / 16), 64 threads: thread = replica.
template <int NXD>
__global__ __launch_bounds__(64) void k_i8_digits(const float *__restrict__ X,
                                                  int8_t *__restrict__ xd, int Nst, int Npad,
                                                  int Rpad, int nsets,
                                                  const int32_t *__restrict__ stop) {
    if (stop && stop[0] >= 0) return;  // a cancelled run: no more samples
    const int r = blockIdx.x * 64 + threadIdx.x;
    const int kb = blockIdx.y, nkb = Npad / 16;
    uint32_t w[NXD][4];
#pragma unroll
    for (int b = 0; b < NXD; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[b][q] = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = kb * 16 + e;
        if (i < Nst) {
            const float x = X[(size_t)i * Rpad + r];
            if (NXD == 1) {
                w[0][e >> 2] |= (uint32_t)(uint8_t)(x >= 0.0f ? 1 : -1) << (8 * (e & 3));
            } else {
                int d[4];
                split4(x_fixed(x), d);
#pragma unroll
                for (int b = 0; b < NXD; ++b)
                    w[b][e >> 2] |= (uint32_t)(uint8_t)d[b] << (8 * (e & 3));
            }
        }
    }
    const size_t set = (size_t)NXD * nkb * Rpad;
    for (int s = 0; s < nsets; ++s)
#pragma unroll
        for (int b = 0; b < NXD; ++b) {
            v4i rec = {(int)w[b][0], (int)w[b][1], (int)w[b][2], (int)w[b][3]};
            reinterpret_cast<v4i *>(xd)[s * set + ((size_t)b * nkb + kb) * Rpad + r] = rec;
        }
}

// One time step (ENERGY = false) or the energy partials of the current state
// (ENERGY = true, sign digits, one-digit J).  Grid (Npad / (128 NT), Rpad / 32).
template <int NJD, int NXD, int KC, bool ENERGY, bool NH, int NT>
__global__ __launch_bounds__(256, NT == 1 ? 2 : 1) void k_i8_field(
    const v4i *__restrict__ jd, const double *__restrict__ rowscale, const v4i *__restrict__ xin,
    int8_t *__restrict__ xout, float *__restrict__ X, float *__restrict__ Y,
    const float *__restrict__ gam, double *__restrict__ epart, int Nst, int Npad, int Rpad,
    float p, float c0, float dt, float a0dt, NHFused nhf, const int32_t *__restrict__ stop) {
    constexpr int NW = (NJD + NXD - 1) < 4 ? (NJD + NXD - 1) : 4;  // accumulated weights
    constexpr int KB = 2 * KC;                                       // K blocks per stage
    constexpr int BTOT = NXD * KB * 32;                              // B records per stage
    constexpr int BPT = (BTOT + 255) / 256;                          // per thread
    // x digits are 2^-30 units, sign digits units; truncating weights > 3 of a
    // four-digit J shifts the combined sum by 2^24
    constexpr double kXs = NXD == 4 ? 0x1p-30 : 1.0;
    constexpr double kTrunc = (NJD + NXD - 1 - NW) == 3 ? 0x1p24 : 1.0;
    __shared__ v4i bs[2][NXD][KB][32];
    // a run stopped by a cancel request: every later step and sample returns
    if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5, l32 = lane & 31;
    // XCD-aware tile order: block L runs on XCD L % 8; each XCD takes a
    // contiguous range of tiles in replica-major order, so the x digits of its
    // replicas stay in its L2 across the spin blocks
    const int gx = gridDim.x, T = gx * gridDim.y;
    const int L = blockIdx.x + gx * blockIdx.y;
    const int tile = (T & 7) == 0 ? (L & 7) * (T >> 3) + (L >> 3) : L;
    const int sb = tile % gx, rb = tile / gx;
    // NT 32-row tiles per wave: 64 rows (one wave per SIMD) or 32 rows (two)
    const int i0 = sb * (128 * NT) + w * (32 * NT), r0 = rb * 32;
    const int nkb = Npad / 16;
    const int S = Npad / (32 * KC);  // stages (even: Npad is a multiple of 256)
    // thermostat: xi(t_k) of this lane's replica, formed before the products so
    // that its loads overlap them.  The eight half-waves of the workgroup (all
    // on the same 32 replicas) each add every eighth partial; the eight sums
    // are then added in a fixed order (no wave has left the kernel yet, so
    // the barrier is reached by all).
    double xi_k = 0.0;
    if constexpr (NH) {
        __shared__ double s_part[8][32];
        const int rr = r0 + l32, grp = 2 * w + h;
        xi_k = nhf.xi_in[rr];
        if (!nhf.first) {
            double Ssum = 0.0;
            for (int q = grp; q < nhf.nparts; q += 8) Ssum += nhf.part_in[(size_t)q * Rpad + rr];
            s_part[grp][l32] = Ssum;
            __syncthreads();
            double S8 = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) S8 += s_part[q][l32];
            xi_k = xi_k + nhf.c * (S8 - nhf.NT);
        }
    }
    v16i acc[NT][NW];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int q = 0; q < NW; ++q) acc[tt][q] = v16i{};

    v4i a0r[NT][NJD][KC], a1r[NT][NJD][KC];
    v4i breg[BPT];

    auto loadA = [&](int s, v4i(&dst)[NT][NJD][KC]) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int a = 0; a < NJD; ++a)
#pragma unroll
                for (int c = 0; c < KC; ++c)
                    dst[tt][a][c] =
                        jd[((size_t)a * nkb + s * KB + 2 * c + h) * Npad + i0 + tt * 32 + l32];
    };
    auto loadB = [&](int s) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int e = t + 256 * q;
            if (BTOT % 256 == 0 || e < BTOT) {
                const int b = e / (KB * 32), kb = (e / 32) % KB, r = e % 32;
                breg[q] = xin[((size_t)b * nkb + s * KB + kb) * Rpad + r0 + r];
            }
        }
    };
    auto storeB = [&](int buf) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int e = t + 256 * q;
            if (BTOT % 256 == 0 || e < BTOT) {
                const int b = e / (KB * 32), kb = (e / 32) % KB, r = e % 32;
                bs[buf][b][kb][r] = breg[q];
            }
        }
    };
    auto compute = [&](int buf, const v4i(&A)[NT][NJD][KC]) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            v4i bf[NXD];
#pragma unroll
            for (int b = 0; b < NXD; ++b) bf[b] = bs[buf][b][2 * c + h][l32];
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                for (int a = 0; a < NJD; ++a)
#pragma unroll
                    for (int b = 0; b < NXD; ++b)
                        if (a + b < NW)
                            acc[tt][a + b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                A[tt][a][c], bf[b], acc[tt][a + b], 0, 0, 0);
        }
    };

    loadB(0);
    storeB(0);
    loadA(0, a0r);
    __syncthreads();
    for (int s = 0; s < S; s += 2) {
        // stage s: operands in a0r / LDS buffer 0; prefetch stage s + 1
        loadA(s + 1, a1r);
        loadB(s + 1);
        compute(0, a0r);
        storeB(1);
        __syncthreads();
        // stage s + 1: a1r / buffer 1; prefetch stage s + 2
        const bool more = s + 2 < S;
        if (more) {
            loadA(s + 2, a0r);
            loadB(s + 2);
        }
        compute(1, a1r);
        if (more) storeB(0);
        __syncthreads();
    }

    const int r = r0 + l32;
    static_assert(NT == 2 || !ENERGY, "energy partials are per 64 rows");
    if (ENERGY) {
        // eq. (1): partial sum_i s_i f_i over this wave's 64 spins, exact in int32
        int part = 0;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
            const int ib = i0 + tt * 32;
            if (ib >= Nst) continue;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = ib + 8 * (v >> 2) + 4 * h + (v & 3);
                const int f = acc[tt][0][v];
                part += X[(size_t)i * Rpad + r] >= 0.0f ? f : -f;
            }
        }
        part += __shfl_xor(part, 32);
        if (h == 0 && i0 < Nst) epart[(size_t)(i0 / 64) * Rpad + r] = (double)part;
        return;
    }

    // every load of the tile's state is issued before the first store, so the
    // 64 loads per lane overlap instead of each waiting behind a store
    if (i0 >= Nst) return;  // Nst is a multiple of 64: a wave's rows are wholly in or out
    float gdt;
    if constexpr (NH) {
        gdt = (float)(-xi_k) * dt;  // the rate -xi(t_k) in eq. (22)'s place
        if (i0 == 0 && h == 0) nhf.xi_out[r] = xi_k;
    } else {
        gdt = gam[r] * dt;
    }
    float xs[NT][16], ys[NT][16];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const size_t idx = (size_t)(i0 + tt * 32 + 8 * (v >> 2) + 4 * h + (v & 3)) * Rpad + r;
            xs[tt][v] = X[idx];
            ys[tt][v] = Y[idx];
        }
    if constexpr (NH) {  // sum of y_i(t_k)^2 over this wave's rows (exact squares)
        double t2 = 0.0;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int v = 0; v < 16; ++v) t2 += (double)ys[tt][v] * (double)ys[tt][v];
        t2 += __shfl_xor(t2, 32);
        if (h == 0) nhf.part_out[(size_t)(i0 / (32 * NT)) * Rpad + r] = t2;
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
        const int ib = i0 + tt * 32;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uint32_t dw[NXD];
#pragma unroll
            for (int b = 0; b < NXD; ++b) dw[b] = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = 4 * m + u;
                const int i = ib + 8 * m + 4 * h + u;
                double Tsum = (double)acc[tt][0][v];
#pragma unroll
                for (int q = 1; q < NW; ++q) Tsum = Tsum * 256.0 + (double)acc[tt][q][v];
                const double sc = (NJD == 1 ? 1.0 : rowscale[i]) * (kXs * kTrunc);
                const float f = (float)(Tsum * sc);
                float &x = xs[tt][v], &y = ys[tt][v];
                sb_update(f, p, c0, dt, a0dt, gdt, x, y);
                if (NXD == 1) {
                    dw[0] |= (uint32_t)(uint8_t)(x >= 0.0f ? 1 : -1) << (8 * u);
                } else {
                    int d[4];
                    split4(x_fixed(x), d);
#pragma unroll
                    for (int b = 0; b < NXD; ++b) dw[b] |= (uint32_t)(uint8_t)d[b] << (8 * u);
                }
            }
            const int ig = ib + 8 * m + 4 * h;  // first of the 4 consecutive spins
#pragma unroll
            for (int b = 0; b < NXD; ++b)
                *reinterpret_cast<uint32_t *>(
                    xout + (((size_t)b * nkb + (ig >> 4)) * Rpad + r) * 16 + (ig & 15)) = dw[b];
        }
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const size_t idx = (size_t)(i0 + tt * 32 + 8 * (v >> 2) + 4 * h + (v & 3)) * Rpad + r;
            X[idx] = xs[tt][v];
            Y[idx] = ys[tt][v];
        }
}

// ------------------------------------------------------- persistent step kernel
//
// The same step as k_i8_field (the thermostat included) for a whole segment
// of steps between two sample points in one launch.  A team of workgroups
// owns one 32-replica block: workgroup k of the team computes spins
// [128 NT k, 128 NT (k + 1)) of those replicas, as in k_i8_field, and keeps
// its part of x and y in LDS for the whole segment (the products need the
// registers).  The x digits of each step go
// through the ping-pong digit buffers (the layout k_i8_field reads), and each
// wave sets its step flag once its digits are stored; before a step's
// products every wave waits for the flags of its team.  The digits of step m
// + 1 overwrite those of step m - 1: their writer has seen every flag of
// step m, set only after the step-(m - 1) products that read them.
//   The team's workgroups are placed on one XCD (block b runs on XCD b % 8;
// team t takes blocks 8 (wpt floor(t / 8) + k) + t % 8), and at start-up
// each one records its XCD id and reads its teammates'.  When they share an
// XCD the digits and flags only have to reach its L2: stores are waited for
// (vmcnt) before the flag, and the readers' loads bypass the L1 (device
// scope).  Otherwise a device-scope release and acquire order them.  Every
// wait is bounded (4 s); a timeout sets the run's error word and bit 1 of its
// status, and every wave then leaves.  The host launches at most as many
// workgroups as are resident at once and clears the flags and the placement
// slots before every launch.

constexpr uint64_t kI8TimeoutTicks = 400000000ull;  // 4 s of the 100 MHz wall clock
constexpr uint32_t kI8NoFlag = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t i8_flag_ld(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int i8_xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20); }

// 16 bytes per lane from global memory (wave-uniform base plus the lane's
// 32-bit byte offset) straight into LDS at lds_base + 16 lane, device scope
// (the L1 is bypassed).  Assembly, so that the compiler does not track it:
// the caller waits for it (vmcnt, counting the loads it issued after it) and
// synchronises the workgroup before any wave reads the bytes; the compiler's
// own vmcnt waits for its tracked loads only get stricter from it.
__device__ __forceinline__ void i8_lds_direct16(const void *base, uint32_t lane_off,
                                                uint32_t lds_base) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1 sc1"
                 :
                 : "v"(lane_off), "s"(base), "s"(lds_base)
                 : "memory", "m0");
}

// The thermostat (eqs. (6)-(8)) in the persistent kernel, in the per-step
// kernel's slots: step j = k - k0 of the run reads xi(t_{k-1}) from slot j & 1
// and the per-wave partials of sum_i y_i(t_{k-1})^2 from partial set
// (j + 1) & 1, and writes the partials of y(t_k) to set j & 1.  Within a
// segment the partials travel with the x digits (stored before the step
// flag); at its end xi of its last step goes to slot (j + 1) & 1, so a later
// segment, or the final xi, finds what the per-step kernel would have left.
struct I8NH {
    double *xi = nullptr;    // [2][Rpad]
    double *part = nullptr;  // [2][nparts][Rpad]
    int nparts = 0, k0 = 0;  // per-wave partials of the state rows; the run's first step
    double c = 0.0, NT = 0.0;
};

template <int NJD, int NXD, int KC, int NT, bool NH>
__global__ __launch_bounds__(256, NT == 1 ? 2 : 1) void k_i8_persist(
    const v4i *__restrict__ jd, const double *__restrict__ rowscale, int8_t *xd,
    uint32_t *sync, float *__restrict__ X, float *__restrict__ Y, const float *__restrict__ gam,
    const float *__restrict__ ptab, int32_t *__restrict__ status, int32_t *err,
    const int32_t *__restrict__ stop, int local_ok, int Nst, int Npad, int Rpad, int team0,
    int nteams, int k0, int k1, float c0, float dt, float a0dt, I8NH nh) {
    constexpr int NW = (NJD + NXD - 1) < 4 ? (NJD + NXD - 1) : 4;
    constexpr int KB = 2 * KC;
    constexpr int BTOT = NXD * KB * 32;
    constexpr int BPT = (BTOT + 255) / 256;
    constexpr double kXs = NXD == 4 ? 0x1p-30 : 1.0;
    constexpr double kTrunc = (NJD + NXD - 1 - NW) == 3 ? 0x1p24 : 1.0;
    static_assert(BTOT % 64 == 0 && KB % 2 == 0, "a wave stages whole pairs of K blocks");
    __shared__ v4i bs[2][NXD][KB][32];
    // thermostat: the eight half-waves' sums of the team's partials
    __shared__ double s_part[NH ? 8 : 1][32];
    // the workgroup's x and y between steps (item v of thread t at [v][t]):
    // in LDS rather than registers, which the products need
    __shared__ float s_x[NT * 16][256], s_y[NT * 16][256];
    __shared__ int wg_abort;
    // a run stopped by a cancel request at an earlier sample point
    if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5, l32 = lane & 31;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int wpt = Npad / (128 * NT);  // workgroups of a team
    const int nwt = 4 * wpt;            // waves of a team (<= 256)
    const int xcd = blockIdx.x & 7, kx = blockIdx.x >> 3;
    const int tl = (kx / wpt) * 8 + xcd;
    if (tl >= nteams) return;  // whole workgroup
    const int team = team0 + tl;
    const int sbk = kx % wpt;
    const int i0 = sbk * (128 * NT) + w * (32 * NT), r0 = team * 32;
    const int r = r0 + l32;
    const int nkb = Npad / 16;
    const int S = Npad / (32 * KC);
    uint32_t *slots = sync;                                 // [gridDim.x]
    uint32_t *flags = sync + gridDim.x + (size_t)tl * nwt;  // this team's
    uint32_t *myflag = flags + sbk * 4 + wu;
    const size_t set = (size_t)NXD * nkb * Rpad * 16;  // bytes of one digit set
    if (t == 0) wg_abort = 0;

    // do all workgroups of this team share one XCD?
    const int my_xcc = i8_xcc_id();
    if (t == 0) __hip_atomic_store(slots + blockIdx.x, (uint32_t)my_xcc, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    bool xcd_local;
    {
        const int mb = 8 * (wpt * (tl >> 3) + (lane < wpt ? lane : 0)) + (tl & 7);
        uint32_t v = i8_flag_ld(slots + mb);
        const uint64_t ts = wall_clock64();
        bool ok = true;
        while (__any(v == kI8NoFlag)) {
            __builtin_amdgcn_s_sleep(1);
            v = i8_flag_ld(slots + mb);
            if (wall_clock64() - ts > kI8TimeoutTicks) {
                ok = false;
                break;
            }
        }
        xcd_local = local_ok && ok && __all(v == (uint32_t)my_xcc);
    }

    const bool live = i0 < Nst;  // Nst is a multiple of 64: a wave's rows are wholly in or out
    auto row_of = [&](int tt, int v) { return i0 + tt * 32 + 8 * (v >> 2) + 4 * h + (v & 3); };
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const size_t idx = (size_t)row_of(tt, v) * Rpad + r;
            s_x[tt * 16 + v][t] = live ? X[idx] : 0.0f;
            s_y[tt * 16 + v][t] = live ? Y[idx] : 0.0f;
        }
    const float gdt_heat = gam[r] * dt;
    double xi_m = 0.0;  // thermostat: xi(t_m) of this lane's replica

    // digits of four consecutive spins (items 4q .. 4q + 3 of tile tt) of x_m
    // into set m & 1
    auto put_digits = [&](int m, int tt, int q, const float (&x4)[4]) {
        int8_t *xo = xd + (size_t)(m & 1) * set;
        uint32_t dw[NXD];
#pragma unroll
        for (int b = 0; b < NXD; ++b) dw[b] = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (NXD == 1) {
                dw[0] |= (uint32_t)(uint8_t)(x4[u] >= 0.0f ? 1 : -1) << (8 * u);
            } else {
                int d[4];
                split4(x_fixed(x4[u]), d);
#pragma unroll
                for (int b = 0; b < NXD; ++b) dw[b] |= (uint32_t)(uint8_t)d[b] << (8 * u);
            }
        }
        const int ig = i0 + tt * 32 + 8 * q + 4 * h;
#pragma unroll
        for (int b = 0; b < NXD; ++b)
            *reinterpret_cast<uint32_t *>(
                xo + (((size_t)b * nkb + (ig >> 4)) * Rpad + r) * 16 + (ig & 15)) = dw[b];
    };
    // this wave's digits of x_m are stored: its flag
    auto set_flag = [&](int m) {
        if (xcd_local) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (lane == 0)
                __hip_atomic_store(myflag, (uint32_t)m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_store(myflag, (uint32_t)m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    // every wave of the team has published x_m (its flag is m, or already m + 1)
    auto wait_team = [&](int m) -> bool {
        uint32_t f[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            f[j] = lane + 64 * j < nwt ? i8_flag_ld(flags + lane + 64 * j) : (uint32_t)m;
        const uint64_t ts = wall_clock64();
        for (int it = 1;; ++it) {
            bool stale = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) stale = stale || (f[j] - (uint32_t)m) > 1u;
            if (!__any(stale)) break;
            if ((it & 31) == 0 &&
                (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                 wall_clock64() - ts > kI8TimeoutTicks)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or(status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (lane + 64 * j < nwt) f[j] = i8_flag_ld(flags + lane + 64 * j);
        }
        if (!xcd_local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        return true;
    };

    v16i acc[NT][NW];
    v4i a0r[NT][NJD][KC], a1r[NT][NJD][KC];
    auto loadA = [&](int s, v4i(&dst)[NT][NJD][KC]) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int a = 0; a < NJD; ++a)
#pragma unroll
                for (int c = 0; c < KC; ++c)
                    dst[tt][a][c] =
                        jd[((size_t)a * nkb + s * KB + 2 * c + h) * Npad + i0 + tt * 32 + l32];
    };
    // stage s of the x digits of the current set into LDS buffer buf: records
    // e = 256 q + 64 w + lane (digit b, K block kb of the stage, replica e % 32)
    auto stageB = [&](const int8_t *xin, int s, int buf) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int e0 = 256 * q + 64 * wu;
            if (BTOT % 256 == 0 || e0 < BTOT) {
                const int b = e0 / (KB * 32), kb = (e0 / 32) % KB;  // lanes 32-63: kb + 1
                const int8_t *base = xin + (((size_t)b * nkb + s * KB + kb) * Rpad + r0) * 16;
                const uint32_t off = (uint32_t)h * (uint32_t)Rpad * 16u + (uint32_t)l32 * 16u;
                i8_lds_direct16(base, off,
                                (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void *)&bs[buf][b][kb][0]);
            }
        }
    };
    auto compute = [&](int buf, const v4i(&A)[NT][NJD][KC]) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            v4i bf[NXD];
#pragma unroll
            for (int b = 0; b < NXD; ++b) bf[b] = bs[buf][b][2 * c + h][l32];
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                for (int a = 0; a < NJD; ++a)
#pragma unroll
                    for (int b = 0; b < NXD; ++b)
                        if (a + b < NW)
                            acc[tt][a + b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                A[tt][a][c], bf[b], acc[tt][a + b], 0, 0, 0);
        }
    };

    // the digits of the segment's first state
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float x4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x4[u] = s_x[tt * 16 + 4 * q + u][t];
            put_digits(k0, tt, q, x4);
        }
    set_flag(k0);
    for (int m = k0; m < k1; ++m) {
        const float p = ptab[m - k0];
        const int8_t *xin = xd + (size_t)(m & 1) * set;
        const int j = m - nh.k0;  // thermostat: step of the run
        if (!wait_team(m)) wg_abort = 1;
        if constexpr (NH) {
            // xi(t_m) = xi(t_{m-1}) + c (sum_i y_i(t_{m-1})^2 - N T), the partials
            // added as the per-step kernel adds them: half-wave g of the
            // workgroup takes partials g, g + 8, ..., then the eight sums in order
            if (m == k0) xi_m = nh.xi[(size_t)(j & 1) * Rpad + r];
            if (j > 0) {
                const uint64_t *pin = reinterpret_cast<const uint64_t *>(
                    nh.part + (size_t)((j + 1) & 1) * nh.nparts * Rpad);
                double Ssum = 0.0;
                for (int q = 2 * w + h; q < nh.nparts; q += 8)
                    Ssum += __longlong_as_double((long long)__hip_atomic_load(
                        pin + (size_t)q * Rpad + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                s_part[2 * w + h][l32] = Ssum;
            }
        }
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int q = 0; q < NW; ++q) acc[tt][q] = v16i{};
        loadA(0, a0r);
        stageB(xin, 0, 0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();  // also publishes wg_abort and the thermostat's sums
        if (wg_abort) break;
        if constexpr (NH) {
            if (j > 0) {
                double S8 = 0.0;
#pragma unroll
                for (int g = 0; g < 8; ++g) S8 += s_part[g][l32];
                xi_m = xi_m + nh.c * (S8 - nh.NT);
            }
        }
        // EARLY: each stage's x digits are loaded before its J fragments, and
        // the barrier waits only for the digits (at most the NA J loads issued
        // after them may be outstanding): the J fragments, which only their
        // own wave reads, stay in flight across it (wait and barrier are one
        // asm statement, so that no memory access moves between them).
        // Measured at N = 2000, R = 1024: sign digits 10.5 -> 9.7 us per step,
        // four-digit J 52.9 -> 51.9; one-digit J with x digits 20.8 -> 21.6,
        // so that combination keeps the full wait.
        constexpr bool EARLY = !(NJD == 1 && NXD == 4);
        constexpr int NA = NT * NJD * KC;
        static_assert(NA <= 63, "vmcnt counts up to 63");
        auto stage_barrier = [&]() {
            if constexpr (EARLY) {
                asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(NA) : "memory");
            } else {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
            }
        };
        auto load_stage = [&](int s, int buf, v4i(&dst)[NT][NJD][KC]) {
            if constexpr (EARLY) {
                stageB(xin, s, buf);
                loadA(s, dst);
            } else {
                loadA(s, dst);
                stageB(xin, s, buf);
            }
        };
        for (int s = 0; s < S; s += 2) {
            load_stage(s + 1, 1, a1r);
            compute(0, a0r);
            stage_barrier();
            const bool more = s + 2 < S;
            if (more) load_stage(s + 2, 0, a0r);
            compute(1, a1r);
            if (more) stage_barrier();
        }
        // the field, exactly rounded once, the update (as k_i8_field) and the
        // digits of x_{m+1}
        const bool pub = m + 1 < k1;
        float gdt = gdt_heat;
        if constexpr (NH) gdt = (float)(-xi_m) * dt;  // the rate -xi(t_m) in eq. (22)'s place
        double t2 = 0.0;  // thermostat: this wave's sum of y_i(t_m)^2 (exact squares)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float x4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int v = 4 * q + u;
                    const int i = row_of(tt, v);
                    double Tsum = (double)acc[tt][0][v];
#pragma unroll
                    for (int k = 1; k < NW; ++k) Tsum = Tsum * 256.0 + (double)acc[tt][k][v];
                    const double sc = (NJD == 1 ? 1.0 : rowscale[i]) * (kXs * kTrunc);
                    const float f = (float)(Tsum * sc);
                    float x = s_x[tt * 16 + v][t], y = s_y[tt * 16 + v][t];
                    if constexpr (NH) t2 += (double)y * (double)y;
                    sb_update(f, p, c0, dt, a0dt, gdt, x, y);
                    s_x[tt * 16 + v][t] = x;
                    s_y[tt * 16 + v][t] = y;
                    x4[u] = x;
                }
                if (pub) put_digits(m + 1, tt, q, x4);
            }
        if constexpr (NH) {
            // the partial of y(t_m), before the flag that publishes x_{m+1}
            t2 += __shfl_xor(t2, 32);
            if (live && h == 0)
                nh.part[((size_t)(j & 1) * nh.nparts + i0 / (32 * NT)) * Rpad + r] = t2;
            if (m + 1 == k1 && i0 == 0 && h == 0) nh.xi[(size_t)((j + 1) & 1) * Rpad + r] = xi_m;
        }
        if (pub) set_flag(m + 1);
    }
    if (live) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const size_t idx = (size_t)row_of(tt, v) * Rpad + r;
                X[idx] = s_x[tt * 16 + v][t];
                Y[idx] = s_y[tt * 16 + v][t];
            }
    }
}

__global__ void k_i8_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// p_k = a0 - (a0 k) / Ns of the steps k0 .. k0 + n - 1, with the host loop's
// single-precision operations and rounding
__global__ void k_i8_ptab(float *ptab, int k0, int n, float a0, float Ns_f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ptab[i] = __fsub_rn(a0, __fdiv_rn(__fmul_rn(a0, (float)(k0 + i)), Ns_f));
}

// ------------------------------------------------------------------- host

namespace {

template <typename T>
int grow(T **p, size_t *cap, size_t n) {
    if (n <= *cap) return HSB_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess)
        return derr(e == hipErrorOutOfMemory ? HSB_ENOMEM : HSB_EDEVICE, "digit buffers: %s",
                    hipGetErrorString(e));
    *cap = n;
    return HSB_OK;
}

// host balanced base-256 digits of |q| <= 2^30
void split4_host(long long q, int d[4]) {
    for (int b = 3; b > 0; --b) {
        const int lo = (int)(int8_t)(uint8_t)(q & 0xFF);
        d[b] = lo;
        q = (q - lo) / 256;
    }
    d[0] = (int)q;
}

// 32-row tiles per wave of a step kernel: one (32-row waves, two per SIMD)
// for four-digit J and for sign digits, measured faster there; two for
// one-digit J with x digits, where the halved operand reuse cost as much as
// the second wave gained; two for the energy partials
constexpr int tiles_per_wave(int njd, int nxd, bool energy) {
    return energy ? 2 : ((njd == 4 || nxd == 1) ? 1 : 2);
}

template <int NJD, int NXD, int KC, bool ENERGY, bool NH = false,
          int NT = tiles_per_wave(NJD, NXD, ENERGY)>
hipError_t launch_field(const I8J *p, const int8_t *xin, int8_t *xout, StateBufs &b, int Nst,
                        int Rpad, float pk, float c0, float dt, float a0dt, hipStream_t s,
                        const NHFused &nhf = NHFused{}) {
    const dim3 grid(p->Npad / (128 * NT), Rpad / 32);
    hipLaunchKernelGGL((k_i8_field<NJD, NXD, KC, ENERGY, NH, NT>), grid, dim3(256), 0, s, p->jd,
                       p->rowscale, reinterpret_cast<const v4i *>(xin), xout, b.X, b.Y, b.gamma,
                       b.epart, Nst, p->Npad, Rpad, pk, c0, dt, a0dt, nhf, b.stop);
    return hipGetLastError();
}

// One step of the plan with nt 32-row tiles per wave (1: 32-row waves, two
// workgroups per CU; 2: 64-row waves, one): both give the same exact sums.
template <int NJD, int NXD, int KC, bool NH>
hipError_t launch_step(int nt, const I8J *p, const int8_t *xin, int8_t *xout, StateBufs &b,
                       int Nst, int Rpad, float pk, float c0, float dt, float a0dt, hipStream_t s,
                       const NHFused &nhf) {
    if (nt == 1)
        return launch_field<NJD, NXD, KC, false, NH, 1>(p, xin, xout, b, Nst, Rpad, pk, c0, dt, a0dt,
                                                        s, nhf);
    return launch_field<NJD, NXD, KC, false, NH, 2>(p, xin, xout, b, Nst, Rpad, pk, c0, dt, a0dt, s,
                                                    nhf);
}

// The persistent kernel of a digit combination, wave height and thermostat.
// Four-digit J with 64-row waves stages one K block pair at a time (KC = 1):
// two would not fit the registers.
template <int NJD, int NXD, int KC, bool NH>
const void *persist_fn(int nt) {
    constexpr int KC2 = NJD == 4 ? 1 : KC;
    return nt == 1 ? reinterpret_cast<const void *>(k_i8_persist<NJD, NXD, KC, 1, NH>)
                   : reinterpret_cast<const void *>(k_i8_persist<NJD, NXD, KC2, 2, NH>);
}

template <bool NH>
const void *persist_kernel_nh(int njd, int nxd, int nt) {
    if (njd == 1) return nxd == 4 ? persist_fn<1, 4, 4, NH>(nt) : persist_fn<1, 1, 4, NH>(nt);
    return nxd == 4 ? persist_fn<4, 4, 2, NH>(nt) : persist_fn<4, 1, 2, NH>(nt);
}

const void *persist_kernel(int njd, int nxd, int nt, bool nh) {
    return nh ? persist_kernel_nh<true>(njd, nxd, nt) : persist_kernel_nh<false>(njd, nxd, nt);
}

// Teams (32-replica blocks) per launch of the persistent kernel: a multiple of
// 8 that keeps every workgroup of the grid resident at once; 0 when the plan
// cannot run persistently (a team larger than one XCD's share of the chip).
int persist_teams_per_launch(const void *fn, int wpt) {
    if (wpt > 64) return 0;  // one lane per teammate in the placement check
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess)
        return 0;
    const int cap = ncu * per_cu;
    return 8 * (cap / (8 * wpt));
}

}  // namespace

int i8_tiles() { return 4; }

int i8_create(const float *hJ, int N, I8J **out) {
    *out = nullptr;
    if (N < 1 || N > kMaxN) return derr(HSB_EUNSUPPORTED, "digit plan: N must be <= %d", kMaxN);
    I8J *p = new (std::nothrow) I8J;
    if (!p) return derr(HSB_ENOMEM, "digit plan: host allocation");
    p->N = N;
    p->Npad = (N + kI8SpinTile - 1) / kI8SpinTile * kI8SpinTile;
    const int Np = p->Npad, nkb = Np / 16;
    bool exact = true;
    for (size_t e = 0; e < (size_t)N * N && exact; ++e) {
        const float v = hJ[e];
        exact = v == std::nearbyint(v) && std::fabs(v) <= 127.0f;
    }
    p->njd = exact ? 1 : 4;
    const size_t rec = (size_t)p->njd * nkb * Np;  // 16-byte records
    std::vector<int8_t> jd(rec * 16, 0);
    std::vector<double> rs(Np, 1.0);
    for (int i = 0; i < N; ++i) {
        double sc = 1.0;
        if (!exact) {
            double m = 0.0;
            for (int j = 0; j < N; ++j) m = std::fmax(m, std::fabs((double)hJ[(size_t)i * N + j]));
            int ex = 0;
            if (m > 0.0) (void)std::frexp(m, &ex);  // m < 2^ex
            sc = std::ldexp(1.0, ex);
            rs[i] = std::ldexp(sc, -30);
        }
        for (int j = 0; j < N; ++j) {
            const double v = hJ[(size_t)i * N + j];
            const size_t off = (((size_t)(j / 16)) * Np + i) * 16 + (j % 16);
            if (exact) {
                jd[off] = (int8_t)v;
            } else {
                int d[4];
                split4_host((long long)std::nearbyint(std::ldexp(v / sc, 30)), d);
                for (int a = 0; a < 4; ++a) jd[(size_t)a * nkb * Np * 16 + off] = (int8_t)d[a];
            }
        }
    }
    hipError_t e = hipMalloc((void **)&p->jd, rec * 16);
    if (e == hipSuccess) e = hipMalloc((void **)&p->rowscale, sizeof(double) * Np);
    if (e == hipSuccess) e = hipMemcpy(p->jd, jd.data(), rec * 16, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->rowscale, rs.data(), sizeof(double) * Np, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        i8_free(p);
        return derr(e == hipErrorOutOfMemory ? HSB_ENOMEM : HSB_EDEVICE, "digit J store: %s",
                    hipGetErrorString(e));
    }
    *out = p;
    return HSB_OK;
}

void i8_free(I8J *p) {
    if (!p) return;
    void *ptrs[] = {p->jd, p->rowscale, p->xd, p->sd, p->sync, p->ptab, p->err};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

int i8_run(I8J *p, const I8Run &run, StateBufs &b, const float *fp32J, hipStream_t s,
           KernelTimer &timer) {
    const int Np = p->Npad, nkb = Np / 16, Rpad = run.Rpad, Nst = run.Nst;
    const bool bsb = run.variant == HSB_BSB;
    const int nxd = bsb ? 4 : 1;
    int rc = grow(&p->xd, &p->xd_bytes, (size_t)2 * nxd * nkb * Rpad * 16);
    if (!rc) rc = grow(&p->sd, &p->sd_bytes, (size_t)nkb * Rpad * 16);
    if (rc) return rc;
    // the caller has checked the premise of the x digits: |x| <= 1 in the start state
    hipError_t e = hipSuccess;
    const dim3 dgrid(Rpad / 64, nkb);
    if (bsb)
        hipLaunchKernelGGL(k_i8_digits<4>, dgrid, dim3(64), 0, s, b.X, p->xd, Nst, Np, Rpad, 2,
                           (const int32_t *)nullptr);
    else
        hipLaunchKernelGGL(k_i8_digits<1>, dgrid, dim3(64), 0, s, b.X, p->xd, Nst, Np, Rpad, 2,
                           (const int32_t *)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return derr(HSB_EDEVICE, "%s", hipGetErrorString(e));

    const size_t set = (size_t)nxd * nkb * Rpad * 16;
    const float a0 = run.a0, c0 = run.c0, dt = run.dt, a0dt = a0 * dt;
    const int k0 = run.k0, k1 = run.k1, interval = run.interval;
    auto is_sample = [&](int m) { return m == k1 || (m > k0 && m % interval == 0); };
    auto sample = [&](int m) -> int {
        hipError_t ee;
        int nblk;
        if (p->njd == 1) {
            hipLaunchKernelGGL(k_i8_digits<1>, dgrid, dim3(64), 0, s, b.X, p->sd, Nst, Np, Rpad,
                               1, b.stop);
            ee = hipGetLastError();
            if (ee == hipSuccess)
                ee = launch_field<1, 1, 4, true>(p, p->sd, nullptr, b, Nst, Rpad, 0.f, 0.f, 0.f,
                                                 0.f, s);
            nblk = Nst / 64;
        } else {
            ee = launch_energy_f64(fp32J, b.X, b.epart, Nst, Rpad, s, b.stop);
            nblk = Nst / 64;
        }
        if (ee == hipSuccess) ee = launch_best(b, nblk, run.N, run.R, Rpad, m, s);
        // a cancel request seen here stops the run at this sample point
        if (ee == hipSuccess && run.cancel && m < k1) ee = launch_poll_cancel(run.cancel, b.stop, m, s);
        if (ee != hipSuccess) return derr(HSB_EDEVICE, "%s", hipGetErrorString(ee));
        return HSB_OK;
    };
    if (k1 == k0) return sample(k0);
    // 32-row tiles per wave: the default of the digit combination, or the
    // other height (odd tiles).  Tiles 0 and 1 run the persistent kernel, 2
    // and 3 one launch per step (the same results).
    const int nt_def = tiles_per_wave(p->njd, bsb ? 4 : 1, false);
    const int nt = (run.tile & 1) ? 3 - nt_def : nt_def;
    // per-wave partials of the thermostat's sum (32 or 64 rows)
    const int nh_parts = Nst / (32 * nt);
    if (run.tile < 2) {
        const void *fn = persist_kernel(p->njd, nxd, nt, run.nh != nullptr);
        const int wpt = Np / (128 * nt), nwt = 4 * wpt;
        const int tpl = persist_teams_per_launch(fn, wpt);
        const int nteams = Rpad / 32;
        if (tpl >= 8) {
            const int tpl_run = nteams < tpl ? 8 * ((nteams + 7) / 8) : tpl;
            const size_t nsync = (size_t)8 * wpt * (tpl_run / 8) + (size_t)tpl_run * nwt;
            const long long seg_max = (long long)(k1 - k0) < interval ? (k1 - k0) : interval;
            rc = grow(&p->sync, &p->sync_n, nsync);
            if (!rc) rc = grow(&p->ptab, &p->ptab_n, (size_t)seg_max);
            if (!rc) rc = grow(&p->err, &p->err_n, (size_t)1);
            if (rc) return rc;
            hipLaunchKernelGGL(k_i8_fill_u32, dim3(1), dim3(1), 0, s,
                               reinterpret_cast<uint32_t *>(p->err), (size_t)1, 0u);
            int local_ok = run.local_exchange ? 1 : 0;
            const float a0dt_v = a0dt;
            I8NH nhp{};
            if (run.nh) nhp = I8NH{run.nh->xi, run.nh->part, nh_parts, k0, run.nh->c, run.nh->NT};
            for (int a = k0; a < k1;) {
                // segment [a, e): up to the next sample point
                const long long nxt = ((long long)a / interval + 1) * interval;
                const int e_k = nxt < k1 ? (int)nxt : k1;
                hipLaunchKernelGGL(k_i8_ptab, dim3((unsigned)((e_k - a + 255) / 256)), dim3(256), 0,
                                   s, p->ptab, a, e_k - a, a0, (float)run.Ns);
                e = timer.begin(s);
                size_t nl = 0;
                for (int t0 = 0; t0 < nteams && e == hipSuccess; t0 += tpl) {
                    const int ntm = nteams - t0 < tpl ? nteams - t0 : tpl;
                    const dim3 grid((unsigned)(8 * ((ntm + 7) / 8) * wpt));
                    const size_t nfill = (size_t)grid.x + (size_t)ntm * nwt;
                    hipLaunchKernelGGL(k_i8_fill_u32, dim3((unsigned)((nfill + 255) / 256)),
                                       dim3(256), 0, s, p->sync, nfill, kI8NoFlag);
                    int Nst_v = Nst, Np_v = Np, Rpad_v = Rpad, t0_v = t0, ntm_v = ntm, a_v = a,
                        e_v = e_k;
                    float c0_v = c0, dt_v = dt;
                    const int32_t *stop = b.stop;
                    void *args[] = {(void *)&p->jd,    (void *)&p->rowscale, (void *)&p->xd,
                                    (void *)&p->sync,  (void *)&b.X,         (void *)&b.Y,
                                    (void *)&b.gamma,  (void *)&p->ptab,     (void *)&b.status,
                                    (void *)&p->err,   (void *)&stop,        (void *)&local_ok,
                                    (void *)&Nst_v,    (void *)&Np_v,        (void *)&Rpad_v,
                                    (void *)&t0_v,     (void *)&ntm_v,       (void *)&a_v,
                                    (void *)&e_v,      (void *)&c0_v,        (void *)&dt_v,
                                    (void *)&a0dt_v,   (void *)&nhp};
                    // every workgroup of the grid is resident at once (the grid
                    // never exceeds the occupancy-derived capacity), and every
                    // wait inside the kernel is bounded
                    e = hipLaunchKernel(fn, grid, dim3(256), args, 0, s);
                    ++nl;
                }
                if (e == hipSuccess) e = timer.end(s, nl);
                if (e != hipSuccess)
                    return derr(HSB_EDEVICE, "digit persistent launch: %s", hipGetErrorString(e));
                if (is_sample(e_k)) {
                    rc = sample(e_k);
                    if (rc) return rc;
                }
                a = e_k;
            }
            if (run.nh) {  // xi after the last step, as after the per-step launches
                e = launch_nh_final(run.nh->xi, run.nh->part, nh_parts, run.R, Rpad, run.nh->xi,
                                    run.nh->c, run.nh->NT, k1 - k0, k0, b.stop, s);
                if (e != hipSuccess) return derr(HSB_EDEVICE, "thermostat: %s", hipGetErrorString(e));
            }
            return HSB_OK;
        }
    }
    int cur = 0;
    size_t nrun = 0;  // step launches since the last energy sample
    for (int k = k0; k < k1; ++k) {
        // a(t_k) = a0 k / Ns in single precision; p = a0 - a(t_k)
        const float ak = (a0 * (float)k) / (float)run.Ns;
        const float pk = a0 - ak;
        const int8_t *xin = p->xd + cur * set;
        int8_t *xout = p->xd + (cur ^ 1) * set;
        e = timer.begin(s);
        if (e == hipSuccess && run.nh) {
            // the thermostat fused into the step: slots alternate with the step
            const int j = k - k0;
            NHFused f;
            f.xi_in = run.nh->xi + (size_t)(j & 1) * Rpad;
            f.xi_out = run.nh->xi + (size_t)((j + 1) & 1) * Rpad;
            f.part_out = run.nh->part + (size_t)(j & 1) * nh_parts * Rpad;
            f.part_in = run.nh->part + (size_t)((j + 1) & 1) * nh_parts * Rpad;
            f.nparts = nh_parts;
            f.first = j == 0;
            f.c = run.nh->c;
            f.NT = run.nh->NT;
            if (p->njd == 1)
                e = bsb ? launch_step<1, 4, 4, true>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                     a0dt, s, f)
                        : launch_step<1, 1, 4, true>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                     a0dt, s, f);
            else
                e = bsb ? launch_step<4, 4, 2, true>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                     a0dt, s, f)
                        : launch_step<4, 1, 2, true>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                     a0dt, s, f);
        } else if (e == hipSuccess) {
            const NHFused none{};
            if (p->njd == 1)
                e = bsb ? launch_step<1, 4, 4, false>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                      a0dt, s, none)
                        : launch_step<1, 1, 4, false>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                      a0dt, s, none);
            else
                e = bsb ? launch_step<4, 4, 2, false>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                      a0dt, s, none)
                        : launch_step<4, 1, 2, false>(nt, p, xin, xout, b, Nst, Rpad, pk, c0, dt,
                                                      a0dt, s, none);
        }
        if (e != hipSuccess) return derr(HSB_EDEVICE, "digit step: %s", hipGetErrorString(e));
        ++nrun;
        cur ^= 1;
        if (is_sample(k + 1)) {
            e = timer.end(s, nrun);
            if (e != hipSuccess) return derr(HSB_EDEVICE, "%s", hipGetErrorString(e));
            nrun = 0;
            rc = sample(k + 1);
            if (rc) return rc;
        }
    }
    if (run.nh) {  // xi after the last step, from its slot and partials, into slot 0
        e = launch_nh_final(run.nh->xi, run.nh->part, nh_parts, run.R, Rpad, run.nh->xi,
                            run.nh->c, run.nh->NT, k1 - k0, k0, b.stop, s);
        if (e != hipSuccess) return derr(HSB_EDEVICE, "thermostat: %s", hipGetErrorString(e));
    }
    return HSB_OK;
}

}  // namespace hsb
