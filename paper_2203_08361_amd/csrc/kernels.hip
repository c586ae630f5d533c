// libhsb kernels: state set-up, the per-step FP32 field GEMM with the fused
// update, energy partial sums, best-sample tracking and output.
//
// The field of eqs. (4)/(5) is the dense product F = J B with B = x (bSB) or
// B = sgn(x) (dSB), J: Npad x Npad, B: Npad x Rpad.  One launch performs one
// time step: every workgroup computes a 64 x 64 tile of F on the FP32 matrix
// cores (v_mfma_f32_32x32x2f32, LDS double-buffered K loop) and applies
// eqs. (16)-(22) to the same tile of (x, y) in its epilogue, writing the next
// step's operand into the other ping-pong buffer (synchronous update: every
// f_i of step k reads x(t_k) only).
#include "hsb_device.h"
#include "kernels.h"

namespace hsb {

// ------------------------------------------------------------ cancellation
//
// A run stops at a sample point when its context's cancel request (a word of
// pinned host memory) is seen there: the per-step plans enqueue a poll after
// each sample, which records the step in the run's stop word, and every later
// step and sample kernel of the run returns at once when that word is set.

__device__ __forceinline__ bool stopped(const int32_t *stop) {
    return stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0;
}

__global__ void k_stop_init(int32_t *stop) { stop[0] = -1; }

// after the sample at step m: stop here if the request is set (and no earlier
// sample has stopped the run)
__global__ void k_poll_cancel(const int32_t *cancel, int32_t *stop, int m) {
    if (stop[0] < 0 && __hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
        stop[0] = m;
}

// stop_step[r]: the step each replica reached -- the run's stop word (per-step
// plans) or its team's (tstop[r / 32], FP4 plan), else k1 -- and bit 2 of the
// status word if any replica stopped before k1
__global__ void k_output_stop(const int32_t *__restrict__ stop, const int32_t *__restrict__ tstop,
                              int R, int k1, int32_t *__restrict__ stop_step,
                              int32_t *__restrict__ status) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    int m = k1;
    if (stop && stop[0] >= 0) m = stop[0];
    if (tstop && tstop[r >> 5] >= 0 && tstop[r >> 5] < m) m = tstop[r >> 5];
    if (stop_step) stop_step[r] = m;
    if (m < k1) __hip_atomic_fetch_or(status, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ state set-up

// Columns [0, ncols) of a state with leading dimension ld: replica r < R of
// spin i < N draws from (seed, r, i); everything else is zero.
__global__ void k_init_seeded(float *__restrict__ X, float *__restrict__ Y, int N, int R, int ncols,
                              int ld, uint64_t seed_v, const uint64_t *__restrict__ seed_p,
                              float amp) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (r >= ncols) return;
    const uint64_t seed = seed_p ? seed_p[0] : seed_v;
    float x = 0.0f, y = 0.0f;
    if (i < N && r < R) {
        x = amp * uniform_open(rng_key(seed, 0, (uint64_t)r, (uint64_t)i));
        y = amp * uniform_open(rng_key(seed, 1, (uint64_t)r, (uint64_t)i));
    }
    X[(size_t)i * ld + r] = x;
    Y[(size_t)i * ld + r] = y;
}

__global__ void k_load_state(float *__restrict__ X, float *__restrict__ Y,
                             const float *__restrict__ x0, const float *__restrict__ y0, int N,
                             int R, int Rpad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (r >= Rpad) return;
    const bool ok = i < N && r < R;
    X[(size_t)i * Rpad + r] = ok ? x0[(size_t)r * N + i] : 0.0f;
    Y[(size_t)i * Rpad + r] = ok ? y0[(size_t)r * N + i] : 0.0f;
}

__global__ void k_make_operand(float *__restrict__ B, const float *__restrict__ X, int variant,
                               size_t n) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    B[e] = variant == 0 ? X[e] : sgnf(X[e]);
}

__global__ void k_fill_gamma(float *__restrict__ g, const float *__restrict__ gamma_rep,
                             float gamma, int R, int Rpad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Rpad) return;
    g[r] = r < R ? (gamma_rep ? gamma_rep[r] : gamma) : 0.0f;
}

// Nose-Hoover thermostat (eqs. (6)-(8)): xi per replica, in FP64.  The
// heating rate of step k is -xi(t_k) rounded to float, written into the
// per-replica gamma array that the step kernels read; then
//   xi(t_k+1) = xi(t_k) + c (sum_i y_i(t_k)^2 - N T),  c = dt / M,
// with the sum of the state before the step (explicit Euler on eq. (8)).
// Start value: xi0[r], or -gamma_r (so that 1/M = 0 is heated SB itself).
// Padding columns get xi = 0, so that the steps read defined values there.
__global__ void k_nh_init(double *__restrict__ xi, const double *__restrict__ xi0,
                          const float *__restrict__ g, int R, int Rpad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < Rpad) xi[r] = r >= R ? 0.0 : (xi0 ? xi0[r] : -(double)g[r]);
}

// xi after the n >= 1 fused steps done (n = steps, or up to the stop word's
// step): the step-(n-1) value in slot n % 2 plus c (its partials in slot
// (n-1) % 2 - N T), into xi_dst.
__global__ void k_nh_final(const double *__restrict__ xi, const double *__restrict__ part,
                           int nparts, int R, int Rpad, double *__restrict__ xi_dst, double c,
                           double NT, int steps, int k0, const int32_t *__restrict__ stop) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int n = (stop && stop[0] >= 0) ? stop[0] - k0 : steps;
    const double *xi_in = xi + (size_t)(n & 1) * Rpad;
    const double *part_in = part + (size_t)((n - 1) & 1) * nparts * Rpad;
    double S = 0.0;
    for (int q = 0; q < nparts; ++q) S += part_in[(size_t)q * Rpad + r];
    xi_dst[r] = xi_in[r] + c * (S - NT);
}

// ---------------------------------------------- incremental dSB field
// For integer J the dSB field f = J sgn(x) (eq. (5)) is an exact integer, so
// it can be carried from step to step: when the spins j flip to s_j, f
// changes by 2 s_j J[:, j].  The field of the current signs is kept as int32,
// replica-major ([Rpad][Npad]); every integer sum is exact in any order.
// J is symmetric, so its column j is the contiguous row j.

// F[r][i] = sum_j J[i][j] sgn(x_j of replica r), rows i < Npad, replicas r < R.
__global__ __launch_bounds__(256) void k_inc_init(const float *__restrict__ J,
                                                  const float *__restrict__ X,
                                                  int32_t *__restrict__ F, int N, int Npad,
                                                  int Rpad, int R) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= Npad) return;
    // replicas r = blockIdx.y, blockIdx.y + gridDim.y, ... (grid.y is capped)
    for (int r = blockIdx.y; r < R; r += gridDim.y) {
        int acc = 0;
        for (int j = 0; j < N; ++j) {
            const int Jv = (int)J[(size_t)j * Npad + i];
            acc += X[(size_t)j * Rpad + r] >= 0.0f ? Jv : -Jv;
        }
        F[(size_t)r * Npad + i] = acc;
    }
}

// One step from the exact field: the update of eqs. (16)-(22) (the common
// canonical form), then every spin whose sign changed goes on its replica's
// list as +(i+1) (now +1) or -(i+1) (now -1).
__global__ __launch_bounds__(256) void k_inc_step(float *__restrict__ X, float *__restrict__ Y,
                                                  const int32_t *__restrict__ F,
                                                  const float *__restrict__ gam,
                                                  int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ list, int N, int Npad,
                                                  int Rpad, int R, float p, float c0, float dt,
                                                  float a0dt, const int32_t *__restrict__ stop) {
    const int r = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
    if (r >= R || i >= N || stopped(stop)) return;
    const size_t idx = (size_t)i * Rpad + r;
    float x = X[idx], y = Y[idx];
    const bool was = x >= 0.0f;
    sb_update((float)F[(size_t)r * Npad + i], p, c0, dt, a0dt, gam[r] * dt, x, y);
    X[idx] = x;
    Y[idx] = y;
    const bool now = x >= 0.0f;
    if (now != was) {
        const int pos = atomicAdd(cnt + r, 1);
        list[(size_t)r * Npad + pos] = now ? i + 1 : -(i + 1);
    }
}

// F[r][i] += 2 s_j J[j][i] over the listed flips of replica r; the block of
// row 0 also clears the next step's counter of r.
__global__ __launch_bounds__(256) void k_inc_field(int32_t *__restrict__ F,
                                                   const float *__restrict__ J,
                                                   const int32_t *__restrict__ cnt,
                                                   const int32_t *__restrict__ list,
                                                   int32_t *__restrict__ cnt_next, int Npad,
                                                   int R, const int32_t *__restrict__ stop) {
    if (stopped(stop)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    // replicas r = blockIdx.y, blockIdx.y + gridDim.y, ... (grid.y is capped)
    for (int r = blockIdx.y; r < R; r += gridDim.y) {
        if (blockIdx.x == 0 && threadIdx.x == 0) cnt_next[r] = 0;
        if (i >= Npad) continue;
        const int n = cnt[r];
        const int32_t *L = list + (size_t)r * Npad;
        int acc = F[(size_t)r * Npad + i];
        for (int q = 0; q < n; ++q) {
            const int e = L[q];
            const int j = (e > 0 ? e : -e) - 1;
            const int Jv = (int)J[(size_t)j * Npad + i];
            acc += e > 0 ? 2 * Jv : -2 * Jv;
        }
        F[(size_t)r * Npad + i] = acc;
    }
}

__global__ void k_zero_i32n(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_copy_f64(double *__restrict__ dst, const double *__restrict__ src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_reset_tracking(double *best_e, double *last_e, int32_t *best_step, int32_t *bad,
                                 int32_t *status, int Rpad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) status[0] = 0;
    if (r >= Rpad) return;
    best_e[r] = __builtin_huge_val();
    last_e[r] = __builtin_nan("");
    best_step[r] = -1;
    bad[r] = 0;
}

// --------------------------------------------------- FP32 GEMM main loop
// 256 threads, four waves in a 2 x 2 arrangement of 32 x 32 tiles.  LDS tiles
// are stored K-major ([k][i] and [k][r]) so that each MFMA operand read is a
// run of 32 consecutive floats.
//
// v_mfma_f32_32x32x2f32 operand layout (lane l of 64):
//   A: A[l % 32][l / 32]     B: B[l / 32][l % 32]
//   D: item v of lane l is D[8*(v/4) + 4*(l/32) + v%4][l % 32]

template <bool SIGN_B>
__device__ __forceinline__ v16f gemm_tile_fp32(const float *__restrict__ J,
                                               const float *__restrict__ Bsrc, int Npad, int Rpad,
                                               int i0, int r0, float (*As)[32][68],
                                               float (*Bs)[32][68]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int a_row = t >> 2, a_col = (t & 3) * 8;
    const int b_row = t >> 3, b_col = (t & 7) * 8;
    const float *Ap = J + (size_t)(i0 + a_row) * Npad + a_col;
    const float *Bp = Bsrc + (size_t)b_row * Rpad + r0 + b_col;
    v4f ra0 = *(const v4f *)(Ap), ra1 = *(const v4f *)(Ap + 4);
    v4f rb0 = *(const v4f *)(Bp), rb1 = *(const v4f *)(Bp + 4);
    v16f acc = {};
    const int nk = Npad / 32;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][a_col + q][a_row] = ra0[q];
            As[buf][a_col + 4 + q][a_row] = ra1[q];
        }
        if (SIGN_B) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rb0[q] = sgnf(rb0[q]);
                rb1[q] = sgnf(rb1[q]);
            }
        }
        *(v4f *)&Bs[buf][b_row][b_col] = rb0;
        *(v4f *)&Bs[buf][b_row][b_col + 4] = rb1;
        __syncthreads();
        if (kt + 1 < nk) {
            Ap += 32;
            Bp += (size_t)32 * Rpad;
            ra0 = *(const v4f *)(Ap);
            ra1 = *(const v4f *)(Ap + 4);
            rb0 = *(const v4f *)(Bp);
            rb1 = *(const v4f *)(Bp + 4);
        }
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const float a = As[buf][2 * kk + (lane >> 5)][32 * wr + (lane & 31)];
            const float b = Bs[buf][2 * kk + (lane >> 5)][32 * wc + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    }
    return acc;
}

// One time step (field + fused eqs. (16)-(22)).  Grid (Rpad/64, Npad/64).
template <int VARIANT, bool NH>
__global__ __launch_bounds__(256) void k_step_fp32(const float *__restrict__ J,
                                                   const float *__restrict__ Bin,
                                                   float *__restrict__ Bout, float *__restrict__ X,
                                                   float *__restrict__ Y,
                                                   const float *__restrict__ gam, int Npad,
                                                   int Rpad, float p, float c0, float dt,
                                                   float a0dt, NHFused nhf,
                                                   const int32_t *__restrict__ stop) {
    __shared__ float As[2][32][68];
    __shared__ float Bs[2][32][68];
    if (stopped(stop)) return;
    const int r0 = blockIdx.x * kTile, i0 = blockIdx.y * kTile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int r = r0 + 32 * wc + (lane & 31);
    // thermostat: xi(t_k) of this lane's replica from the previous step's
    // 32-row partials; the four half-waves on the same replicas each add every
    // fourth, combined in a fixed order (before the products, so that the
    // loads overlap them)
    double xi_k = 0.0;
    if constexpr (NH) {
        __shared__ double s_part[2][4][32];
        const int grp = 2 * wr + (lane >> 5);
        xi_k = nhf.xi_in[r];
        if (!nhf.first) {
            double Ssum = 0.0;
            for (int q = grp; q < nhf.nparts; q += 4) Ssum += nhf.part_in[(size_t)q * Rpad + r];
            s_part[wc][grp][lane & 31] = Ssum;
            __syncthreads();
            double S4 = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) S4 += s_part[wc][q][lane & 31];
            xi_k = xi_k + nhf.c * (S4 - nhf.NT);
        }
        if (i0 == 0 && wr == 0 && (lane >> 5) == 0) nhf.xi_out[r] = xi_k;
    }
    const v16f acc = gemm_tile_fp32<false>(J, Bin, Npad, Rpad, i0, r0, As, Bs);
    const float gdt = NH ? (float)(-xi_k) * dt : gam[r] * dt;
    // all loads of the tile's state before the first store (they overlap)
    float xs[16], ys[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = i0 + 32 * wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        xs[v] = X[(size_t)i * Rpad + r];
        ys[v] = Y[(size_t)i * Rpad + r];
    }
    if constexpr (NH) {  // sum of y_i(t_k)^2 over this wave's 32 rows (exact squares)
        double t2 = 0.0;
#pragma unroll
        for (int v = 0; v < 16; ++v) t2 += (double)ys[v] * (double)ys[v];
        t2 += __shfl_xor(t2, 32);
        if ((lane >> 5) == 0) nhf.part_out[(size_t)((i0 + 32 * wr) / 32) * Rpad + r] = t2;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = i0 + 32 * wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const size_t idx = (size_t)i * Rpad + r;
        float x = xs[v], y = ys[v];
        sb_update(acc[v], p, c0, dt, a0dt, gdt, x, y);
        X[idx] = x;
        Y[idx] = y;
        Bout[idx] = VARIANT == 0 ? x : sgnf(x);
    }
}

// Energy partials, exact for integer-valued J: F = J sgn(x) on FP32 matrix
// cores (every product and sum is an integer below 2^24), then per 32-row
// block sum_i s_i F_i.  epart[(Npad/32)][Rpad].
__global__ __launch_bounds__(256) void k_energy_fp32(const float *__restrict__ J,
                                                     const float *__restrict__ X,
                                                     double *__restrict__ epart, int Npad,
                                                     int Rpad, const int32_t *__restrict__ stop) {
    __shared__ float As[2][32][68];
    __shared__ float Bs[2][32][68];
    if (stopped(stop)) return;
    const int r0 = blockIdx.x * kTile, i0 = blockIdx.y * kTile;
    const v16f acc = gemm_tile_fp32<true>(J, X, Npad, Rpad, i0, r0, As, Bs);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int r = r0 + 32 * wc + (lane & 31);
    float part = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = i0 + 32 * wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        part += sgnf(X[(size_t)i * Rpad + r]) * acc[v];
    }
    part += __shfl_xor(part, 32);
    if (lane < 32) epart[(size_t)(blockIdx.y * 2 + wr) * Rpad + r] = (double)part;
}

// Energy partials in FP64 for any J: 64 x 64 tile, each thread 4 x 4 outputs,
// fixed summation order.  epart[(Npad/64)][Rpad].
__global__ __launch_bounds__(256) void k_energy_f64(const float *__restrict__ J,
                                                    const float *__restrict__ X,
                                                    double *__restrict__ epart, int Npad,
                                                    int Rpad, const int32_t *__restrict__ stop) {
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    __shared__ double red[16][65];
    if (stopped(stop)) return;
    const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
    const int r0 = blockIdx.x * kTile, i0 = blockIdx.y * kTile;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < Npad; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            const int ai = e >> 4, ak = e & 15;
            As[ak][ai] = (double)J[(size_t)(i0 + ai) * Npad + k0 + ak];
            const int bk = e >> 6, br = e & 63;
            Bs[bk][br] = (double)sgnf(X[(size_t)(k0 + bk) * Rpad + r0 + br]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[k][tr + 16 * q];
                b[q] = Bs[k][tc + 16 * q];
            }
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) acc[ii][rr] = __fma_rn(a[ii], b[rr], acc[ii][rr]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        double part = 0.0;
        const int r = r0 + tc + 16 * rr;
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
            const int i = i0 + tr + 16 * ii;
            part += (double)sgnf(X[(size_t)i * Rpad + r]) * acc[ii][rr];
        }
        red[tr][tc + 16 * rr] = part;
    }
    __syncthreads();
    if (t < 64) {
        double s = 0.0;
        for (int q = 0; q < 16; ++q) s += red[q][t];
        epart[(size_t)blockIdx.y * Rpad + r0 + t] = s;
    }
}

// Best-sample tracking after a sample point `step`: total energy per replica
// in a fixed order, non-finite detection, strict-improvement best update
// (ties keep the earliest sample) with a copy of the spins.  A workgroup of
// 1024 threads owns 64 replicas (lane = replica); its 16 waves split the rows.
// With traces, row `trow` of trace_e / trace_t ([.][R]) receives the energy
// and T_inst = (1/N) sum_i y_i^2 (eq. (9); FP64 sums in a fixed order).
__global__ __launch_bounds__(1024) void k_best(const double *__restrict__ epart, int nblk,
                                               const float *__restrict__ X,
                                               const float *__restrict__ Y, int N, int R,
                                               int Rpad, double *__restrict__ best_e,
                                               double *__restrict__ last_e,
                                               int32_t *__restrict__ best_step,
                                               int32_t *__restrict__ bad,
                                               int8_t *__restrict__ best_s,
                                               int32_t *__restrict__ status, int step,
                                               double *__restrict__ trace_e,
                                               double *__restrict__ trace_t, int trow,
                                               const int32_t *__restrict__ stop) {
    __shared__ int s_bad[16][64];
    if (stopped(stop)) return;
    __shared__ double s_t[16][64];
    __shared__ int s_take[64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + l;
    int nf = 0;
    double t = 0.0;
    if (r < R)
        for (int i = w; i < N; i += 16) {
            const float x = X[(size_t)i * Rpad + r], y = Y[(size_t)i * Rpad + r];
            nf |= !(isfinite(x) && isfinite(y));
            t += (double)y * (double)y;
        }
    s_bad[w][l] = nf;
    s_t[w][l] = t;
    __syncthreads();
    if (w == 0) {
        int take = 0;
        if (r < R) {
            for (int q = 1; q < 16; ++q) {
                nf |= s_bad[q][l];
                t += s_t[q][l];
            }
            double e = 0.0;
            for (int b = 0; b < nblk; ++b) e += epart[(size_t)b * Rpad + r];
            e = -0.5 * e;
            if (nf) {
                bad[r] = 1;
                status[0] = 1;
                e = __builtin_nan("");
            }
            last_e[r] = e;
            if (trace_e) trace_e[(size_t)trow * R + r] = e;
            if (trace_t) trace_t[(size_t)trow * R + r] = t / N;
            if (e < best_e[r]) {
                best_e[r] = e;
                best_step[r] = step;
                take = 1;
            }
        }
        s_take[l] = take;
    }
    __syncthreads();
    if (!s_take[l]) return;
    for (int i = w; i < N; i += 16)
        best_s[(size_t)i * Rpad + r] = X[(size_t)i * Rpad + r] >= 0.0f ? 1 : -1;
}

__global__ void k_output_spins(const float *__restrict__ X, const float *__restrict__ Y,
                               const int8_t *__restrict__ best_s,
                               const int32_t *__restrict__ best_step, int N, int R, int Rpad,
                               int return_best, int8_t *__restrict__ spins,
                               float *__restrict__ x_out, float *__restrict__ y_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int r = blockIdx.y; r < R; r += gridDim.y) {
        const size_t src = (size_t)i * Rpad + r, dst = (size_t)r * N + i;
        const float x = X[src];
        spins[dst] = (return_best && best_step[r] >= 0) ? best_s[src] : (x >= 0.0f ? 1 : -1);
        if (x_out) x_out[dst] = x;
        if (y_out) y_out[dst] = Y[src];
    }
}

__global__ void k_output_energy(const double *__restrict__ best_e,
                                const double *__restrict__ last_e,
                                const int32_t *__restrict__ best_step_in,
                                const int32_t *__restrict__ bad, int R, int return_best,
                                double *__restrict__ energy, double *__restrict__ best_energy,
                                double *__restrict__ final_energy,
                                int32_t *__restrict__ best_step) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double nan = __builtin_nan("");
    const bool b = bad[r] != 0;
    energy[r] = b ? nan : (return_best ? best_e[r] : last_e[r]);
    if (best_energy) best_energy[r] = b ? nan : best_e[r];
    if (final_energy) final_energy[r] = b ? nan : last_e[r];
    if (best_step) best_step[r] = best_step_in[r];
}

// flag[0] = 1 if any of the n values has |x| > 1 or is not finite
__global__ void k_bound_flag(const float *__restrict__ X, size_t n, int32_t *flag) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (!(fabsf(X[e]) <= 1.0f)) atomicOr(flag, 1);
}

__global__ void k_clear_i32(int32_t *p) { p[0] = 0; }

// job of column r: the last job with col0 <= r (jobs sorted by col0)
__device__ __forceinline__ int batch_job_of(const BatchJob *jobs, int njobs, int r) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].col0 <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_init_batch(float *__restrict__ X, float *__restrict__ Y, float *__restrict__ gamma,
                             const BatchJob *__restrict__ jobs, int njobs, int Rtot, float amp) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (r >= Rtot) return;
    const BatchJob jb = jobs[batch_job_of(jobs, njobs, r)];
    const int rep = r - jb.col0;
    const bool col_ok = rep >= 0 && rep < jb.R;
    float x = 0.0f, y = 0.0f;
    if (col_ok && i < jb.N) {
        x = amp * uniform_open(rng_key(jb.seed, 0, (uint64_t)rep, (uint64_t)i));
        y = amp * uniform_open(rng_key(jb.seed, 1, (uint64_t)rep, (uint64_t)i));
    }
    X[(size_t)i * Rtot + r] = x;
    Y[(size_t)i * Rtot + r] = y;
    if (i == 0) gamma[r] = col_ok ? jb.gamma : 0.0f;
}

__global__ void k_output_batch_spins(const float *__restrict__ X, const int8_t *__restrict__ best_s,
                                     const int32_t *__restrict__ best_step,
                                     const BatchJob *__restrict__ jobs, int njobs, int Rtot,
                                     int return_best) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int r = blockIdx.y; r < Rtot; r += gridDim.y) {
        const BatchJob jb = jobs[batch_job_of(jobs, njobs, r)];
        const int rep = r - jb.col0;
        if (rep < 0 || rep >= jb.R || i >= jb.N) continue;
        const size_t src = (size_t)i * Rtot + r;
        jb.spins[(size_t)rep * jb.N + i] =
            (return_best && best_step[r] >= 0) ? best_s[src] : (X[src] >= 0.0f ? 1 : -1);
    }
}

__global__ void k_output_batch_energy(const double *__restrict__ best_e,
                                      const double *__restrict__ last_e,
                                      const int32_t *__restrict__ bad,
                                      const BatchJob *__restrict__ jobs, int njobs, int Rtot,
                                      int return_best) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Rtot) return;
    const BatchJob jb = jobs[batch_job_of(jobs, njobs, r)];
    const int rep = r - jb.col0;
    if (rep < 0 || rep >= jb.R) return;
    jb.energy[rep] = bad[r] ? __builtin_nan("") : (return_best ? best_e[r] : last_e[r]);
}

// ------------------------------------------------------------ launchers

void free_state_bufs(StateBufs &b) {
    void *ptrs[] = {b.X,      b.Y,         b.B[0],      b.B[1], b.gamma, b.epart,
                    b.best_e, b.last_e,    b.best_step, b.bad,  b.best_s, b.status};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    b = StateBufs{};
}

hipError_t alloc_state(StateBufs &b, int Npad, int Rpad, bool fp32_plan) {
    b = StateBufs{};
    const size_t nr = (size_t)Rpad, ns = (size_t)Npad * nr;
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    alloc((void **)&b.X, ns * sizeof(float));
    alloc((void **)&b.Y, ns * sizeof(float));
    if (fp32_plan) {
        alloc((void **)&b.B[0], ns * sizeof(float));
        alloc((void **)&b.B[1], ns * sizeof(float));
    }
    alloc((void **)&b.gamma, nr * sizeof(float));
    if (fp32_plan) alloc((void **)&b.epart, (size_t)(Npad / 32) * nr * sizeof(double));
    alloc((void **)&b.best_e, nr * sizeof(double));
    alloc((void **)&b.last_e, nr * sizeof(double));
    alloc((void **)&b.best_step, nr * sizeof(int32_t));
    alloc((void **)&b.bad, nr * sizeof(int32_t));
    alloc((void **)&b.best_s, ns);
    alloc((void **)&b.status, sizeof(int32_t));
    if (e != hipSuccess) free_state_bufs(b);
    return e;
}

static inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_init_seeded(float *X, float *Y, int N, int R, int Npad, int ncols, int ld,
                              uint64_t seed, float amp, hipStream_t s, const uint64_t *seed_p) {
    hipLaunchKernelGGL(k_init_seeded, dim3(cdiv(ncols, 256), Npad), dim3(256), 0, s, X, Y, N, R,
                       ncols, ld, seed, seed_p, amp);
    return hipGetLastError();
}

hipError_t launch_init_batch(float *X, float *Y, float *gamma, const BatchJob *jobs, int njobs,
                             int Npad, int Rtot, float amp, hipStream_t s) {
    hipLaunchKernelGGL(k_init_batch, dim3(cdiv(Rtot, 256), Npad), dim3(256), 0, s, X, Y, gamma,
                       jobs, njobs, Rtot, amp);
    return hipGetLastError();
}

hipError_t launch_output_batch(const StateBufs &b, const BatchJob *jobs, int njobs, int Nmax,
                               int Rtot, int return_best, hipStream_t s) {
    hipLaunchKernelGGL(k_output_batch_spins, dim3(cdiv(Nmax, 256), Rtot < 32768 ? Rtot : 32768),
                       dim3(256), 0, s, b.X, b.best_s, b.best_step, jobs, njobs, Rtot,
                       return_best);
    hipLaunchKernelGGL(k_output_batch_energy, dim3(cdiv(Rtot, 256)), dim3(256), 0, s, b.best_e,
                       b.last_e, b.bad, jobs, njobs, Rtot, return_best);
    return hipGetLastError();
}

hipError_t launch_load_state(float *X, float *Y, const float *x0, const float *y0, int N, int R,
                             int Npad, int Rpad, hipStream_t s) {
    hipLaunchKernelGGL(k_load_state, dim3(cdiv(Rpad, 256), Npad), dim3(256), 0, s, X, Y, x0, y0,
                       N, R, Rpad);
    return hipGetLastError();
}

hipError_t launch_make_operand(float *B, const float *X, int variant, int Npad, int Rpad,
                               hipStream_t s) {
    const size_t n = (size_t)Npad * Rpad;
    hipLaunchKernelGGL(k_make_operand, dim3(cdiv(n, 256)), dim3(256), 0, s, B, X, variant, n);
    return hipGetLastError();
}

hipError_t launch_fill_gamma(float *g, const float *gamma_rep, float gamma, int R, int Rpad,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_fill_gamma, dim3(cdiv(Rpad, 256)), dim3(256), 0, s, g, gamma_rep, gamma,
                       R, Rpad);
    return hipGetLastError();
}

hipError_t launch_nh_init(const NHState &nh, const double *xi0, const float *gamma, int R,
                          int Rpad, hipStream_t s) {
    hipLaunchKernelGGL(k_nh_init, dim3(cdiv(Rpad, 256)), dim3(256), 0, s, nh.xi, xi0, gamma, R,
                       Rpad);
    return hipGetLastError();
}

hipError_t launch_nh_final(const double *xi, const double *part, int nparts, int R, int Rpad,
                           double *xi_dst, double c, double NT, int steps, int k0,
                           const int32_t *stop, hipStream_t s) {
    hipLaunchKernelGGL(k_nh_final, dim3(cdiv(R, 256)), dim3(256), 0, s, xi, part, nparts, R, Rpad,
                       xi_dst, c, NT, steps, k0, stop);
    return hipGetLastError();
}

// grid.y of the per-replica incremental launches: at most 32768 (the
// hardware limit is 65535); the kernels stride over the remaining replicas
static unsigned inc_grid_y(int R) { return (unsigned)(R < 32768 ? R : 32768); }

hipError_t launch_inc_init(const float *J, const float *X, IncState &inc, int N, int Npad,
                          int Rpad, int R, hipStream_t s) {
    hipLaunchKernelGGL(k_inc_init, dim3(cdiv(Npad, 256), inc_grid_y(R)), dim3(256), 0, s, J, X,
                       inc.F, N, Npad, Rpad, R);
    hipLaunchKernelGGL(k_zero_i32n, dim3(cdiv(2 * (size_t)Rpad, 256)), dim3(256), 0, s, inc.cnt,
                       2 * Rpad);
    return hipGetLastError();
}

hipError_t launch_inc_step(const float *J, float *X, float *Y, const float *gamma, IncState &inc,
                           int j, int N, int Npad, int Rpad, int R, float p, float c0, float dt,
                           float a0dt, hipStream_t s, const int32_t *stop) {
    int32_t *cnt = inc.cnt + (size_t)(j & 1) * Rpad, *next = inc.cnt + (size_t)((j + 1) & 1) * Rpad;
    hipLaunchKernelGGL(k_inc_step, dim3(cdiv(R, 256), N), dim3(256), 0, s, X, Y, inc.F, gamma,
                       cnt, inc.list, N, Npad, Rpad, R, p, c0, dt, a0dt, stop);
    hipLaunchKernelGGL(k_inc_field, dim3(cdiv(Npad, 256), inc_grid_y(R)), dim3(256), 0, s, inc.F,
                       J, cnt, inc.list, next, Npad, R, stop);
    return hipGetLastError();
}

hipError_t launch_copy_f64(double *dst, const double *src, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_f64, dim3(cdiv(n, 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_bound_check(const float *X, size_t n, int32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(1), 0, s, flag);
    hipLaunchKernelGGL(k_bound_flag, dim3(cdiv(n, 256)), dim3(256), 0, s, X, n, flag);
    return hipGetLastError();
}

hipError_t launch_reset_tracking(const StateBufs &b, int Rpad, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_tracking, dim3(cdiv(Rpad, 256)), dim3(256), 0, s, b.best_e,
                       b.last_e, b.best_step, b.bad, b.status, Rpad);
    return hipGetLastError();
}

hipError_t launch_step_fp32(int variant, const float *J, const float *Bin, float *Bout, float *X,
                            float *Y, const float *gamma, int Npad, int Rpad, float p, float c0,
                            float dt, float a0dt, hipStream_t s, const NHFused *nh,
                            const int32_t *stop) {
    const dim3 grid(Rpad / kTile, Npad / kTile);
    const NHFused f = nh ? *nh : NHFused{};
    if (variant == 0 && !nh)
        hipLaunchKernelGGL((k_step_fp32<0, false>), grid, dim3(256), 0, s, J, Bin, Bout, X, Y,
                           gamma, Npad, Rpad, p, c0, dt, a0dt, f, stop);
    else if (variant == 0)
        hipLaunchKernelGGL((k_step_fp32<0, true>), grid, dim3(256), 0, s, J, Bin, Bout, X, Y,
                           gamma, Npad, Rpad, p, c0, dt, a0dt, f, stop);
    else if (!nh)
        hipLaunchKernelGGL((k_step_fp32<1, false>), grid, dim3(256), 0, s, J, Bin, Bout, X, Y,
                           gamma, Npad, Rpad, p, c0, dt, a0dt, f, stop);
    else
        hipLaunchKernelGGL((k_step_fp32<1, true>), grid, dim3(256), 0, s, J, Bin, Bout, X, Y,
                           gamma, Npad, Rpad, p, c0, dt, a0dt, f, stop);
    return hipGetLastError();
}

hipError_t launch_energy_fp32(const float *J, const float *X, double *epart, int Npad, int Rpad,
                              hipStream_t s, const int32_t *stop) {
    hipLaunchKernelGGL(k_energy_fp32, dim3(Rpad / kTile, Npad / kTile), dim3(256), 0, s, J, X,
                       epart, Npad, Rpad, stop);
    return hipGetLastError();
}

hipError_t launch_energy_f64(const float *J, const float *X, double *epart, int Npad, int Rpad,
                             hipStream_t s, const int32_t *stop) {
    hipLaunchKernelGGL(k_energy_f64, dim3(Rpad / kTile, Npad / kTile), dim3(256), 0, s, J, X,
                       epart, Npad, Rpad, stop);
    return hipGetLastError();
}

hipError_t launch_best(const StateBufs &b, int nblk, int N, int R, int Rpad, int step,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_best, dim3(cdiv(R, 64)), dim3(1024), 0, s, b.epart, nblk, b.X, b.Y, N, R,
                       Rpad, b.best_e, b.last_e, b.best_step, b.bad, b.best_s, b.status, step,
                       b.trace_e, b.trace_t,
                       (b.trace_e || b.trace_t) ? trace_row(step, b.trace_k0, b.trace_interval) : 0,
                       b.stop);
    return hipGetLastError();
}

hipError_t launch_stop_init(int32_t *stop, hipStream_t s) {
    hipLaunchKernelGGL(k_stop_init, dim3(1), dim3(1), 0, s, stop);
    return hipGetLastError();
}

hipError_t launch_poll_cancel(const int32_t *cancel, int32_t *stop, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_poll_cancel, dim3(1), dim3(1), 0, s, cancel, stop, m);
    return hipGetLastError();
}

hipError_t launch_output_stop(const int32_t *stop, const int32_t *tstop, int R, int k1,
                              int32_t *stop_step, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_output_stop, dim3(cdiv(R, 256)), dim3(256), 0, s, stop, tstop, R, k1,
                       stop_step, status);
    return hipGetLastError();
}

hipError_t launch_output(const StateBufs &b, int N, int R, int Rpad, int return_best,
                         int8_t *spins, double *energy, float *x_out, float *y_out,
                         double *best_energy, double *final_energy, int32_t *best_step,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_output_spins, dim3(cdiv(N, 256), R < 32768 ? R : 32768), dim3(256), 0, s,
                       b.X, b.Y, b.best_s, b.best_step, N, R, Rpad, return_best, spins, x_out,
                       y_out);
    hipLaunchKernelGGL(k_output_energy, dim3(cdiv(R, 256)), dim3(256), 0, s, b.best_e, b.last_e,
                       b.best_step, b.bad, R, return_best, energy, best_energy, final_energy,
                       best_step);
    return hipGetLastError();
}

}  // namespace hsb
