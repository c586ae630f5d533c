// Launch wrappers of the libhsb kernels (host side).  Every device array of
// the state uses the spin-major layout [Npad][Rpad]: element (i, r) at
// i*Rpad + r, replicas contiguous.  Padding rows/columns hold zeros.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace hsb {

// HIP-event brackets around launches of a run's dominant kernel.  A bracket
// may hold several back-to-back launches of that kernel (the per-step plans
// bracket each run of consecutive steps between two energy samples), so the
// average launch duration is the bracketed time over the launch count.
struct KernelTimer {
    bool on = false;
    bool open = false;
    size_t used = 0;      // closed brackets
    size_t launches = 0;  // launches inside them
    std::vector<hipEvent_t> ev;  // pairs: begin, end
    void reset(bool enable) {
        on = enable;
        open = false;
        used = 0;
        launches = 0;
    }
    hipError_t begin(hipStream_t s) {
        if (!on || open) return hipSuccess;
        if (ev.size() < 2 * (used + 1)) {
            for (int q = 0; q < 2; ++q) {
                hipEvent_t e;
                hipError_t rc = hipEventCreate(&e);
                if (rc != hipSuccess) return rc;
                ev.push_back(e);
            }
        }
        open = true;
        return hipEventRecord(ev[2 * used], s);
    }
    // close the open bracket, which held n launches
    hipError_t end(hipStream_t s, size_t n = 1) {
        if (!on || !open) return hipSuccess;
        hipError_t rc = hipEventRecord(ev[2 * used + 1], s);
        ++used;
        launches += n;
        open = false;
        return rc;
    }
    hipError_t total_ms(double *ms) const {
        double t = 0.0;
        for (size_t i = 0; i < used; ++i) {
            float f = 0.0f;
            hipError_t rc = hipEventSynchronize(ev[2 * i + 1]);
            if (rc == hipSuccess) rc = hipEventElapsedTime(&f, ev[2 * i], ev[2 * i + 1]);
            if (rc != hipSuccess) return rc;
            t += f;
        }
        *ms = t;
        return hipSuccess;
    }
    void release() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        used = 0;
        launches = 0;
        open = false;
    }
};

// Tile sizes of the per-step FP32 path: Npad and Rpad are multiples of 64.
constexpr int kTile = 64;

struct StateBufs {
    float *X, *Y;         // [Npad][Rpad]
    float *B[2];          // field operand ping-pong: x (bSB) or sgn(x) (dSB)
    float *gamma;         // [Rpad] per-replica gamma
    double *epart;        // [Npad/32][Rpad] energy partial sums
    double *best_e;       // [Rpad]
    double *last_e;       // [Rpad]
    int32_t *best_step;   // [Rpad]
    int32_t *bad;         // [Rpad] non-finite flag per replica
    int8_t *best_s;       // [Npad][Rpad]
    int32_t *status;      // [1] bit 0: a replica non-finite; bit 1: an exchange wait timed
                          // out; bit 2: the run was cancelled
    // the run's stop word (per-step plans): -1, or the sample step at which a
    // cancel request stopped it; every later step and sample kernel returns
    // at once.  nullptr: the run cannot stop early.
    int32_t *stop = nullptr;
    // FP4 plan: the stop step of each 32-replica team (-1: not stopped)
    int32_t *tstop = nullptr;
    // optional per-call traces, [n_samples][R] (caller memory, not owned):
    // energy and T_inst of every sample point of the run steps trace_k0 ..
    double *trace_e = nullptr, *trace_t = nullptr;
    int trace_k0 = 0, trace_interval = 1;
};

// Row of the trace that receives the sample at step m of a call starting at
// step k0: the multiples of the interval in (k0, m) come before it.
inline int trace_row(int m, int k0, int interval) {
    return m / interval - k0 / interval - ((m > k0 && m % interval == 0) ? 1 : 0);
}

// rows [0, Npad) x columns [0, ncols) of a state with leading dimension ld; the
// seed is `seed`, or *seed_p (device memory, read when the kernel runs) if given
hipError_t launch_init_seeded(float *X, float *Y, int N, int R, int Npad, int ncols, int ld,
                              uint64_t seed, float amp, hipStream_t s,
                              const uint64_t *seed_p = nullptr);
hipError_t launch_load_state(float *X, float *Y, const float *x0, const float *y0, int N, int R,
                             int Npad, int Rpad, hipStream_t s);
hipError_t launch_make_operand(float *B, const float *X, int variant, int Npad, int Rpad,
                               hipStream_t s);
// g[r] = gamma_rep[r] (or gamma) for r < R, 0 for R <= r < Rpad
hipError_t launch_fill_gamma(float *g, const float *gamma_rep, float gamma, int R, int Rpad,
                             hipStream_t s);
// Nose-Hoover thermostat of a run (eqs. (6)-(8)): xi in FP64 [2][Rpad] (slot 0
// holds the start and the final value), partial sums of y^2 [2 Npad/32][Rpad];
// c = dt / M and NT = N T.
struct NHState {
    double *xi = nullptr, *part = nullptr;
    double c = 0.0, NT = 0.0;
};
// One thermostat step fused into a step kernel (FP32 and digit plans): the
// kernel forms xi(t_k) = xi_in + c (sum of part_in's nparts per-wave partials
// - NT), or takes xi_in as it is on the first step, heats at the rate -xi(t_k),
// stores xi(t_k) in xi_out (row block 0) and the per-wave partials of
// sum_i y_i(t_k)^2 of the state it reads in part_out.  Consecutive steps swap
// the slots, so no launch reads what it writes.
struct NHFused {
    const double *xi_in = nullptr;
    double *xi_out = nullptr;
    const double *part_in = nullptr;
    double *part_out = nullptr;
    int nparts = 0, first = 1;
    double c = 0.0, NT = 0.0;
};
// xi_dst[r] = xi_in[r] + c (sum of part_in's nparts partials - NT): the value
// after the last fused step
hipError_t launch_nh_final(const double *xi, const double *part, int nparts, int R, int Rpad,
                           double *xi_dst, double c, double NT, int steps, int k0,
                           const int32_t *stop, hipStream_t s);
// xi = xi0 (device [R]) if given, else -gamma[r]; 0 in the padding columns [R, Rpad)
hipError_t launch_nh_init(const NHState &nh, const double *xi0, const float *gamma, int R,
                          int Rpad, hipStream_t s);
// Incremental dSB field (integer J, |J_ij| <= 127, N <= 16384, so every field
// is an exact int32): the field of the current signs F [Rpad][Npad], the
// per-replica lists of flipped spins [Rpad][Npad] and their counters [2][Rpad]
// (one set per step parity).  J is the zero-padded FP32 store [Npad][Npad].
struct IncState {
    int32_t *F = nullptr, *list = nullptr, *cnt = nullptr;
};
// F = J sgn(X) for replicas < R; counters to 0
hipError_t launch_inc_init(const float *J, const float *X, IncState &inc, int N, int Npad,
                           int Rpad, int R, hipStream_t s);
// step j of the call: update X, Y from F, list the flips, add them to F
hipError_t launch_inc_step(const float *J, float *X, float *Y, const float *gamma, IncState &inc,
                           int j, int N, int Npad, int Rpad, int R, float p, float c0, float dt,
                           float a0dt, hipStream_t s, const int32_t *stop = nullptr);
hipError_t launch_copy_f64(double *dst, const double *src, int n, hipStream_t s);
// allocation of the run state for Npad rows and Rpad columns (all or nothing);
// without the FP32 plan's operand and energy buffers (B, epart) if !fp32_plan
hipError_t alloc_state(StateBufs &b, int Npad, int Rpad, bool fp32_plan = true);

// One job of a batch class: its columns [col0, col0 + R) of the class state
// (then up to the next job's col0: zero padding), its instance size N, seed,
// gamma and output buffers.
struct BatchJob {
    int col0, R, N;
    float gamma;
    uint64_t seed;
    int8_t *spins;   // [R][N]
    double *energy;  // [R]
};
// Seeded initial state and gamma of every job of a class in one launch:
// column r belongs to the job with the largest col0 <= r (jobs sorted by
// col0); columns past a job's R and rows past its N are zero.
hipError_t launch_init_batch(float *X, float *Y, float *gamma, const BatchJob *jobs, int njobs,
                             int Npad, int Rtot, float amp, hipStream_t s);
// Spins and energies of every job of a class (as launch_output per job)
hipError_t launch_output_batch(const StateBufs &b, const BatchJob *jobs, int njobs, int Nmax,
                               int Rtot, int return_best, hipStream_t s);
void free_state_bufs(StateBufs &b);
hipError_t launch_reset_tracking(const StateBufs &b, int Rpad, hipStream_t s);
// *flag (device) = 1 if any of X[0 .. n) has |x| > 1 or is not finite, else 0
hipError_t launch_bound_check(const float *X, size_t n, int32_t *flag, hipStream_t s);
// one step of the FP32 plan; with nh, the thermostat fused into it (32-row
// partials, see NHFused)
hipError_t launch_step_fp32(int variant, const float *J, const float *Bin, float *Bout, float *X,
                            float *Y, const float *gamma, int Npad, int Rpad, float p, float c0,
                            float dt, float a0dt, hipStream_t s, const NHFused *nh = nullptr,
                            const int32_t *stop = nullptr);
// energy partials: exact path (FP32 products, J integer-valued) -> nblk = Npad/32
hipError_t launch_energy_fp32(const float *J, const float *X, double *epart, int Npad, int Rpad,
                              hipStream_t s, const int32_t *stop = nullptr);
// energy partials in FP64 (any J) -> nblk = Npad/64
hipError_t launch_energy_f64(const float *J, const float *X, double *epart, int Npad, int Rpad,
                             hipStream_t s, const int32_t *stop = nullptr);
hipError_t launch_best(const StateBufs &b, int nblk, int N, int R, int Rpad, int step,
                       hipStream_t s);
// Cancellation (the stop word of StateBufs): set it to -1; after the sample
// at step m, record m in it if the cancel request (pinned host word) is set;
// finally stop_step[r] (optional) = the step replica r reached (the stop
// word, or its team's entry of tstop [R/32] on the FP4 plan, else k1), and
// bit 2 of status if any replica stopped before k1.
hipError_t launch_stop_init(int32_t *stop, hipStream_t s);
hipError_t launch_poll_cancel(const int32_t *cancel, int32_t *stop, int m, hipStream_t s);
hipError_t launch_output_stop(const int32_t *stop, const int32_t *tstop, int R, int k1,
                              int32_t *stop_step, int32_t *status, hipStream_t s);
hipError_t launch_output(const StateBufs &b, int N, int R, int Rpad, int return_best,
                         int8_t *spins, double *energy, float *x_out, float *y_out,
                         double *best_energy, double *final_energy, int32_t *best_step,
                         hipStream_t s);

}  // namespace hsb
