/*
 * hsb.h -- C ABI of libhsb: heated simulated bifurcation on one AMD MI355X (gfx950).
 *
 * The library integrates many independent replicas of heated ballistic SB
 * (HbSB) and heated discrete SB (HdSB) on a dense all-to-all Ising problem
 * (T. Kanao and H. Goto, "Simulated bifurcation assisted by thermal
 * fluctuation", arXiv:2203.08361):
 *
 *   problem   find s in {-1,+1}^N minimising E = -1/2 sum_ij J_ij s_i s_j     eq. (1)
 *             with J symmetric and J_ii = 0
 *   field     f = J x (bSB, eq. (4))  or  f = J sgn(x) (dSB, eq. (5))
 *   step      y~ = y + {-[a0 - a(t_k)] x + c0 f} dt                          eq. (16)
 *             x~ = x + a0 y~ dt                                             eq. (17)
 *             x' = g(x~), y~~ = h(x~, y~)  (perfectly inelastic walls)        eqs. (18)-(21)
 *             y' = y~~ + gamma y dt        (heating with the OLD y)          eq. (22)
 *   pump      a(t_k) = a0 k / Ns, linear from 0 to a0 over the run (Results, after eq. (11))
 *   readout   s = sgn(x) with sgn(0) = +1 (Results, after eq. (5)); the energy
 *             is sampled every `energy_interval` steps and at the last step, and
 *             the best sample is returned (Results, K2000 protocol)
 *   init      x_i, y_i uniform in the open interval (-amp, amp) (Results, after
 *             eq. (12) with amp = 1; the library default is amp = 0.1), drawn
 *             from a counter-based generator: SplitMix64's output mixer
 *             (Steele, Lea, Flood 2014) chained over (seed, stream, replica, spin)
 *
 * gamma = 0 gives the unheated bSB / dSB of the same equations.
 *
 * Conventions common to every entry point
 *   - Every function returns an hsb_status; on failure hsb_last_error() holds
 *     a message for the calling thread.  HSB_EINVAL is returned before any
 *     device work is queued and nothing is written to any output.
 *   - Matrices are row-major.  Spin/state arrays are replica-major:
 *     element (r, i) of an [R][N] array is at offset r*N + i.
 *   - Determinism: the same (J, arguments, seed, options) give bitwise the same
 *     outputs.  Replica r depends only on (seed, r): its result is the same for
 *     any R, apart from the effect of the precision plan on bSB (below).
 *   - Precision: the state x, y is single precision (Methods, last sentence).
 *     For dSB with integer-valued J the field is an exact integer, so the
 *     trajectory is bitwise the same whichever plan runs it.  For bSB the
 *     field is rounded differently by each plan (FP32 sums of FP32 products,
 *     or the exactly rounded sum of the integer-digit plan); see
 *     hsb_set_option(HSB_OPT_PRECISION).
 *   - Thread safety: one context may be used by one thread at a time.
 *   - Sharing the GPU: the persistent kernels (the FP4 plan, batch queues and
 *     the digit plan's segments) need every workgroup of a launch resident at
 *     once, and size their grids for an otherwise idle device.  Runs of other
 *     contexts or processes executing at the same time can keep part of a
 *     launch from being scheduled; every wait inside these kernels is bounded,
 *     so such a run then ends with HSB_EDEVICE (after at most a few seconds)
 *     rather than hanging.  Run one persistent run per GPU at a time.
 */
#ifndef HSB_H
#define HSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsb_ctx hsb_ctx; /* opaque; owns the device copies of J */

typedef enum {
    HSB_BSB = 0, /* ballistic SB, field eq. (4) */
    HSB_DSB = 1  /* discrete SB, field eq. (5) */
} hsb_variant;

typedef enum {
    HSB_OK = 0,
    HSB_EINVAL = -1,      /* invalid argument; nothing was written */
    HSB_ENOMEM = -2,      /* device allocation failed */
    HSB_EDEVICE = -3,     /* HIP runtime error or no usable gfx950 device */
    HSB_ENUMERIC = -4,    /* a replica's state became non-finite; its energy is NaN,
                             all other outputs are valid */
    HSB_ECANCELED = -5,   /* the run was stopped by hsb_cancel at a sample point; the
                             outputs hold the state and samples up to where each replica
                             stopped (hsb_run_args.stop_step) */
    HSB_EUNSUPPORTED = -6 /* a requested precision plan cannot run this problem */
} hsb_status;

typedef enum {
    HSB_OPT_INIT_AMP = 0,        /* amplitude of the uniform initial x, y; default 0.1, > 0 */
    HSB_OPT_ENERGY_INTERVAL = 1, /* energy sampled every this many steps (and at the end);
                                    default 100, >= 1 */
    HSB_OPT_RETURN_BEST = 2,     /* 1 (default): return the best sampled spins and energy;
                                    0: return the final state's */
    HSB_OPT_PRECISION = 3,       /* hsb_precision; default HSB_PREC_AUTO */
    HSB_OPT_TIMING = 4,          /* 1: bracket the launches of the dominant kernel (the
                                    field+update kernel of the plan) with HIP events on the
                                    run's stream, one bracket per run of consecutive
                                    launches between two energy samples; default 0 */
    HSB_OPT_KERNEL_MS = 5,       /* read only: summed bracketed time (ms) of the last run with
                                    timing on (synchronises the events) */
    HSB_OPT_KERNEL_LAUNCHES = 6, /* read only: number of launches inside those brackets */
    HSB_OPT_LAST_PLAN = 7,       /* read only: plan of the last successful run, an hsb_plan */
    HSB_OPT_LOCAL_EXCHANGE = 8,  /* FP4 plan and the digit plan's persistent kernel: 1
                                    (default): a team of workgroups that share
                                    one XCD exchanges its per-step data through that XCD's L2
                                    (workgroup-scope stores, no cache invalidation); 0: always
                                    device scope (slower; results are the same).  Batches use
                                    the option of their first context. */
    HSB_OPT_GRAPH = 9,           /* 1 (default): hsb_run_ex / hsb_run on the FP4 plan (dSB;
                                    bSB from a seeded start state with INIT_AMP <= 1) keep a
                                    HIP graph of the last repeated run.  The first call
                                    with given arguments, options and buffers runs as usual;
                                    the next identical call captures its queued work into a
                                    graph (on a stream of the context, ordered after and
                                    before the caller's stream by events) and launches it;
                                    later identical calls launch the graph again.  Results
                                    are those of the eager run.  Any other call on the
                                    context, or one that reallocates a buffer the graph uses,
                                    drops the graph.  Not used while timing is on or while
                                    the caller's stream is being captured.  0: always eager */
    HSB_OPT_GRAPH_LAUNCHES = 10, /* read only: runs of this context served by a graph launch */
    HSB_OPT_AUTOTUNE = 11,       /* 1: pick the kernel variant of each run (hsb_run_ex, and the
                                    queue placement of batches led by this context) from an
                                    on-disk cache, timing every variant on the first 200
                                    steps of the run's own shape the first time a (plan,
                                    variant, padded N, padded R, J kind, thermostat) shape
                                    is seen and storing the fastest.  The variants give
                                    bitwise the same results; only the time differs.  The
                                    cache file is $HSB_TUNE_CACHE, else
                                    $XDG_CACHE_HOME/hsb/tune.txt, else
                                    $HOME/.cache/hsb/tune.txt.  0 (default): variant 0 */
    HSB_OPT_TILE = 12,           /* -1 (default): variant from AUTOTUNE (else 0); k >= 0: force
                                    variant k.  FP4 dSB: 0..2 = operand read 2, 1, 4 K blocks
                                    ahead of the products; FP4 bSB: 0..1 = 4, 2 fragments
                                    ahead; DIGITS: 0..1 = one persistent launch per
                                    segment between sample points with the default wave
                                    height of the digit combination or the other one (32 or
                                    64 rows: two or one workgroups per CU), 2..3 = one launch
                                    per step with those heights; batch queues: 0..1 =
                                    longest-first, round robin.  A variant the plan lacks:
                                    HSB_EINVAL */
    HSB_OPT_LAST_TILE = 13,      /* read only: the variant of the last successful run */
    HSB_OPT_CANCELLABLE = 14     /* 1: runs of this context (hsb_run, hsb_run_ex,
                                    hsb_run_ex_noalloc) can be stopped by hsb_cancel; the
                                    FP4 plan then runs its dSB kernel's cancellable
                                    variant, about 6% slower at N = 2000 (its request
                                    checks change the step's instruction schedule).
                                    0 (default): hsb_cancel returns HSB_EINVAL for this
                                    context and every plan runs without the checks */
} hsb_option;

typedef enum {
    HSB_PREC_AUTO = 0,  /* the FP4 plan where MIXED takes it; the digit plan for bSB and
                           for dSB with integer J in [-127, 127]; FP32 otherwise */
    HSB_PREC_FP32 = 1,  /* plain FP32 field products (the baseline form) */
    HSB_PREC_MIXED = 2, /* J exact in FP4 (entries in {0, +-0.5, +-1, +-1.5, +-2, +-3, +-4,
                           +-6}) and N <= 2048: the FP4 plan (dSB exact; bSB from base-8
                           digits of x); otherwise, N <= 16384: the integer-digit plan */
    HSB_PREC_DIGITS = 3, /* the integer-digit plan (N <= 16384) whatever J */
    HSB_PREC_INCREMENTAL = 4 /* dSB with integer J in [-127, 127], N <= 16384: the exact
                                integer field of the current signs is carried from step
                                to step, changed by 2 s_j J[:, j] for each spin j that
                                flipped (never chosen by AUTO; bSB, other J or the
                                thermostat: HSB_EUNSUPPORTED) */
} hsb_precision;

/*
 * Execution plans (HSB_OPT_LAST_PLAN).  The field of eqs. (4)/(5) is
 *   HSB_PLAN_FP32    FP32 matrix-core products, one launch per step;
 *   HSB_PLAN_FP4     FP4 x FP4 products, every step in one persistent launch.
 *                    dSB: exact.  bSB: x as eight base-8 digits in [-4, 3] per
 *                    32-row chunk, weighted by the operand's block scales
 *                    (x to 2^-23 of the chunk's largest |x|), FP32 sums;
 *   HSB_PLAN_DIGITS  int8 products of digits, one launch per step:
 *                    x = rint(x 2^30) 2^-30 as four base-256 digits (exact for
 *                    |x| >= 2^-6), sgn(x) as one digit, J as one digit when every
 *                    entry is an integer in [-127, 127] (then the field is the
 *                    exactly rounded FP32 value of sum_j J_ij x_j) or as four
 *                    digits of a per-row power-of-two scaled J (real J: relative
 *                    error about 2^-31 per entry).  bSB on this plan needs
 *                    |x| <= 1 in the start state (eqs. (18)-(21) keep it so), as
 *                    does bSB on HSB_PLAN_FP4: otherwise MIXED and DIGITS return
 *                    HSB_EUNSUPPORTED and AUTO runs FP32.
 */
typedef enum {
    HSB_PLAN_FP32 = 0,
    HSB_PLAN_FP4 = 1,
    HSB_PLAN_DIGITS = 2,
    HSB_PLAN_INCREMENTAL = 3 /* HSB_PREC_INCREMENTAL: two launches per step, work per
                                step proportional to the number of flipped spins */
} hsb_plan;

/*
 * hsb_create -- validate J and build its device copies (the J store).
 *
 *   J    host pointer, N*N floats, row-major; read only during the call
 *        (the caller keeps ownership and may free it afterwards).
 *   N    number of spins, >= 1.
 *   out  receives the new context.
 *
 * J must be finite, symmetric (J[i*N+j] == J[j*N+i] exactly) and have a zero
 * diagonal (eq. (1)); otherwise HSB_EINVAL.  Uses the current HIP device.
 */
int hsb_create(const float *J, int N, hsb_ctx **out);

/* hsb_destroy -- free the context and all its device memory.  NULL is ignored. */
void hsb_destroy(hsb_ctx *h);

/* hsb_last_error -- message of the last failure on this thread ("" if none). */
const char *hsb_last_error(void);

/*
 * hsb_set_option / hsb_get_option -- run options kept in the context
 * (hsb_option keys).  Invalid key or value: HSB_EINVAL, option unchanged.
 */
int hsb_set_option(hsb_ctx *h, int key, double value);
int hsb_get_option(hsb_ctx *h, int key, double *value);

/*
 * hsb_run -- integrate R replicas for `steps` steps; host outputs.
 *
 *   variant  HSB_BSB or HSB_DSB
 *   a0, c0, dt, gamma  constants of eqs. (10)-(11), (16)-(22); finite, dt > 0,
 *            gamma >= 0 (gamma = 0: unheated).  a(t) rises from 0 to a0 over
 *            the `steps` steps.
 *   steps    Ns >= 0 (0 returns the initial state's spins and energy)
 *   R        number of replicas >= 1
 *   seed     initial-state seed; replica r draws from (seed, r)
 *   spins    host, [R][N] int8, receives +-1 (best sample or final, per
 *            HSB_OPT_RETURN_BEST)
 *   energy   host, [R] double, receives eq. (1) of `spins` (FP64)
 *
 * Returns HSB_ENUMERIC if any replica became non-finite (its energy is NaN).
 */
int hsb_run(hsb_ctx *h, int variant, float a0, float c0, float dt, float gamma, int steps, int R,
            uint64_t seed, int8_t *spins, double *energy);

/*
 * hsb_run_args -- arguments of hsb_run_ex.  All pointers are DEVICE pointers
 * (memory of the context's device), all optional ones may be NULL.  Zero-fill
 * the struct, then set what is needed; `struct_size` must be
 * sizeof(hsb_run_args).
 */
typedef struct {
    size_t struct_size;
    int32_t variant;        /* HSB_BSB / HSB_DSB */
    int32_t steps;          /* steps to run in this call, >= 0 */
    int32_t R;              /* replicas, >= 1 */
    int32_t start_step;     /* first step index k0 of this call, >= 0 (resume) */
    int32_t schedule_steps; /* Ns defining a(t_k) = a0 k / Ns; 0 means start_step + steps */
    int32_t thermostat;     /* hsb_thermostat: HSB_THERMO_HEAT (0, the zero fill) or
                               HSB_THERMO_NOSE_HOOVER */
    float a0, c0, dt, gamma;
    uint64_t seed;
    const float *gamma_rep; /* optional [R] per-replica gamma (overrides gamma) */
    const float *x0, *y0;   /* optional [R][N] initial state (both or neither);
                               default: seeded draw */
    float *x_out, *y_out;   /* optional [R][N] final state */
    int8_t *spins;          /* [R][N] best or final spins (required) */
    double *energy;         /* [R] energy of `spins` (required) */
    double *best_energy;    /* optional [R] best sampled energy */
    double *final_energy;   /* optional [R] energy of the final state */
    int32_t *best_step;     /* optional [R] step count of the best sample */
    void *stream;           /* hipStream_t; NULL = the null stream */
    double *trace_energy;   /* optional [n_samples][R]: eq. (1) of sgn(x) at every sample
                               point of the call, in step order (hsb_num_samples) */
    double *trace_tinst;    /* optional [n_samples][R]: the instantaneous temperature
                               T_inst = (1/N) sum_i y_i^2 of eq. (9) at the same points,
                               summed in FP64 */
    /* HSB_THERMO_NOSE_HOOVER only (must be 0 / NULL otherwise): */
    double nh_inv_mass;     /* 1/M >= 0 of eq. (8), finite; 0 keeps xi constant */
    double nh_temperature;  /* T >= 0 of eq. (8), finite */
    const double *xi0;      /* optional [R] xi at start_step; default -gamma (per replica) */
    double *xi_out;         /* optional [R] xi after the last step (to resume) */
    int32_t *stop_step;     /* optional [R]: the step count each replica reached:
                               start_step + steps, or where hsb_cancel stopped it */
} hsb_run_args;

/*
 * hsb_thermostat -- what drives the heating term of eq. (22).
 *
 *   HSB_THERMO_HEAT         the constant rate gamma (per replica with gamma_rep):
 *                           heated SB, eqs. (10)-(11) and (16)-(22).
 *   HSB_THERMO_NOSE_HOOVER  the Nose-Hoover thermostat that heated SB comes from,
 *                           eqs. (6)-(8): every replica carries xi (FP64); step k
 *                           heats at the rate -xi(t_k) (rounded to float, in
 *                           eq. (22)'s place) and then
 *                             xi(t_k+1) = xi(t_k) + (dt/M)(sum_i y_i(t_k)^2 - N T),
 *                           explicit Euler on eq. (8) with the state before the
 *                           step.  xi starts at -gamma, so 1/M = 0 is exactly
 *                           heated SB.  The sum over all spins is formed every
 *                           step in FP64 from per-wave partials in a fixed
 *                           order.  Every plan runs it; on the FP4 plan inside
 *                           the persistent kernels (dSB: each workgroup's
 *                           partial is exchanged with the sign words; bSB: each
 *                           wave's partial travels with its digits).  In a
 *                           context with HSB_OPT_CANCELLABLE = 1, bSB thermostat
 *                           runs that would take the FP4 plan take the
 *                           integer-digit plan (the FP4 bSB kernel's thermostat
 *                           variant takes no cancel requests).
 */
typedef enum { HSB_THERMO_HEAT = 0, HSB_THERMO_NOSE_HOOVER = 1 } hsb_thermostat;

/*
 * hsb_run_ex -- hsb_run with device buffers, a caller stream, per-replica gamma,
 * a caller initial state and resumable scheduling.  Work is queued on
 * `stream`; the call returns after queuing except that it synchronises the
 * stream to report HSB_ENUMERIC.  Sample points are step counts m with
 * start_step < m <= start_step + steps and m % energy_interval == 0, plus the
 * state after the last step of the call (and the initial state when steps = 0).
 * The traces, if given, receive the energy and T_inst of every sample point;
 * the entries of a replica that became non-finite are unspecified.
 */
int hsb_run_ex(hsb_ctx *h, const hsb_run_args *args);

/*
 * hsb_cancel -- ask the run in progress on h (hsb_run, hsb_run_ex,
 * hsb_run_ex_noalloc) to stop early.  Callable from any thread at any time; it
 * only sets a request word that the device reads.
 *
 * The run stops at a sample point: a step count m, start_step < m <
 * start_step + steps, that is a multiple of HSB_OPT_ENERGY_INTERVAL.
 *   - Per-step plans (FP32, DIGITS, INCREMENTAL): the request is read after
 *     each sample; the first sample point at which it is seen is where every
 *     replica stops.
 *   - FP4 plan: the replicas of each 32-replica team stop together at the
 *     first sample point after the team's first wave has seen the request
 *     (it reads the request at the start of the launch and at each sample
 *     point); different teams may stop at different sample points.
 * A stopped replica's outputs are those of a run of that many steps: its
 * state (x_out, y_out), its samples up to the stop (energy, best and final
 * energies, best step, traces; later trace rows are unspecified), and xi.
 * stop_step[r] receives the step count replica r reached, and the run
 * returns HSB_ECANCELED (before HSB_ENUMERIC) if any replica stopped early.
 * A run resumes from there with x0 = x_out, y0 = y_out, start_step = the stop
 * step, and the same schedule_steps.
 *
 * The request belongs to the context's next or current run and is cleared
 * when that run returns, whether or not it stopped the run (a request that
 * arrives after the run's last sample point has no effect).  Batches
 * (hsb_run_batch) are not cancelled.  Only a context with
 * HSB_OPT_CANCELLABLE = 1 takes requests; on others, and for NULL, HSB_EINVAL.
 */
int hsb_cancel(hsb_ctx *h);

/*
 * hsb_run_ex_noalloc -- hsb_run_ex for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  It runs what hsb_run_ex runs on the FP4 plan and gives
 * bitwise the same outputs, but every buffer of the run besides the caller's
 * inputs and outputs (the state x, y, the exchange words, the sample
 * snapshots and energies, the best-sample tracking) lives in one fixed array
 * of HSB_NOALLOC_SCRATCH_BYTES per device, which the library holds from its
 * first context on that device until the process ends.  No hipMalloc,
 * hipFree, host-pinned allocation, event, stream or graph is created.
 *
 *   h, args  as for hsb_run_ex (device pointers, the caller's stream).
 *
 * Scope: dSB (HSB_DSB) on the FP4 plan, i.e. J exact in FP4 with N <= 2048 and
 * precision AUTO or MIXED (the FP4 J store is built by hsb_create); constant
 * heating (HSB_THERMO_HEAT), no traces.  Otherwise HSB_EUNSUPPORTED.  A run
 * whose state (about 18 (N rounded up to 64) bytes per replica, R rounded up to
 * 64) does not fit, together with the exchange words and at least one sample,
 * returns HSB_EINVAL before any device work: at N = 2000 up to about 3000
 * replicas fit.  Longer runs take more launches (fewer samples per launch);
 * the results are the same.  The timing options are ignored.
 *
 * Every call on a device shares that device's array and leaves its contents
 * behind: each call initialises what it reads.  Calls that overlap on one
 * device (from several threads or on several streams) race on the array and
 * must be serialised by the caller.
 */
#define HSB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hsb_run_ex_noalloc(hsb_ctx *h, const hsb_run_args *args);

/*
 * hsb_num_samples -- number of sample points of a call of hsb_run_ex with this
 * start_step and steps under the context's HSB_OPT_ENERGY_INTERVAL I: the
 * multiples of I in (start_step, start_step + steps], plus the last state if
 * it is not one of them (the initial state when steps = 0).  This is the
 * leading dimension of trace_energy and trace_tinst; row j is the j-th sample
 * point in step order.  start_step, steps >= 0, else HSB_EINVAL.
 */
int hsb_num_samples(hsb_ctx *h, int start_step, int steps, int *n);

/*
 * hsb_plan_info -- the precision plan AUTO (or the forced option) would use
 * for `variant` on this J: HSB_PREC_FP32, HSB_PREC_MIXED or HSB_PREC_INCREMENTAL.
 */
int hsb_plan_info(hsb_ctx *h, int variant, int *precision);

/*
 * hsb_run_batch -- many independent runs ("jobs") over several instances in
 * one call: the parameter sweeps and instance sets of the Results section
 * (each job is a set of trials of one instance at one heating rate).
 *
 *   hs      n_inst contexts (the instances), all on the current device
 *   jobs    n_jobs job descriptions (host array); job j runs jobs[j].R replicas
 *           of instance hs[jobs[j].instance] with its own c0, gamma and seed
 *   args    what all jobs share: variant, steps (Ns), a0, dt, initial
 *           amplitude, energy interval, best/final output, stream
 *
 * Job j gives exactly what hsb_run_ex on its instance gives with the same
 * variant, steps, R, a0, c0, dt, gamma and seed (and the batch's amplitude,
 * interval and return mode), under the plan its instance's precision option
 * selects.  Jobs on the FP4 plan (J exact in FP4 with N <= 2048; for bSB also
 * initial amplitude <= 1) run together:
 *   dSB  all of them in ONE persistent launch (scheduler HSB_SCHED_QUEUE, the
 *        default): every 32 replicas of a job form a team; the teams are
 *        placed longest-first on eight device job queues (one per XCD slot,
 *        balanced by workgroups x estimated step time), and the resident
 *        workgroups take a team's parts from their queue until it is empty.
 *        The initial state, the energy samples of eq. (1) and the best sample
 *        are formed inside that launch.  A batch identical to the previous one
 *        of the same lead context hs[0] (same jobs, arguments and buffers) is
 *        captured and replayed as one HIP graph, as hsb_run_ex does under
 *        HSB_OPT_GRAPH of hs[0].  HSB_SCHED_CLASSES runs them as bSB does;
 *   bSB  one persistent launch sequence per padded size for all their
 *        instances, so a batch of small instances fills the device.
 * Other jobs run one after another.
 * Outputs are device pointers owned by the caller: jobs[j].spins [R][N] int8
 * and jobs[j].energy [R] double.  Validation failures return HSB_EINVAL before
 * any device work; HSB_ENUMERIC if any replica of any job became non-finite.
 * Contexts' own options (amplitude, interval, return mode) are not changed.
 * Jobs run heated SB at their constant rate (HSB_THERMO_HEAT) and give no
 * traces; runs with the thermostat or traces go through hsb_run_ex.
 */
typedef struct {
    int32_t instance; /* index into hs[] */
    int32_t R;        /* replicas, >= 1 */
    float c0;         /* c0 of eq. (16) for this job, finite */
    float gamma;      /* heating rate of every replica of the job, finite, >= 0 */
    uint64_t seed;    /* replica r of the job draws its initial state from (seed, r) */
    int8_t *spins;    /* device, [R][N of the instance], receives +-1 */
    double *energy;   /* device, [R], receives eq. (1) of spins */
} hsb_job;

typedef struct {
    size_t struct_size;      /* sizeof(hsb_batch_args) */
    int32_t variant;         /* HSB_BSB / HSB_DSB */
    int32_t steps;           /* Ns >= 0 for every job */
    float a0, dt;            /* finite, dt > 0 */
    double init_amp;         /* > 0 (0 means 0.1) */
    int32_t energy_interval; /* >= 1 (0 means 100) */
    int32_t return_best;     /* 1: best sample, 0: final state */
    void *stream;            /* hipStream_t, or NULL for the null stream */
    int32_t scheduler;       /* hsb_scheduler of the dSB jobs on the FP4 plan */
} hsb_batch_args;

typedef enum {
    HSB_SCHED_QUEUE = 0,   /* one persistent launch fed by job queues (default) */
    HSB_SCHED_CLASSES = 1  /* one launch sequence per padded size, one class after another */
} hsb_scheduler;

int hsb_run_batch(hsb_ctx *const *hs, int n_inst, const hsb_job *jobs, int n_jobs,
                  const hsb_batch_args *args);

#ifdef __cplusplus
}
#endif

#endif /* HSB_H */
