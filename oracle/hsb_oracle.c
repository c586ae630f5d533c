/*
 * Heated simulated bifurcation -- CPU ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, deliberately
 * unoptimised statement of what the GPU library computes, used by the test
 * suite, by the smoke check and by the benchmark's CPU-baseline leg to check
 * the GPU results.  No product code path may call it.  It shares no code with
 * the GPU library.
 *
 * Paper: T. Kanao and H. Goto, "Simulated bifurcation assisted by thermal
 * fluctuation" (arXiv:2203.08361).
 *
 * What is computed, with the passage each part follows:
 *   - Ising energy E = -1/2 sum_ij J_ij s_i s_j ............ eq. (1)
 *   - cut value C = 1/2 sum_ij w_ij (1 - s_i s_j)/2, w = -J .. eq. (13)
 *   - local field f_i = sum_j J_ij x_j (bSB) ............... eq. (4)
 *                 f_i = sum_j J_ij sgn(x_j) (dSB) .......... eq. (5)
 *   - one time step of heated SB (Methods):
 *       y~  = y(t_k) + {-[a0 - a(t_k)] x(t_k) + c0 f} dt ... eq. (16)
 *       x~  = x(t_k) + a0 y~ dt ............................. eq. (17)
 *       x(t_k+1) = g(x~), y~~ = h(x~, y~) ................... eqs. (18)-(21)
 *       y(t_k+1) = y~~ + gamma y(t_k) dt .................... eq. (22)
 *     gamma = 0 is the unheated bSB/dSB of the same equations.
 *   - pump a(t) raised linearly from 0 to a0 (Results, after eq. (11)),
 *     sampled at t_k: a(t_k) = a0 k / Ns.
 *   - readout s_i = sgn(x_i) (Results, after eq. (5)); the energy is sampled
 *     every `interval` steps and the best sample is kept (Results, K2000
 *     trials: evaluation every 100 steps, best value output); interval = Ns
 *     evaluates the last step only (Results, 700-spin instances).
 *   - instantaneous temperature T_inst = (1/N) sum_i y_i^2 ... eq. (9)
 *   - the Nose-Hoover thermostat that heated SB is derived from (eqs. (6)-(8)):
 *     the heating rate of eq. (22) is -xi, a variable of each run, with
 *       xi(t_k+1) = xi(t_k) + (dt / M) (sum_i y_i(t_k)^2 - N T)
 *     (explicit Euler on eq. (8), with the state at t_k as in eq. (22)); xi
 *     starts at -gamma (or a given value; gamma rounded to float in the FP32
 *     mirror).  1/M = 0 keeps xi = -gamma, which is heated SB itself.
 *   - exhaustive ground state for small N (brute force over 2^N states).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   sgn(0) = +1 (also for -0.0); the wall test is strict |x~| > 1; the heating
 *   term uses the OLD y(t_k); a(t_k) = a0 k / Ns for k = 0 .. Ns-1.
 *
 * Two precisions:
 *   precision 0 (FP64): every quantity in double, textbook evaluation order.
 *   precision 1 (FP32 mirror): the state is single precision, which is the
 *     precision the Methods section states for the variables.  The field is
 *     summed in double and rounded once to float (exact for integer J with
 *     dSB).  The update is evaluated as
 *       u = fmaf(-p, x, c0*f); y~ = fmaf(u, dt, y); x~ = fmaf(a0dt, y~, x);
 *       y(t_k+1) = fmaf(gdt, y, y~~)
 *     with p = a0 - a_k, a_k = (a0*k)/Ns, a0dt = a0*dt, gdt = gamma*dt, all
 *     rounded to float.  The paper fixes no rounding order; this one keeps
 *     the paper's grouping of eqs. (16), (17) and (22).
 *
 * Initial state: x_i, y_i uniform in the open interval (-amp, amp) (Results,
 * paragraph after eq. (12), with amp = 1; the workloads here use amp = 0.1),
 * drawn from the counter-based generator built on the SplitMix64 output mixer
 * (Steele, Lea and Flood, OOPSLA 2014):
 *   key(seed, stream, a, b) = mix(mix(mix(seed + G(stream+1)) + G(a+1)) + G(b+1))
 *   v = (2m + 1 - 2^24) 2^-24 with m = key >> 40;  x0 = fl32(amp * v)
 * with stream 0 for x and 1 for y, a = replica index, b = spin index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_GOLDEN 0x9E3779B97F4A7C15ULL

/* ---------------------------------------------------------------- RNG --- */

static uint64_t orc_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_key(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b)
{
    uint64_t h = orc_mix(seed + ORC_GOLDEN * (stream + 1));
    h = orc_mix(h + ORC_GOLDEN * (a + 1));
    h = orc_mix(h + ORC_GOLDEN * (b + 1));
    return h;
}

float orc_uniform_open(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b)
{
    int64_t m = (int64_t)(orc_key(seed, stream, a, b) >> 40);
    double v = (double)(2 * m + 1 - (1LL << 24)) * (1.0 / 16777216.0);
    return (float)v; /* exact: |2m+1-2^24| < 2^24 */
}

/* x0[r*N + i] for replicas r0 .. r0+R-1 (replica-major layout). */
void orc_init_state(uint64_t seed, int r0, int R, int N, float amp, float *x0, float *y0)
{
    for (int r = 0; r < R; ++r)
        for (int i = 0; i < N; ++i) {
            x0[(size_t)r * N + i] = amp * orc_uniform_open(seed, 0, (uint64_t)(r0 + r), (uint64_t)i);
            y0[(size_t)r * N + i] = amp * orc_uniform_open(seed, 1, (uint64_t)(r0 + r), (uint64_t)i);
        }
}

/* ------------------------------------------------------- definitions --- */

static int orc_sgn(double x) { return x >= 0.0 ? 1 : -1; } /* sgn(0) = +1 */

/* eq. (1) */
double orc_energy(int N, const double *J, const int8_t *s)
{
    double e = 0.0;
    for (int i = 0; i < N; ++i) {
        double row = 0.0;
        for (int j = 0; j < N; ++j)
            row += J[(size_t)i * N + j] * (double)s[j];
        e += (double)s[i] * row;
    }
    return -0.5 * e;
}

/* eq. (13), written with the weights w_ij = -J_ij directly (not via eq. (14)). */
double orc_cut(int N, const double *J, const int8_t *s)
{
    double c = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double w = -J[(size_t)i * N + j];
            c += w * (1.0 - (double)s[i] * (double)s[j]) / 2.0;
        }
    return 0.5 * c;
}

/* Exhaustive minimum of eq. (1) over all 2^N spin states (state m has
 * s_i = -1 iff bit i of m is set).  Returns E_min; s_out gets the first
 * minimiser in enumeration order; *n_min the number of minimisers. */
double orc_brute_force(int N, const double *J, int8_t *s_out, long long *n_min)
{
    if (N < 1 || N > 26) return NAN;
    int8_t *s = (int8_t *)malloc((size_t)N);
    double best = INFINITY;
    long long count = 0;
    for (uint64_t m = 0; m < (1ULL << N); ++m) {
        for (int i = 0; i < N; ++i) s[i] = ((m >> i) & 1ULL) ? -1 : 1;
        double e = orc_energy(N, J, s);
        if (e < best) {
            best = e;
            count = 1;
            if (s_out) memcpy(s_out, s, (size_t)N);
        } else if (e == best) {
            ++count;
        }
    }
    free(s);
    if (n_min) *n_min = count;
    return best;
}

/* eqs. (4) / (5) for one replica, FP64. */
void orc_field(int N, const double *J, const double *x, int variant, double *f)
{
    for (int i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int j = 0; j < N; ++j) {
            double b = variant == 1 ? (double)orc_sgn(x[j]) : x[j];
            acc += J[(size_t)i * N + j] * b;
        }
        f[i] = acc;
    }
}

/* g and h of the Methods section, eqs. (20)-(21). */
static double orc_g(double x) { return x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x); }
static double orc_h(double x, double y) { return fabs(x) > 1.0 ? 0.0 : y; }

/* One step of eqs. (16)-(22) for one replica in FP64, given its field f
 * (computed from x(t_k)).  p = a0 - a(t_k). */
void orc_update64(int N, const double *f, double p, double a0, double c0, double dt, double gamma,
                  double *x, double *y)
{
    for (int i = 0; i < N; ++i) {
        double xk = x[i], yk = y[i];
        double yt = yk + (-p * xk + c0 * f[i]) * dt;   /* eq. (16) */
        double xt = xk + a0 * yt * dt;                  /* eq. (17) */
        double x1 = orc_g(xt);                          /* eq. (18) */
        double ytt = orc_h(xt, yt);                     /* eq. (19) */
        x[i] = x1;
        y[i] = ytt + gamma * yk * dt;                   /* eq. (22), old y */
    }
}

/* The same step with single-precision state (the FP32 mirror). */
void orc_update32(int N, const double *f, float p, float a0, float c0, float dt, float gamma,
                  float *x, float *y)
{
    float a0dt = a0 * dt, gdt = gamma * dt;
    for (int i = 0; i < N; ++i) {
        float xk = x[i], yk = y[i];
        float fi = (float)f[i];
        float u = fmaf(-p, xk, c0 * fi);
        float yt = fmaf(u, dt, yk);                     /* eq. (16) */
        float xt = fmaf(a0dt, yt, xk);                  /* eq. (17) */
        int wall = fabsf(xt) > 1.0f;
        float x1 = wall ? (xt > 0.0f ? 1.0f : -1.0f) : xt; /* eq. (18) */
        float ytt = wall ? 0.0f : yt;                   /* eq. (19) */
        x[i] = x1;
        y[i] = fmaf(gdt, yk, ytt);                      /* eq. (22), old y */
    }
}

/* -------------------------------------------------------------- runs --- */

typedef struct {
    int32_t N, R, steps, variant;       /* variant 0 = bSB, 1 = dSB */
    int32_t interval, precision;        /* precision 0 = FP64, 1 = FP32 mirror */
    int32_t return_best;
    int32_t start_step;                 /* k0: first step index (resumed runs); 0 normally */
    int32_t schedule_steps;             /* Ns of a(t_k) = a0 k / Ns; 0 means start_step + steps */
    int32_t thermostat;                 /* 0: heating at rate gamma; 1: Nose-Hoover xi */
    double a0, c0, dt, gamma;
    const double *gamma_rep;            /* optional per-replica gamma [R] */
    double nh_inv_mass, nh_temperature; /* 1/M >= 0 and T of eq. (8) (thermostat 1) */
    const double *xi0;                  /* optional [R] initial xi (default -gamma) */
} orc_params;

typedef struct {
    double *x, *y;          /* [R][N] final state (optional) */
    int8_t *spins;          /* [R][N] best or final spins (optional) */
    double *energy;         /* [R] energy of `spins` (optional) */
    double *best_e;         /* [R] (optional) */
    double *final_e;        /* [R] (optional) */
    int32_t *best_step;     /* [R] step count of the best sample (optional) */
    double *trace_e;        /* [n_samples][R] energy at each sample (optional) */
    double *trace_tinst;    /* [n_samples][R] T_inst at each sample (optional) */
    double *xi;             /* [R] xi after the last step (thermostat 1, optional) */
} orc_outputs;

/* Sample points of a run over steps k0 .. k1-1: step counts m in (k0, k1]
 * with m % interval == 0, plus m = k1 (which is m = k0 when no step runs). */
int orc_num_samples_range(int k0, int k1, int interval)
{
    int n = k1 / interval - k0 / interval;
    if (k1 == k0 || k1 % interval) ++n;
    return n;
}

int orc_num_samples(int steps, int interval) { return orc_num_samples_range(0, steps, interval); }

static int is_sample(int m, int k0, int k1, int interval)
{
    return (m == k1) || (m > k0 && m % interval == 0);
}

int orc_run(const orc_params *P, const double *J, const float *x0, const float *y0, orc_outputs *O)
{
    const int N = P->N, R = P->R;
    const int k0 = P->start_step, k1 = P->start_step + P->steps;
    const int Ns = P->schedule_steps > 0 ? P->schedule_steps : k1;
    if (N < 1 || R < 1 || P->steps < 0 || k0 < 0 || P->interval < 1 || Ns < k1) return -1;
    if (P->thermostat != 0 && P->thermostat != 1) return -1;
    if (P->thermostat == 1 && !(P->nh_inv_mass >= 0.0 && P->nh_temperature >= 0.0)) return -1;

    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < R; ++r) {
        double *f = (double *)malloc(sizeof(double) * (size_t)N);
        double *xd = (double *)malloc(sizeof(double) * (size_t)N);
        double *yd = (double *)malloc(sizeof(double) * (size_t)N);
        float *xf = (float *)malloc(sizeof(float) * (size_t)N);
        float *yf = (float *)malloc(sizeof(float) * (size_t)N);
        int8_t *s = (int8_t *)malloc((size_t)N);
        int8_t *best_s = (int8_t *)malloc((size_t)N);
        const double gamma = P->gamma_rep ? P->gamma_rep[r] : P->gamma;
        for (int i = 0; i < N; ++i) {
            xf[i] = x0[(size_t)r * N + i];
            yf[i] = y0[(size_t)r * N + i];
            xd[i] = xf[i];
            yd[i] = yf[i];
        }
        double best = INFINITY, last = NAN;
        int best_m = -1, sample = 0;
        /* Nose-Hoover variable (thermostat 1); the FP32 mirror holds gamma as a
         * float, as its heated step does */
        double xi = P->xi0 ? P->xi0[r] : -(P->precision == 1 ? (double)(float)gamma : gamma);
        for (int m = k0; m <= k1; ++m) {
            /* state after m steps is in (xd,yd) or (xf,yf) */
            if (is_sample(m, k0, k1, P->interval)) {
                const int is32 = P->precision == 1;
                double t = 0.0;
                for (int i = 0; i < N; ++i) {
                    double xi = is32 ? (double)xf[i] : xd[i];
                    double yi = is32 ? (double)yf[i] : yd[i];
                    s[i] = (int8_t)orc_sgn(xi);
                    t += yi * yi;
                }
                double e = orc_energy(N, J, s);
                if (O->trace_e) O->trace_e[(size_t)sample * R + r] = e;
                if (O->trace_tinst) O->trace_tinst[(size_t)sample * R + r] = t / N; /* eq. (9) */
                ++sample;
                if (e < best) { /* strict: ties keep the earliest sample */
                    best = e;
                    best_m = m;
                    memcpy(best_s, s, (size_t)N);
                }
                last = e;
            }
            if (m == k1) break;
            /* heating rate of this step: gamma, or -xi(t_k) under the thermostat,
             * whose xi(t_k+1) integrates sum_i y_i(t_k)^2 (eq. (8)) */
            double rate = gamma, sum_y2 = 0.0;
            if (P->thermostat == 1) {
                rate = -xi;
                for (int i = 0; i < N; ++i) {
                    double yi = P->precision == 1 ? (double)yf[i] : yd[i];
                    sum_y2 += yi * yi;
                }
            }
            if (P->precision == 1) {
                /* a(t_k) as a float: (a0*k)/Ns; p = a0 - a(t_k) */
                float a0f = (float)P->a0;
                float ak = (a0f * (float)m) / (float)Ns;
                float p = a0f - ak;
                for (int i = 0; i < N; ++i) xd[i] = xf[i];
                orc_field(N, J, xd, P->variant, f);
                orc_update32(N, f, p, a0f, (float)P->c0, (float)P->dt, (float)rate, xf, yf);
            } else {
                double p = P->a0 - P->a0 * (double)m / (double)Ns;
                orc_field(N, J, xd, P->variant, f);
                orc_update64(N, f, p, P->a0, P->c0, P->dt, rate, xd, yd);
            }
            if (P->thermostat == 1) {
                /* dt as the step used it: a float in the FP32 mirror */
                const double dt = P->precision == 1 ? (double)(float)P->dt : P->dt;
                xi = xi + dt * P->nh_inv_mass * (sum_y2 - (double)N * P->nh_temperature);
            }
        }
        (void)sample;
        for (int i = 0; i < N; ++i) {
            double xi = P->precision == 1 ? (double)xf[i] : xd[i];
            double yi = P->precision == 1 ? (double)yf[i] : yd[i];
            if (O->x) O->x[(size_t)r * N + i] = xi;
            if (O->y) O->y[(size_t)r * N + i] = yi;
            s[i] = (int8_t)orc_sgn(xi);
        }
        if (O->best_e) O->best_e[r] = best;
        if (O->final_e) O->final_e[r] = last;
        if (O->best_step) O->best_step[r] = best_m;
        if (O->xi) O->xi[r] = xi;
        if (O->spins) memcpy(O->spins + (size_t)r * N, P->return_best ? best_s : s, (size_t)N);
        if (O->energy) O->energy[r] = P->return_best ? best : last;
        if (!isfinite(last)) {
#pragma omp atomic write
            rc = -4;
        }
        free(f); free(xd); free(yd); free(xf); free(yf); free(s); free(best_s);
    }
    return rc;
}
