// Persistent dSB path: FP4 field products, register-resident J and state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace hsb {

struct PersistentJ;     // FP4 J store of one instance plus its run scratch
struct PersistentWork;  // scratch of one persistent run

// One team (32 replicas) of a persistent launch: its instance's FP4 J
// fragments (device), that instance's N and the c0 of eq. (16).
struct FP4Team {
    const void *jpk;
    int N;
    float c0;
};

struct PersistentRun {
    float *X, *Y;          // [Npad][Rpad] state in/out
    const float *gamma;    // [Rpad] per-replica gamma
    int Npad, Rpad, R;
    int k0, k1, Ns, interval;
    float a0, c0, dt;
    double *epart;         // unused by this path (its own partials are kept per sample)
    int local_exchange = 1;  // 0: device-scope exchange even for XCD-local teams
    int tile = 0;            // kernel variant, 0 .. persistent_tiles(variant) - 1
    const int32_t *cancel = nullptr;  // the cancel request (device view of pinned host
                                      // memory), or nullptr: the run cannot stop early
    // dSB only: the Nose-Hoover thermostat (eqs. (6)-(8)) with xi in nh->xi[0 .. Rpad)
    // (its value at k0 in, at the last step out), or nullptr: constant heating
    const NHState *nh = nullptr;
};

bool persistent_supported(int N);
// Number of result-invariant kernel variants of the plan (the autotuner's
// candidates; 0 is the default).
int persistent_tiles(int variant);
int persistent_max_n();
const char *persistent_error();
int persistent_create(const float *J, int N, PersistentJ **out);
void persistent_free(PersistentJ *pj);
// Runs steps k0 .. k1-1 with energy samples, updating the tracking buffers of `b`.
// variant HSB_DSB: field J sgn(x) (exact); HSB_BSB: field J x from base-8 digits of x.
int persistent_run(PersistentJ *pj, int variant, const PersistentRun &run, StateBufs &b, int N,
                   hipStream_t s, KernelTimer &timer);
// The same for a batch: team t owns columns [32 t, 32 t + 32) of the state
// (run.Rpad columns, run.R of them real) and runs the instance host_teams[t];
// every instance has `nkb` K blocks (the same padded size).  Nrows: rows of
// the state decoded into best spins.
int persistent_run_teams(PersistentWork *w, int variant, int nkb, const FP4Team *host_teams,
                         int nteams, const PersistentRun &run, StateBufs &b, int Nrows,
                         hipStream_t s, KernelTimer &timer);
// A dSB run of the FP4 plan (every team on pj's instance, c0 = run.c0) whose
// work buffers are carved from `scratch` (device memory of `bytes` bytes, 256-byte
// aligned) instead of being allocated: nothing is allocated or freed.  The
// samples per launch shrink to what fits; HSB_EINVAL if not even one does.
int persistent_run_in(void *scratch, size_t bytes, const PersistentJ *pj, const PersistentRun &run,
                      StateBufs &b, int Nrows, hipStream_t s);
int persistent_work_create(PersistentWork **out);
void persistent_work_free(PersistentWork *w);
int persistent_nkb(const PersistentJ *pj);
const void *persistent_jpk(const PersistentJ *pj);
// Raised whenever a scratch buffer of the instance's own runs is reallocated or its
// team table re-uploaded: device work queued before depends on the old state.
uint64_t persistent_gen(const PersistentJ *pj);

}  // namespace hsb
