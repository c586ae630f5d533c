// Persistent dSB path: FP4 field products, register-resident J and state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace hsb {

struct PersistentJ;  // FP4 J store plus the path's scratch buffers

struct PersistentRun {
    float *X, *Y;          // [Npad][Rpad] state in/out
    const float *gamma;    // [Rpad] per-replica gamma
    int Npad, Rpad, R;
    int k0, k1, Ns, interval;
    float a0, c0, dt;
    double *epart;         // unused by this path (its own partials are kept per sample)
};

bool persistent_supported(int N);
int persistent_max_n();
const char *persistent_error();
int persistent_create(const float *J, int N, PersistentJ **out);
void persistent_free(PersistentJ *pj);
// Runs steps k0 .. k1-1 with energy samples, updating the tracking buffers of `b`.
int persistent_run(PersistentJ *pj, const PersistentRun &run, StateBufs &b, int N, hipStream_t s,
                   KernelTimer &timer);

}  // namespace hsb
