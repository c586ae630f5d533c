// Batched discrete SB on the FP4 plan: every job of a batch in one persistent
// launch fed by per-XCD job queues (host interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "kernels.h"

namespace hsb {

// One team of the queue launch: 32 consecutive replicas of one job, run by
// Npad/128 workgroups of 4 waves (one 32-row chunk of spins per wave).
struct QTeam {
    const void *jpk;   // the instance's FP4 J fragments (persistent_jpk)
    int8_t *spins;     // the job's output [R][N] (device)
    double *energy;    // the job's output [R] (device)
    uint64_t seed;     // replica r of the job draws its initial state from (seed, r)
    int N, nkb;        // instance size and its K blocks of 64 spins (a multiple of 4)
    int rep0, nrep;    // first replica of the job in this team, replicas in it (<= 32)
    float c0, gamma;   // eq. (16) coupling and eq. (22) heating rate of the job
};

// What every job of the launch shares.
struct QRun {
    int steps, interval, return_best;
    float a0, dt, amp;
    int local_exchange;
};

struct QueueWork;  // device tables and exchange buffers, kept between calls

int queue_work_create(QueueWork **out);
void queue_work_free(QueueWork *w);
const char *queue_error();
// Raised whenever a buffer is reallocated or a table re-uploaded: device work
// queued before (a captured graph) depends on the old contents.
uint64_t queue_gen(const QueueWork *w);

// How the teams are spread over the eight queues and ordered in each.
//   policy 0: longest processing time first, each team to the least loaded
//             queue (load = workgroups x estimated step time);
//   policy 1: round robin in job order (for comparison).
// Returns the estimated makespan in workgroup-step units of the fullest queue.
double queue_schedule(const std::vector<QTeam> &teams, int policy, std::vector<uint32_t> &units,
                      std::vector<int> &qoff);

// Queue the launch on s (table uploads only when they changed, then fills, the
// persistent launch and the energy output).  The caller reads the status word
// (queue_status) after synchronising: bit 0 a non-finite replica, bit 1 an
// exchange wait that timed out.
int queue_run(QueueWork *w, const std::vector<QTeam> &teams, const QRun &run, int policy,
              hipStream_t s, KernelTimer &timer);
const int32_t *queue_status(const QueueWork *w);

}  // namespace hsb
