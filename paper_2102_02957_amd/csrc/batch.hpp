// Host-side handle of one prepared batch launch (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "qsv_internal.hpp"

namespace qsv {

struct BatchTraj;
struct BatchTask;
struct ScaleBlock;

struct BatchLaunch {
    void *block = nullptr;          // one device allocation holding every table below
    BatchTraj *trajs = nullptr;
    BatchTask *tasks = nullptr;
    uint32_t *counters = nullptr;   // [0] next task, [1] error flag, [2..] section completions
    double *parts = nullptr;        // per-chunk norm partials of the last sections
    ScaleBlock *sblocks = nullptr;
    DevSection *secs = nullptr;
    DevPhase *phases = nullptr;
    DevOp *ops = nullptr;
    void *mats = nullptr;
    uint32_t ntasks = 0, ncounters = 0, nsblocks = 0, count = 0;
    uint64_t total_amps = 0;
    int r = 0, kmax = 0;
    size_t lds = 0;
    int grid = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void *states = nullptr;
    double *norms = nullptr;
};

// Build the combined tables for these plans, upload them and capture the graph
// (counter reset, |0> init, persistent kernel, norms, rescale).
qsv_status batch_prepare(qsv_dtype dt, int count, const Plan *const *plans,
                         const uint64_t *offsets, void *states, double *norms,
                         BatchLaunch &L, std::string &err, uint32_t spin_limit);
void batch_release(BatchLaunch &L);
hipError_t batch_replay(const BatchLaunch &L, hipStream_t s);

}  // namespace qsv
