// Host-side handle of one prepared batch launch (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qsv_internal.hpp"

namespace qsv {

struct BatchTraj;
struct BatchItem;
struct ScaleBlock;

struct BatchLaunch {
    void *block = nullptr;          // one device allocation holding every table below
    BatchTraj *trajs = nullptr;
    ScaleBlock *sblocks = nullptr;
    BatchItem *items = nullptr;     // (trajectory, chunk) work items of every depth
    double *partials = nullptr;     // per-chunk FP64 norms of the last sections
    std::vector<uint32_t> depth_off, depth_count;  // items of depth d (host)
    DevSection *secs = nullptr;
    DevPhase *phases = nullptr;
    DevOp *ops = nullptr;
    void *mats = nullptr;
    uint32_t nsblocks = 0, count = 0;
    uint64_t total_amps = 0;
    int r = 0, kmax = 0;
    size_t lds = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void *states = nullptr;
    double *norms = nullptr;
};

// Build the combined tables for these plans, upload them and capture the graph
// (|0> init, one kernel per section depth, norms, rescale).
qsv_status batch_prepare(qsv_dtype dt, int count, const Plan *const *plans,
                         const uint64_t *offsets, void *states, double *norms,
                         BatchLaunch &L, std::string &err);
void batch_release(BatchLaunch &L);
hipError_t batch_replay(const BatchLaunch &L, hipStream_t s);

}  // namespace qsv
