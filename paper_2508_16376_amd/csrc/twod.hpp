// Two-dimensional fault simulation: light faults one per lane, heavy faults
// split structurally across a wavefront, both fed by a persistent work queue.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <string>

#include "kernels.hpp"
#include "riros.h"

namespace riros {

struct TwoDWorkspace {
    void* mem = nullptr;
    size_t bytes = 0;
    void* ctr = nullptr;   // device counters of the last run (error flag at word 5)
};

struct TwoDParams {
    float theta = INFINITY;
    int light_cap = 0;
    int chunk = 0;
    int waves_per_cu = 0;
    int num_cu = 0;
    float monitor_rate = 0.f;   // hand a light fault over above this many events per cycle (0 = never)
};

// Light kernel over the faults whose priority is <= theta (all faults when
// priority is NULL), in descending priority order, then the heavy kernel over
// the faults above theta and the faults the light lanes handed over.
// heavy_ws / heavy_blocks: per-wave workspace of the heavy kernel.
int run_twod(const DevDesign& d, TwoDWorkspace& ws, const GoldenView& gv,
             const riros_fault* faults, const float* priority, uint32_t F, int drop,
             const TwoDParams& p, PlainWorkspace heavy_ws, uint32_t heavy_blocks,
             uint32_t* detect, uint64_t* events, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s,
             std::string& err);

void twod_free(TwoDWorkspace& ws);

}  // namespace riros
