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

// Batched campaign: many designs in one persistent launch.  The device tables
// td/tg hold each design's image and golden views; did[f] is fault f's design,
// off[k]..off[k+1] design k's fault range in the concatenated list.
struct BatchPlan {
    uint32_t n = 0, F = 0;
    const DevDesign* td = nullptr;
    const GoldenView* tg = nullptr;
    DevDesign td_host0{};     // unused by the table path; keeps the source layout uniform
    GoldenView tg_host0{};
    const uint16_t* did = nullptr;
    const uint32_t* off = nullptr;
    uint32_t Nmax = 0, Lmax = 0, Rmax = 0;
    const riros_fault* faults = nullptr;
    const uint32_t* order = nullptr;
    int drop = 1;
    int light_cap = 8;
    uint32_t rate_num = 0;
    uint32_t blocks = 0;
    uint64_t span = 0;        // an upper bound of the stamps one block can use
    PlainWorkspace ws{};
    uint32_t* detect = nullptr;
    uint64_t* events = nullptr;
    riros_coverage* cov = nullptr;
};

// Kernel attributes (outside any capture).
hipError_t prepare_twod_batch(const BatchPlan& b);
// Order the concatenated faults by priority (NULL: keep them in order); sets
// the heavy prefix.  Not capturable.
int order_batch(TwoDWorkspace& ws, const float* priority, uint32_t F, float theta, const uint32_t** order,
                hipStream_t s, std::string& err);
// The capturable part of a campaign run: counter reset, launches A and B,
// stamp advance, per-design coverage.  ws must have been prepared by order_batch.
hipError_t launch_twod_batch(const BatchPlan& b, TwoDWorkspace& ws, hipStream_t s);

void twod_free(TwoDWorkspace& ws);

}  // namespace riros
