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
    void* ctr = nullptr;   // device counters of the last run
};

struct TwoDParams {
    float theta = INFINITY;
    int light_cap = 0;
    int unified = 0;            // waves out of light work take handed-over faults during launch A
    int share = 0;              // launch A wavefronts per structural workspace (0 = as the LDS needs)
    int heavy_wg = 64;          // threads that simulate one structural fault (64, 128 or 256)
    bool w32 = false;           // every node at most 32 bits wide: light lanes keep 32-bit values
    int lockstep = 0;           // light lanes of a wavefront start their cycles together
    uint32_t deal = 0;          // light queue dealt in groups of this many faults (0 = queue order)
    uint32_t head_lanes = 0;    // a wavefront's first take, finished before it takes more (0 = off)
    bool xcd = false;           // per-XCD light queues (with priorities)
    int waves_per_cu = 0;
    int num_cu = 0;
    float monitor_rate = 0.f;   // hand a light fault over above this many events per cycle (0 = never)
};

// Launch A: the faults whose priority is above theta on the structural path
// first, then the rest one per lane in descending priority order (all faults
// in list order when priority is NULL), then (unified) handed-over faults;
// launch B: the handed-over faults left.  heavy_ws / heavy_blocks: per-wave
// workspace of the structural path and the grid size.
int run_twod(const DevDesign& d, TwoDWorkspace& ws, const GoldenView& gv,
             const riros_fault* faults, const float* priority, uint32_t F, int drop,
             const TwoDParams& p, PlainWorkspace heavy_ws, uint32_t heavy_blocks,
             uint32_t* detect, uint64_t* events, uint64_t* words, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s,
             std::string& err);

// Synchronises s and checks the last run's counters: every handed-over fault
// was simulated (RIROS_EDEVICE otherwise).
int twod_check(const TwoDWorkspace& ws, hipStream_t s, std::string& err);

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
    uint32_t wpp = 64;        // structural schedule words per pass
    const riros_fault* faults = nullptr;
    const uint32_t* order = nullptr;
    bool heavy = false;       // a heavy prefix exists (priorities with a finite threshold)
    int unified = 0;          // phase 3 in launch A (see riros_sim_opts.unified)
    int share = 0;            // launch A wavefronts per structural workspace (see riros_sim_opts.struct_share)
    uint32_t heavy_wg = 64;   // threads per structural fault (see riros_sim_opts.heavy_wg)
    bool w32 = false;         // every node of every design at most 32 bits wide (32-bit light lanes)
    int lockstep = 0;         // light lanes of a wavefront start their cycles together
    uint32_t deal = 0;        // light queue dealt in groups of this many faults (0 = queue order)
    uint32_t head_lanes = 0;  // a wavefront's first take, finished before it takes more (0 = off)
    bool xcd = false;         // per-XCD light queues (with priorities; the order was partitioned at creation)
    int drop = 1;
    int light_cap = 8;
    uint32_t rate_num = 0;
    uint32_t blocks = 0;      // launch B (and workspace) grid
    uint32_t blocks_a = 0;    // launch A grid (at most what is resident at once)
    uint32_t threads_a = 64;  // launch A workgroup size (64 * wavefronts sharing a structural workspace)
    uint32_t blocks_b = 0;    // launch B grid (likewise)
    uint64_t span = 0;        // an upper bound of the stamps one block can use
    PlainWorkspace ws{};
    uint32_t* detect = nullptr;
    uint64_t* events = nullptr;
    uint64_t* words = nullptr;
    riros_coverage* cov = nullptr;
};

// Kernel attributes (outside any capture).
hipError_t prepare_twod_batch(BatchPlan& b);
// Order the concatenated faults by priority (NULL: keep them in order), faults
// of one site together within a priority band; sets the heavy prefix.  Not
// capturable.
int order_batch(TwoDWorkspace& ws, const float* priority, const riros_fault* faults, uint32_t F, float theta, int xcd,
                const uint32_t** order, hipStream_t s, std::string& err);
// The capturable part of a campaign run: counter reset, launches A and B,
// stamp advance, per-design coverage.  ws must have been prepared by order_batch.
hipError_t launch_twod_batch(const BatchPlan& b, TwoDWorkspace& ws, hipStream_t s);

void twod_free(TwoDWorkspace& ws);

}  // namespace riros
