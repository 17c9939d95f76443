// Two-dimensional fault simulation: light faults one per lane, heavy faults
// split structurally across a wavefront, both fed by a persistent work queue.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "kernels.hpp"
#include "riros.h"

namespace riros {

struct TwoDWorkspace {
    void* mem = nullptr;
    size_t bytes = 0;
};

struct TwoDParams {
    float theta = INFINITY;
    int light_cap = 0;
    int chunk = 0;
    int waves_per_cu = 0;
    int num_cu = 0;
};

int run_twod(const DevDesign& d, TwoDWorkspace& ws, const uint64_t* G, uint32_t T,
             const riros_fault* faults, const float* priority, uint32_t F, int drop,
             const TwoDParams& p, uint32_t* detect, uint64_t* events, hipEvent_t ev0,
             hipEvent_t ev1, hipStream_t s, std::string& err);

void twod_free(TwoDWorkspace& ws);

}  // namespace riros
