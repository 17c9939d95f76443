// Concurrent (node-major) fault simulation: groups of 64 faults, one per lane
// of a wavefront, walk the union of their divergent frontiers node by node.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "kernels.hpp"
#include "riros.h"

namespace riros {

// Device memory of the concurrent mode, grown on demand and kept with the
// design.  sim: per resident wavefront ("slot") the faulty state of 64
// faults, node-major; sort: the fault order of the last call.
struct ConcWorkspace {
    void* sim = nullptr;
    size_t sim_bytes = 0;
    uint32_t slots = 0;      // slots the sim buffer was laid out for
    uint32_t N = 0, R = 0;   // design shape it was laid out for
    void* sort = nullptr;
    size_t sort_bytes = 0;
};

void conc_free(ConcWorkspace& ws);

// Bytes of dynamic LDS of the concurrent kernel for a design: the frontier
// bitmap, its summary and the next-cycle register bitmap.
size_t conc_lds_bytes(uint32_t N, uint32_t R);

// Device bytes of one slot's faulty state.
size_t conc_slot_bytes(uint32_t N, uint32_t R);

// Largest device memory the concurrent mode takes for faulty state: this,
// and at most 60% of what the device has free when the state is laid out.
constexpr size_t kConcMaxSimBytes = 128ull << 30;

// Order the faults by site and simulate them in groups of 64.  waves_per_cu
// bounds the resident wavefronts per compute unit (0 = as many as LDS and
// the faulty-state budget allow).  ev0/ev1 bracket the sort and the kernel.
int run_concurrent(const DevDesign& d, ConcWorkspace& ws, const GoldenView& gv, const riros_fault* faults,
                   uint32_t F, int drop, int waves_per_cu, int num_cu, uint32_t* detect, uint64_t* events,
                   uint64_t* words,
                   hipEvent_t ev0, hipEvent_t ev1, hipStream_t s, std::string& err);

}  // namespace riros
