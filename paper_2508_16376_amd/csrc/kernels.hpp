// Launch wrappers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "design.hpp"

namespace riros {

// Device-resident levelised design.
struct DevDesign {
    const Desc* desc;
    const uint32_t* lvl_off;
    const uint32_t* level;
    const uint32_t* fo_off;
    const uint32_t* fo;
    const uint32_t* fo_lvl;
    const uint32_t* rfo_off;
    const uint32_t* rfo;
    const uint32_t* u2i;
    const uint8_t* uwidth;     // width per user node id
    uint32_t N, L, R, npi;
};

// Per-node faulty value with the cycle stamp that makes it valid.
struct __attribute__((aligned(16))) Slot {
    uint64_t v;
    uint32_t stamp;
    uint32_t pad;
};

hipError_t launch_golden(const DevDesign& d, const uint64_t* stim, uint32_t T, uint64_t* G, hipStream_t s);

struct PlainWorkspace {
    Slot* slots;          // [blocks][N]
    uint64_t* regs;       // [blocks][2][R]
    uint32_t stamp_base;
};

// Bytes of dynamic LDS the plain kernel needs for a design.
size_t plain_lds_bytes(const DevDesign& d);

hipError_t launch_fault_plain(const DevDesign& d, const uint64_t* G, uint32_t T,
                              const riros_fault* faults, uint32_t F, int drop, uint32_t blocks,
                              const PlainWorkspace& ws, uint32_t* detect, uint64_t* events,
                              hipStream_t s);

hipError_t launch_validate_faults(const DevDesign& d, const riros_fault* faults, uint32_t F,
                                  uint32_t* bad_count, hipStream_t s);

hipError_t launch_coverage(const uint32_t* detect, const uint64_t* events, uint32_t F, uint32_t T,
                           riros_coverage* cov, hipStream_t s);

}  // namespace riros
