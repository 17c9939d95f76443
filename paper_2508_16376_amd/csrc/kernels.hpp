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
    const NodeRec* rec;        // per internal node: descriptor + fan-out ranges
    const LaneRec* lrec;       // per internal node: the record with its first users inline (light path)
    const uint64_t* fo_pk;     // fan-out entries: user id | user level << 32
    const uint32_t* bp_off;    // per internal node: first bit-plane row
    uint32_t N, L, R, npi;
    uint32_t bp_rows;
};

// Golden trace in three layouts: row-major G[t][n] (what the golden kernel
// writes and riros_golden_read returns; the structural path reads it in
// dense passes, where a level's nodes are neighbours), node-major Gn[n][t]
// (read by every sparse evaluation: a node evaluated in consecutive cycles
// stays in one cache line for sixteen cycles), and bit-planes Bp[row][w]
// with row = bp_off[n] + bit, word w holding cycles 64w..64w+63.
struct GoldenView {
    const uint64_t* G;
    const uint64_t* Gn;
    const uint64_t* Bp;
    uint32_t T;
    uint32_t TW;   // words per bit-plane row = ceil(T / 64)
    // Node-major 32-bit copy Gn32[n][t] when no node is wider than 32 bits
    // (else NULL): the light path's golden reads, a 128-byte line holding 32
    // cycles of a node instead of 16.
    const uint32_t* Gn32;
};

hipError_t launch_golden_layouts(const DevDesign& d, const uint64_t* G, uint32_t T, uint64_t* Gn, uint64_t* Bp,
                                 uint32_t* Gn32, hipStream_t s);

// Per-node faulty value with the cycle stamp that makes it valid.
struct __attribute__((aligned(16))) Slot {
    uint64_t v;
    uint64_t stamp;
};

hipError_t launch_golden(const DevDesign& d, const uint64_t* stim, uint32_t T, uint64_t* G, hipStream_t s);

// A design's golden parts on the device (build_golden_parts); P = 0 when the
// design has none (it then runs on one workgroup).
struct DevGoldenParts {
    const GNode* node;
    const uint32_t* part_off;
    const uint32_t* lvl;
    const uint32_t* lvl_off;
    uint32_t P, max_nodes;
};

// Golden trace by parts: one workgroup per part, the part's values of the
// current and the previous cycle in LDS.  golden_parts_setup (once, outside
// any graph capture) allows the kernel the LDS of the largest part.
hipError_t golden_parts_setup();

// One part of one design's golden machine, for launches that run the parts
// of many designs at once.
struct GPartJob {
    const GNode* node;
    const uint32_t* part_off;
    const uint32_t* lvl;
    const uint32_t* lvl_off;
    const uint64_t* stim;
    uint64_t* G;
    uint32_t part, npi, N, T;
};

// n part jobs in one launch, one workgroup each (jobs: a device table);
// max_nodes: the largest of their parts.
hipError_t launch_golden_parts_many(uint32_t n, const GPartJob* jobs, uint32_t max_nodes, hipStream_t s);
hipError_t launch_golden_parts(const DevDesign& d, const DevGoldenParts& gp, const uint64_t* stim, uint32_t T,
                               uint64_t* G, hipStream_t s);

// One design's golden run of a batched launch: its device stimulus [T][npi],
// cycle count and row-major trace.
struct GoldenJob {
    const uint64_t* stim;
    uint64_t* G;
    uint32_t T;
    uint32_t design;   // index into the launch's design table
};

// n golden traces in one launch, one workgroup per job (jobs: a device table
// of n entries; td: the design table their indexes refer to).
hipError_t launch_golden_many(uint32_t n, const DevDesign* td, const GoldenJob* jobs, hipStream_t s);

struct PlainWorkspace {
    Slot* slots;              // [blocks][N]
    uint64_t* regs;           // [blocks][2][R]
    uint64_t* stamp_dev;      // device-resident: stamps above it are unused in every block's slots
};

// Advance the device-resident stamp base (the last launch of every run, so a
// replayed graph never reuses a stamp).
hipError_t launch_advance_stamp(uint64_t* stamp_dev, uint64_t by, hipStream_t s);

// Bytes of dynamic LDS the plain kernel needs for a design.
size_t plain_lds_bytes(const DevDesign& d, uint32_t wpp);

hipError_t launch_fault_plain(const DevDesign& d, const GoldenView& g,
                              const riros_fault* faults, uint32_t F, int drop, uint32_t blocks,
                              const PlainWorkspace& ws, uint32_t wpp, uint32_t* detect, uint64_t* events,
                              uint64_t* words, hipStream_t s);

hipError_t launch_validate_faults(const DevDesign& d, const riros_fault* faults, uint32_t F,
                                  uint32_t* bad_count, hipStream_t s);

// Fill n 32-bit words with v (a kernel, so that it can be captured).
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);

hipError_t launch_coverage(const uint32_t* detect, const uint64_t* events, const uint64_t* words, uint32_t F,
                           uint32_t T, riros_coverage* cov, hipStream_t s);

}  // namespace riros
