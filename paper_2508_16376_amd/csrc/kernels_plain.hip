// Golden simulation, the plain fault-parallel kernel, fault validation and
// coverage reduction.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"
#include "wave_fault.hpp"

namespace riros {

// ---------------------------------------------------------------------------
// Golden machine: one workgroup walks the levels of every cycle; the nodes of a
// level are independent and are spread over the workgroup's lanes.  Row t of G
// is the working array of cycle t; registers read row t-1.  A campaign runs
// one workgroup per design in a single launch (its designs are independent).
// ---------------------------------------------------------------------------
__device__ void golden_design(const DevDesign& d, const uint64_t* __restrict__ stim, uint32_t T,
                              uint64_t* __restrict__ G)
{
    const uint32_t N = d.N;
    for (uint32_t t = 0; t < T; ++t) {
        uint64_t* row = G + (size_t)t * N;
        const uint64_t* prev = row - N;
        for (uint32_t l = 0; l < d.L; ++l) {
            const uint32_t lo = d.lvl_off[l], hi = d.lvl_off[l + 1];
            for (uint32_t n = lo + threadIdx.x; n < hi; n += blockDim.x) {
                const Desc x = d.desc[n];
                uint64_t v;
                switch (x.op) {
                case RIROS_OP_CONST: v = make_u64(x.a, x.b); break;
                case RIROS_OP_PI: v = stim[(size_t)t * d.npi + x.a] & width_mask(x.width); break;
                case RIROS_OP_REG: v = t == 0 ? make_u64(x.b, x.c) : prev[x.a]; break;
                default: {
                    const int ar = dev_arity(x.op);
                    uint64_t x0 = row[x.a];
                    uint64_t x1 = ar >= 2 ? row[x.b] : 0;
                    uint64_t x2 = ar >= 3 ? row[x.c] : 0;
                    v = apply_op(x, x0, x1, x2);
                }
                }
                row[n] = v;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(1024) void k_golden(DevDesign d, const uint64_t* __restrict__ stim, uint32_t T,
                                                 uint64_t* __restrict__ G)
{
    golden_design(d, stim, T, G);
}

// Workgroup k: design k of a campaign (device tables of n entries).
__global__ __launch_bounds__(1024) void k_golden_many(const DevDesign* __restrict__ td,
                                                      const GoldenJob* __restrict__ jobs)
{
    const GoldenJob j = jobs[blockIdx.x];
    golden_design(td[j.design], j.stim, j.T, j.G);
}

hipError_t launch_golden(const DevDesign& d, const uint64_t* stim, uint32_t T, uint64_t* G, hipStream_t s)
{
    hipLaunchKernelGGL(k_golden, dim3(1), dim3(1024), 0, s, d, stim, T, G);
    return hipGetLastError();
}

hipError_t launch_golden_many(uint32_t n, const DevDesign* td, const GoldenJob* jobs, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_golden_many, dim3(n), dim3(1024), 0, s, td, jobs);
    return hipGetLastError();
}

// Golden machine by parts: workgroup p simulates part p (independent of every
// other part: its components read only each other and the inputs and
// constants copied into it) for every cycle.  The part's values of the current
// cycle (cur) and the previous one (prev, which registers read) stay in LDS;
// each level's nodes are spread over the workgroup's lanes, a barrier between
// levels; at the end of a cycle the part writes the trace columns it owns.
__device__ void golden_part(const GPartJob& j, uint32_t max_nodes)
{
    extern __shared__ uint64_t gpv[];
    const uint32_t o = j.part_off[j.part], m = j.part_off[j.part + 1] - o;
    const uint32_t l0 = j.lvl_off[j.part], l1 = j.lvl_off[j.part + 1];
    const GNode* __restrict__ nd = j.node + o;
    const uint64_t* __restrict__ stim = j.stim;
    uint64_t* __restrict__ G = j.G;
    const uint32_t T = j.T, npi = j.npi;
    uint64_t* cur = gpv;
    uint64_t* prev = gpv + max_nodes;
    const size_t N = j.N;
    for (uint32_t t = 0; t < T; ++t) {
        for (uint32_t li = l0; li + 1 < l1; ++li) {
            const uint32_t lo = j.lvl[li], hi = j.lvl[li + 1];
            for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
                const GNode x = nd[i];
                uint64_t v;
                switch (x.op) {
                case RIROS_OP_CONST: v = make_u64(x.a, x.b); break;
                case RIROS_OP_PI: v = stim[(size_t)t * npi + x.a] & width_mask(x.width); break;
                case RIROS_OP_REG: v = t == 0 ? make_u64(x.b, x.c) : prev[x.a]; break;
                default: {
                    const int ar = dev_arity(x.op);
                    const uint64_t x0 = cur[x.a];
                    const uint64_t x1 = ar >= 2 ? cur[x.b] : 0;
                    const uint64_t x2 = ar >= 3 ? cur[x.c] : 0;
                    v = apply_opw(x.op, x.width, x.b, x.c, x0, x1, x2);
                }
                }
                cur[i] = v;
            }
            __syncthreads();
        }
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            const uint32_t gid = nd[i].gid;
            if (gid != kNoGid) G[(size_t)t * N + gid] = cur[i];
        }
        uint64_t* tmp = cur;
        cur = prev;
        prev = tmp;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_golden_parts(DevDesign d, DevGoldenParts gp,
                                                      const uint64_t* __restrict__ stim, uint32_t T,
                                                      uint64_t* __restrict__ G)
{
    const GPartJob j{gp.node, gp.part_off, gp.lvl, gp.lvl_off, stim, G, blockIdx.x, d.npi, d.N, T};
    golden_part(j, gp.max_nodes);
}

// Workgroup k: part jobs[k] (parts of many designs in one launch).
__global__ __launch_bounds__(256) void k_golden_parts_many(const GPartJob* __restrict__ jobs, uint32_t max_nodes)
{
    golden_part(jobs[blockIdx.x], max_nodes);
}

hipError_t golden_parts_setup()
{
    const int lds = (int)(2 * kGoldenPartCap * sizeof(uint64_t));
    hipError_t e = hipFuncSetAttribute((const void*)k_golden_parts, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_golden_parts_many, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e;
}

hipError_t launch_golden_parts(const DevDesign& d, const DevGoldenParts& gp, const uint64_t* stim, uint32_t T,
                               uint64_t* G, hipStream_t s)
{
    const size_t lds = (size_t)2 * gp.max_nodes * sizeof(uint64_t);
    hipLaunchKernelGGL(k_golden_parts, dim3(gp.P), dim3(256), lds, s, d, gp, stim, T, G);
    return hipGetLastError();
}

hipError_t launch_golden_parts_many(uint32_t n, const GPartJob* jobs, uint32_t max_nodes, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_golden_parts_many, dim3(n), dim3(256), (size_t)2 * max_nodes * sizeof(uint64_t), s, jobs,
                       max_nodes);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Golden layouts for per-lane walks: a 64-node x 64-cycle tile of the
// row-major trace is staged in LDS, written out node-major (coalesced along
// cycles), and each bit of each node becomes one 64-cycle bit-plane word by a
// wave ballot with lane = cycle.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_golden_layouts(DevDesign d, const uint64_t* __restrict__ G, uint32_t T,
                                                       uint32_t TW, uint64_t* __restrict__ Gn,
                                                       uint64_t* __restrict__ Bp, uint32_t* __restrict__ Gn32)
{
    __shared__ uint64_t tile[64][65];
    const uint32_t lane = threadIdx.x;
    const uint32_t N = d.N;
    const uint32_t n0 = blockIdx.x * 64, wb = blockIdx.y, t0 = wb * 64;
    for (uint32_t i = 0; i < 64; ++i) {
        const uint32_t t = t0 + i, n = n0 + lane;
        tile[i][lane] = (t < T && n < N) ? G[(size_t)t * N + n] : 0ull;
    }
    __syncthreads();
    const uint32_t t = t0 + lane;
    const bool tv = t < T;
    const uint32_t nend = min(64u, N - n0);
    for (uint32_t j = 0; j < nend; ++j) {
        const uint32_t n = n0 + j;
        const uint64_t v = tile[lane][j];
        if (tv) Gn[(size_t)n * T + t] = v;
        if (tv && Gn32) Gn32[(size_t)n * T + t] = (uint32_t)v;
        const uint32_t w = d.rec[n].width;
        const uint32_t row0 = d.bp_off[n];
        uint64_t mine = 0;
        for (uint32_t b = 0; b < w; ++b) {
            const uint64_t word = __ballot(tv && ((v >> b) & 1ull));
            if (lane == b) mine = word;
        }
        if (lane < w) Bp[(size_t)(row0 + lane) * TW + wb] = mine;
    }
}

hipError_t launch_golden_layouts(const DevDesign& d, const uint64_t* G, uint32_t T, uint64_t* Gn, uint64_t* Bp,
                                 uint32_t* Gn32, hipStream_t s)
{
    const uint32_t TW = (T + 63) / 64;
    hipLaunchKernelGGL(k_golden_layouts, dim3((d.N + 63) / 64, TW), dim3(64), 0, s, d, G, T, TW, Gn, Bp, Gn32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain fault-parallel kernel: one fault per wavefront (one-wave workgroups),
// faults taken in index order by a grid-stride loop; each fault is simulated
// by wave_sim_fault (the divergent frontier of each level compacted from an
// LDS bitmap and split across the 64 lanes).  A node is visited only when it
// is the fault site, a register whose state diverged, or a user of a
// divergent node (the check of whether a task's inputs changed, Alg. 1).
// Global workspace per block: slots[N] faulty value + validity stamp,
// regs[2][R] next state of diverged registers (ping-pong by cycle parity).
// ---------------------------------------------------------------------------
size_t plain_lds_bytes(const DevDesign& d, uint32_t wpp)
{
    return wave_lds_words(d.N, d.L, d.R, wpp) * sizeof(uint32_t);
}

__global__ __launch_bounds__(64) void k_fault_plain(DevDesign d, const uint64_t* __restrict__ Gr,
                                                    const uint64_t* __restrict__ Gn,
                                                    const uint64_t* __restrict__ Bp, uint32_t T, uint32_t TW,
                                                    const riros_fault* __restrict__ faults,
                                                    uint32_t F, int drop, PlainWorkspace ws, uint32_t wpp,
                                                    uint32_t* __restrict__ detect_out,
                                                    uint64_t* __restrict__ events_out,
                                                    uint64_t* __restrict__ words_out)
{
    extern __shared__ uint32_t lds[];
    const WaveLds s = wave_lds_carve(lds, d.N, d.L, d.R, wpp);
    wave_lds_clear(s, d.N, d.L, d.R);
    __syncthreads();
    Slot* slots = ws.slots + (size_t)blockIdx.x * d.N;
    uint64_t* regs = ws.regs + (size_t)blockIdx.x * 2 * d.R;
    uint64_t stamp0 = *ws.stamp_dev;
    for (uint32_t fi = blockIdx.x; fi < F; fi += gridDim.x) {
        uint32_t det;
        uint64_t ev, wk;
        wave_sim_fault(d, Gr, Gn, Bp, T, TW, faults[fi], drop, s, slots, regs, stamp0, det, ev, wk);
        if (threadIdx.x == 0) {
            detect_out[fi] = det;
            if (events_out) events_out[fi] = ev;
            if (words_out) words_out[fi] = wk;
        }
    }
}

__global__ void k_advance_stamp(uint64_t* stamp_dev, uint64_t by)
{
    if (threadIdx.x == 0) *stamp_dev += by;
}

hipError_t launch_advance_stamp(uint64_t* stamp_dev, uint64_t by, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_stamp, dim3(1), dim3(64), 0, s, stamp_dev, by);
    return hipGetLastError();
}

hipError_t launch_fault_plain(const DevDesign& d, const GoldenView& g,
                              const riros_fault* faults, uint32_t F, int drop, uint32_t blocks,
                              const PlainWorkspace& ws, uint32_t wpp, uint32_t* detect, uint64_t* events,
                              uint64_t* words, hipStream_t s)
{
    const size_t lds = plain_lds_bytes(d, wpp);
    hipError_t e = hipFuncSetAttribute((const void*)k_fault_plain,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fault_plain, dim3(blocks), dim3(64), lds, s, d, g.G, g.Gn, g.Bp, g.T, g.TW, faults, F, drop, ws,
                       wpp, detect, events, words);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fault validation (device-resident fault lists) and coverage totals.
// ---------------------------------------------------------------------------
__global__ void k_validate(DevDesign d, const riros_fault* __restrict__ faults, uint32_t F,
                           uint32_t* __restrict__ bad)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool b = false;
    if (i < F) {
        const riros_fault f = faults[i];
        b = f.site >= d.N || f.stuck > RIROS_FAULT_FLIP || f.bit >= d.uwidth[f.site < d.N ? f.site : 0];
    }
    const uint64_t bal = __ballot(b);
    if (lane_id() == 0 && bal) atomicAdd(bad, (uint32_t)__popcll(bal));
}

hipError_t launch_validate_faults(const DevDesign& d, const riros_fault* faults, uint32_t F,
                                  uint32_t* bad_count, hipStream_t s)
{
    if (F == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3((F + 255) / 256), dim3(256), 0, s, d, faults, F, bad_count);
    return hipGetLastError();
}

__global__ void k_coverage(const uint32_t* __restrict__ detect, const uint64_t* __restrict__ events,
                           const uint64_t* __restrict__ words, uint32_t F, uint32_t T,
                           riros_coverage* __restrict__ cov)
{
    uint64_t det = 0, fc = 0, ev = 0, wk = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < F; i += gridDim.x * blockDim.x) {
        const uint32_t dc = detect[i];
        det += dc != RIROS_UNDETECTED;
        fc += dc != RIROS_UNDETECTED ? (uint64_t)dc + 1 : (uint64_t)T;
        if (events) ev += events[i];
        if (words) wk += words[i];
    }
    det = wave_sum_u64(det);
    fc = wave_sum_u64(fc);
    ev = wave_sum_u64(ev);
    wk = wave_sum_u64(wk);
    if (lane_id() == 0) {
        atomicAdd((unsigned long long*)&cov->detected, (unsigned long long)det);
        atomicAdd((unsigned long long*)&cov->fault_cycles, (unsigned long long)fc);
        atomicAdd((unsigned long long*)&cov->events, (unsigned long long)ev);
        atomicAdd((unsigned long long*)&cov->words, (unsigned long long)wk);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long*)&cov->total, (unsigned long long)F);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void k_zero_cov(riros_coverage* cov)
{
    if (threadIdx.x == 0) {
        cov->detected = 0;
        cov->total = 0;
        cov->fault_cycles = 0;
        cov->events = 0;
        cov->words = 0;
    }
}

hipError_t launch_coverage(const uint32_t* detect, const uint64_t* events, const uint64_t* words, uint32_t F,
                           uint32_t T, riros_coverage* cov, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_cov, dim3(1), dim3(64), 0, s, cov);
    uint32_t blocks = (F + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_coverage, dim3(blocks), dim3(256), 0, s, detect, events, words, F, T, cov);
    return hipGetLastError();
}

}  // namespace riros
