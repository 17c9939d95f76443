// Golden simulation, the plain fault-parallel kernel, fault validation and
// coverage reduction.
#include "device_common.hpp"
#include "kernels.hpp"

namespace riros {

// ---------------------------------------------------------------------------
// Golden machine: one workgroup walks the levels of every cycle; the nodes of a
// level are independent and are spread over the workgroup's lanes.  Row t of G
// is the working array of cycle t; registers read row t-1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_golden(DevDesign d, const uint64_t* __restrict__ stim,
                                                 uint32_t T, uint64_t* __restrict__ G)
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

hipError_t launch_golden(const DevDesign& d, const uint64_t* stim, uint32_t T, uint64_t* G, hipStream_t s)
{
    hipLaunchKernelGGL(k_golden, dim3(1), dim3(1024), 0, s, d, stim, T, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain fault-parallel kernel: one fault per wavefront (one-wave workgroups),
// faults taken in index order by a grid-stride loop.  Inside a fault, the
// divergent frontier of each level is compacted from an LDS bitmap and split
// across the 64 lanes (the paper's structural parallelism, applied to one
// faulty machine).  A node is visited only when it is the fault site, a
// register whose state diverged, or a user of a divergent node (the check of
// whether a task's inputs changed, Alg. 1).
//
// LDS (dynamic): sched[N/32] nodes to evaluate this cycle; lvlm[L/32] levels
// holding scheduled nodes; rcur/rnext[R/32] registers whose state diverges in
// this / the next cycle; list[2048] compacted node ids; flags.
// Global workspace per block: slots[N] faulty value + validity stamp,
// regs[2][R] next-state of diverged registers (ping-pong by cycle parity).
// ---------------------------------------------------------------------------
constexpr uint32_t kListCap = 2048;

size_t plain_lds_bytes(const DevDesign& d)
{
    size_t W = (d.N + 31) / 32, WL = (d.L + 31) / 32, WR = (d.R + 31) / 32;
    return (W + WL + 2 * WR + kListCap + 4) * sizeof(uint32_t);
}

__global__ __launch_bounds__(64) void k_fault_plain(DevDesign d, const uint64_t* __restrict__ G,
                                                    uint32_t T, const riros_fault* __restrict__ faults,
                                                    uint32_t F, int drop, PlainWorkspace ws,
                                                    uint32_t* __restrict__ detect_out,
                                                    uint64_t* __restrict__ events_out)
{
    extern __shared__ uint32_t lds[];
    const uint32_t N = d.N, R = d.R;
    const uint32_t W = (N + 31) / 32, WL = (d.L + 31) / 32, WR = (R + 31) / 32;
    uint32_t* sched = lds;
    uint32_t* lvlm = sched + W;
    uint32_t* rcur = lvlm + WL;
    uint32_t* rnext = rcur + WR;
    uint32_t* list = rnext + WR;
    uint32_t* flags = list + kListCap;
    const uint32_t lane = threadIdx.x;

    for (uint32_t i = lane; i < W; i += 64) sched[i] = 0;
    for (uint32_t i = lane; i < WL; i += 64) lvlm[i] = 0;
    for (uint32_t i = lane; i < 2 * WR; i += 64) rcur[i] = 0;
    __syncthreads();

    Slot* slots = ws.slots + (size_t)blockIdx.x * N;
    uint64_t* regs = ws.regs + (size_t)blockIdx.x * 2 * R;
    uint32_t stamp0 = ws.stamp_base;

    for (uint32_t fi = blockIdx.x; fi < F; fi += gridDim.x) {
        const riros_fault f = faults[fi];
        const uint32_t site = d.u2i[f.site];
        const uint32_t site_lvl = d.level[site];
        const uint32_t fbit = f.bit, fval = f.stuck;
        for (uint32_t i = lane; i < WR; i += 64) rnext[i] = 0;
        uint32_t ev = 0;
        uint32_t det = RIROS_UNDETECTED;
        __syncthreads();
        for (uint32_t t = 0; t < T; ++t) {
            const uint32_t stamp = stamp0 + t + 1;
            const uint64_t* g = G + (size_t)t * N;
            const uint64_t* rst = regs + (size_t)(t & 1) * R;
            uint64_t* rnx = regs + (size_t)((t + 1) & 1) * R;
            // Cycle start: registers whose D diverged last cycle are scheduled.
            uint32_t any = 0;
            for (uint32_t i = lane; i < WR; i += 64) {
                uint32_t m = rnext[i];
                rcur[i] = m;
                rnext[i] = 0;
                sched[i] |= m;
                any |= m;
            }
            const bool anyreg = __ballot(any != 0) != 0;
            if (lane == 0) flags[0] = 0;
            __syncthreads();
            if (lane == 0) {
                sched[site >> 5] |= 1u << (site & 31);
                lvlm[site_lvl >> 5] |= 1u << (site_lvl & 31);
                if (anyreg) lvlm[0] |= 1u;
            }
            __syncthreads();
            for (;;) {
                // Lowest level with scheduled nodes (users are always at higher levels).
                int lv = -1;
                for (uint32_t wb = 0; wb < WL; wb += 64) {
                    const uint32_t w = wb + lane;
                    const uint32_t m = w < WL ? lvlm[w] : 0u;
                    const uint64_t bal = __ballot(m != 0);
                    if (bal) {
                        const int first = __ffsll((unsigned long long)bal) - 1;
                        const uint32_t mw = __shfl(m, first, 64);
                        lv = (int)((wb + first) * 32 + __ffs(mw) - 1);
                        break;
                    }
                }
                if (lv < 0) break;
                __syncthreads();
                if (lane == 0) lvlm[lv >> 5] &= ~(1u << (lv & 31));
                const uint32_t lo = d.lvl_off[lv], hi = d.lvl_off[lv + 1];
                const uint32_t w0 = lo >> 5, w1 = (hi - 1) >> 5;
                for (uint32_t wb = w0; wb <= w1; wb += 64) {
                    const uint32_t w = wb + lane;
                    uint32_t bits = 0;
                    if (w <= w1) {
                        uint32_t m = ~0u;
                        if (w == w0) m &= ~0u << (lo & 31);
                        if (w == w1 && (hi & 31)) m &= (1u << (hi & 31)) - 1u;
                        const uint32_t word = sched[w];
                        bits = word & m;
                        if (bits) sched[w] = word & ~m;
                    }
                    const uint32_t cnt = __popc(bits);
                    const uint32_t incl = wave_incl_scan(cnt);
                    const uint32_t total = __shfl(incl, 63, 64);
                    uint32_t off = incl - cnt;
                    while (bits) {
                        const int b = __ffs(bits) - 1;
                        bits &= bits - 1;
                        list[off++] = w * 32 + (uint32_t)b;
                    }
                    __syncthreads();
                    for (uint32_t i = lane; i < total; i += 64) {
                        const uint32_t n = list[i];
                        const Desc x = d.desc[n];
                        const uint64_t gv = g[n];
                        bool din = false;
                        uint64_t v;
                        if (x.op == RIROS_OP_REG) {
                            din = (rcur[n >> 5] >> (n & 31)) & 1u;
                            v = din ? rst[n] : gv;
                        } else if (x.op == RIROS_OP_PI || x.op == RIROS_OP_CONST) {
                            v = gv;
                        } else {
                            const int ar = dev_arity(x.op);
                            uint64_t xs[3] = {0, 0, 0};
                            const uint32_t ins[3] = {x.a, x.b, x.c};
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                if (k < ar) {
                                    const Slot sl = slots[ins[k]];
                                    const uint64_t gx = g[ins[k]];
                                    const bool dv = sl.stamp == stamp;
                                    xs[k] = dv ? sl.v : gx;
                                    din |= dv;
                                }
                            }
                            v = apply_op(x, xs[0], xs[1], xs[2]);
                        }
                        if (n == site) v = force_bit(v, fbit, fval);
                        const bool dout = v != gv;
                        ev += (din || dout) ? 1u : 0u;
                        if (dout) {
                            Slot sl;
                            sl.v = v;
                            sl.stamp = stamp;
                            sl.pad = 0;
                            slots[n] = sl;
                            if (x.flags & DF_PO) flags[0] = 1;
                            if (x.flags & DF_COMBFO) {
                                const uint32_t e1 = d.fo_off[n + 1];
                                for (uint32_t e = d.fo_off[n]; e < e1; ++e) {
                                    const uint32_t c = d.fo[e], lc = d.fo_lvl[e];
                                    atomicOr(&sched[c >> 5], 1u << (c & 31));
                                    atomicOr(&lvlm[lc >> 5], 1u << (lc & 31));
                                }
                            }
                            if (x.flags & DF_REGFO) {
                                const uint32_t e1 = d.rfo_off[n + 1];
                                for (uint32_t e = d.rfo_off[n]; e < e1; ++e) {
                                    const uint32_t r = d.rfo[e];
                                    rnx[r] = v;
                                    atomicOr(&rnext[r >> 5], 1u << (r & 31));
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            if (flags[0] && det == RIROS_UNDETECTED) det = t;
            __syncthreads();
            if (drop && det != RIROS_UNDETECTED) break;
        }
        stamp0 += T;
        const uint64_t tot = wave_sum_u64((uint64_t)ev);
        if (lane == 0) {
            detect_out[fi] = det;
            if (events_out) events_out[fi] = tot;
        }
    }
}

hipError_t launch_fault_plain(const DevDesign& d, const uint64_t* G, uint32_t T,
                              const riros_fault* faults, uint32_t F, int drop, uint32_t blocks,
                              const PlainWorkspace& ws, uint32_t* detect, uint64_t* events,
                              hipStream_t s)
{
    const size_t lds = plain_lds_bytes(d);
    hipError_t e = hipFuncSetAttribute((const void*)k_fault_plain,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fault_plain, dim3(blocks), dim3(64), lds, s, d, G, T, faults, F, drop, ws,
                       detect, events);
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
        b = f.site >= d.N || f.stuck > 1 || f.bit >= d.uwidth[f.site < d.N ? f.site : 0];
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
                           uint32_t F, uint32_t T, riros_coverage* __restrict__ cov)
{
    uint64_t det = 0, fc = 0, ev = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < F; i += gridDim.x * blockDim.x) {
        const uint32_t dc = detect[i];
        det += dc != RIROS_UNDETECTED;
        fc += dc != RIROS_UNDETECTED ? (uint64_t)dc + 1 : (uint64_t)T;
        if (events) ev += events[i];
    }
    det = wave_sum_u64(det);
    fc = wave_sum_u64(fc);
    ev = wave_sum_u64(ev);
    if (lane_id() == 0) {
        atomicAdd((unsigned long long*)&cov->detected, (unsigned long long)det);
        atomicAdd((unsigned long long*)&cov->fault_cycles, (unsigned long long)fc);
        atomicAdd((unsigned long long*)&cov->events, (unsigned long long)ev);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long*)&cov->total, (unsigned long long)F);
}

__global__ void k_zero_cov(riros_coverage* cov)
{
    if (threadIdx.x == 0) {
        cov->detected = 0;
        cov->total = 0;
        cov->fault_cycles = 0;
        cov->events = 0;
    }
}

hipError_t launch_coverage(const uint32_t* detect, const uint64_t* events, uint32_t F, uint32_t T,
                           riros_coverage* cov, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_cov, dim3(1), dim3(64), 0, s, cov);
    uint32_t blocks = (F + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_coverage, dim3(blocks), dim3(256), 0, s, detect, events, F, T, cov);
    return hipGetLastError();
}

}  // namespace riros
