// Concurrent fault simulation on a wavefront (Sec. II-B, Sec. IV-B).
//
// In concurrent fault simulation a node carries its good gate and one bad
// gate for each fault whose value at the node differs from the good value,
// and a node is executed only when one of its inputs changed (the check step
// of Alg. 1).  Here one wavefront takes a group of 64 faults, one per lane.
// The group's frontier is the union of the lanes' frontiers: a bitmap over
// node ids in LDS, taken in ascending id order (ids are level-major, so a
// node's users come after it).  Each frontier node is fetched once (record,
// golden values, which lanes hold a bad gate on each input) and all 64 lanes
// evaluate it together.  A lane with no bad gate on any input computes the
// good value and counts no event, so every fault's detect cycle and event
// count equal those of simulating it alone.
//
// Faulty state in device memory, per resident wavefront ("slot"):
//   mask[n]            lanes whose value at node n differs from the golden
//                      one this cycle, with the cycle stamp that makes it
//                      valid; written and read by lane 0 only (the others
//                      take lane 0's copy), so no lane reads a global write
//                      of another lane
//   val[n][64]         each lane's faulty value at n (lane-private)
//   rmask[2][R], rval[2][R][64]   register states for this and the next cycle
//   base               the slot's stamp counter (stamps only grow)
// The LDS holds the frontier bitmap, one summary bit per non-empty bitmap
// word, and the registers whose state diverges in the next cycle.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "concurrent.hpp"
#include "device_common.hpp"

namespace riros {

namespace {

struct __attribute__((aligned(16))) LaneMask {
    uint64_t mask;
    uint64_t stamp;
};

struct ConcState {
    uint32_t* tickets;   // [1] next group
    uint64_t* base;      // [slots]
    LaneMask* mask;      // [slots][N]
    LaneMask* rmask;     // [slots][2][R]
    uint64_t* val;       // [slots][N][64]
    uint64_t* rval;      // [slots][2][R][64]
};

__device__ __forceinline__ uint64_t lane0_u64(uint64_t x)
{
    return make_u64(__builtin_amdgcn_readfirstlane((uint32_t)x), __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)));
}

// Orders this wavefront's LDS accesses across its lanes and waits for them;
// outstanding global memory operations are not waited for.
__device__ __forceinline__ void lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x)
{
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, k, 64));
    return x;
}

// Whether the fault changes its site's value in cycle t in an otherwise good
// machine: the golden site bit differs from the stuck value, or it is the
// flip's cycle.  srow: the site bit's golden bit-plane, 64 cycles a word.
__device__ __forceinline__ bool excited_at(const uint64_t* srow, uint32_t stuck, uint32_t t0, uint32_t t)
{
    if (stuck == RIROS_FAULT_FLIP) return t == t0;
    const uint32_t b = (uint32_t)(srow[t >> 6] >> (t & 63)) & 1u;
    return b != stuck;
}

// First cycle at or after t in which the site is excited, or T.
__device__ __forceinline__ uint32_t next_excited(const uint64_t* srow, uint32_t stuck, uint32_t t0, uint32_t t,
                                                 uint32_t T)
{
    if (stuck == RIROS_FAULT_FLIP) return (t <= t0 && t0 < T) ? t0 : T;
    while (t < T) {
        const uint32_t wb = t >> 6;
        uint64_t w = srow[wb];
        if (stuck) w = ~w;
        const uint32_t valid = T - (wb << 6);
        if (valid < 64) w &= (1ull << valid) - 1ull;
        const uint64_t m = w >> (t & 63);
        if (m) return t + (uint32_t)__builtin_ctzll(m);
        t = (wb + 1) << 6;
    }
    return T;
}

// One wavefront per workgroup; each takes groups of 64 consecutive faults of
// the order from a ticket counter until none is left (every wavefront reaches
// the exit once the tickets pass the group count).
__global__ void __launch_bounds__(64) k_concurrent(DevDesign d, const uint64_t* __restrict__ Gn,
                                                   const uint64_t* __restrict__ Bp, uint32_t T, uint32_t TW,
                                                   const riros_fault* __restrict__ faults,
                                                   const uint32_t* __restrict__ order, uint32_t F, int drop,
                                                   ConcState st, uint32_t* __restrict__ detect,
                                                   uint64_t* __restrict__ events, uint64_t* __restrict__ words)
{
    extern __shared__ uint64_t conc_lds[];
    const uint32_t N = d.N, R = d.R;
    const uint32_t NW = (N + 63) / 64, NS = (NW + 63) / 64, RW = (R + 63) / 64;
    uint64_t* const bm = conc_lds;    // [NW] frontier of this cycle
    uint64_t* const sm = bm + NW;     // [NS] non-empty bm words
    uint64_t* const rn = sm + NS;     // [RW] registers divergent next cycle
    const uint32_t lane = threadIdx.x;
    const uint32_t slot = blockIdx.x;
    LaneMask* const mask = st.mask + (size_t)slot * N;
    LaneMask* const rmask = st.rmask + (size_t)slot * 2 * R;
    uint64_t* const val = st.val + (size_t)slot * N * 64;
    uint64_t* const rval = st.rval + (size_t)slot * 2 * R * 64;
    for (uint32_t i = lane; i < NW + NS + RW; i += 64) conc_lds[i] = 0;
    uint64_t base = lane0_u64(st.base[slot]);
    const uint32_t G = (F + 63) / 64;
    lds_order();
    for (;;) {
        uint32_t g = 0;
        if (lane == 0) g = atomicAdd(st.tickets, 1u);
        g = __builtin_amdgcn_readfirstlane(g);
        if (g >= G) break;
        const uint32_t pos = g * 64 + lane;
        bool active = pos < F;
        uint32_t fi = 0, site = 0xFFFFFFFFu, fbit = 0, fst = 0, ft0 = 0;
        const uint64_t* srow = Bp;
        if (active) {
            fi = order ? order[pos] : pos;
            const riros_fault f = faults[fi];
            site = d.u2i[f.site];
            fbit = f.bit;
            fst = f.stuck;
            ft0 = f.t0;
            srow = Bp + (size_t)(d.bp_off[site] + fbit) * TW;
        }
        uint32_t det = RIROS_UNDETECTED;
        uint64_t ev = 0, wk = 0;   // events and byte-model words of the lane's fault
        bool rpend = false;   // registers were scheduled for the next cycle (uniform)
        for (uint32_t i = lane; i < RW; i += 64) rn[i] = 0;
        lds_order();
        uint32_t t = 0;
        while (t < T) {
            bool exc = active && excited_at(srow, fst, ft0, t);
            if (!rpend && __ballot(exc) == 0) {
                // No lane holds divergent state and no site is excited: every
                // machine of the group equals the golden one until the next
                // cycle in which some site is excited (no event, no detection
                // in between).
                uint32_t nx = active ? next_excited(srow, fst, ft0, t + 1, T) : T;
                nx = wave_min_u32(nx);
                if (nx >= T) break;
                t = nx;
                exc = active && excited_at(srow, fst, ft0, t);
            }
            const uint64_t stamp = base + t + 1;
            const uint32_t p = t & 1, q = p ^ 1;
            // Seed the frontier: registers whose D diverged last cycle (they
            // have the lowest ids, words below RW, all empty at cycle start)
            // and the excited sites.
            if (rpend) {
                for (uint32_t i = lane; i < RW; i += 64) {
                    const uint64_t m = rn[i];
                    if (m) {
                        rn[i] = 0;
                        bm[i] = m;
                        atomicOr(&sm[i >> 6], 1ull << (i & 63));
                    }
                }
                lds_order();
            }
            if (exc) {
                atomicOr(&bm[site >> 6], 1ull << (site & 63));
                atomicOr(&sm[site >> 12], 1ull << ((site >> 6) & 63));
            }
            rpend = false;
            lds_order();
            for (uint32_t sw = 0; sw < NS; ++sw) {
                for (;;) {
                    uint64_t s = 0;
                    if (lane == 0) s = sm[sw];
                    s = lane0_u64(s);
                    if (!s) break;
                    const uint32_t wi = (uint32_t)__builtin_ctzll(s);
                    const uint32_t w = sw * 64 + wi;
                    uint64_t cur = 0;
                    if (lane == 0) {
                        sm[sw] = s & ~(1ull << wi);
                        cur = bm[w];
                        bm[w] = 0;
                    }
                    cur = lane0_u64(cur);
                    lds_order();
                    while (cur) {
                        const uint32_t n = w * 64 + (uint32_t)__builtin_ctzll(cur);
                        cur &= cur - 1;
                        const NodeRec x = d.rec[n];
                        const uint64_t gv = Gn[(size_t)n * T + t];
                        const bool isreg = x.op == RIROS_OP_REG;
                        const bool comb = !isreg && x.op != RIROS_OP_PI && x.op != RIROS_OP_CONST;
                        uint64_t v = gv;
                        bool din = false;
                        if (isreg) {
                            const size_t ri = (size_t)p * R + n;
                            const LaneMask m = rmask[ri];
                            const uint64_t rv = rval[ri * 64 + lane];
                            const uint64_t k = lane0_u64(m.stamp) == stamp ? lane0_u64(m.mask) : 0ull;
                            din = (k >> lane) & 1ull;
                            if (din) v = rv;
                        } else if (comb) {
                            // Every load of the node issued together: which
                            // lanes hold a bad gate on each input, the lane's
                            // faulty input values and the golden ones (an
                            // input the operator does not read repeats the
                            // first).
                            const int ar = dev_arity(x.op);
                            const uint32_t i0 = x.a, i1 = ar > 1 ? x.b : i0, i2 = ar > 2 ? x.c : i0;
                            const LaneMask m0 = mask[i0], m1 = mask[i1], m2 = mask[i2];
                            const uint64_t v0 = val[(size_t)i0 * 64 + lane];
                            const uint64_t v1 = val[(size_t)i1 * 64 + lane];
                            const uint64_t v2 = val[(size_t)i2 * 64 + lane];
                            const uint64_t g0 = Gn[(size_t)i0 * T + t];
                            const uint64_t g1 = Gn[(size_t)i1 * T + t];
                            const uint64_t g2 = Gn[(size_t)i2 * T + t];
                            const uint64_t k0 = lane0_u64(m0.stamp) == stamp ? lane0_u64(m0.mask) : 0ull;
                            const uint64_t k1 = (ar > 1 && lane0_u64(m1.stamp) == stamp) ? lane0_u64(m1.mask) : 0ull;
                            const uint64_t k2 = (ar > 2 && lane0_u64(m2.stamp) == stamp) ? lane0_u64(m2.mask) : 0ull;
                            const bool b0 = (k0 >> lane) & 1ull, b1 = (k1 >> lane) & 1ull, b2 = (k2 >> lane) & 1ull;
                            din = b0 || b1 || b2;
                            v = apply_opw(x.op, x.width, x.b, x.c, b0 ? v0 : g0, b1 ? v1 : g1, b2 ? v2 : g2);
                        }
                        if (n == site) v = apply_fault(v, fbit, fst, t, ft0);
                        const bool dout = active && v != gv;
                        din = din && active;
                        ev += (din || dout) ? 1u : 0u;
                        const uint32_t ew = (din || dout) ? (uint32_t)x.words : 0u;
                        wk += (isreg && din) ? 2u * ew : ew;
                        const uint64_t dm = __ballot(dout);
                        if (dm == 0) continue;
                        val[(size_t)n * 64 + lane] = v;
                        if (lane == 0) mask[n] = LaneMask{dm, stamp};
                        if (dout && (x.flags & DF_PO) && det == RIROS_UNDETECTED) det = t;
                        bool same = false;
                        for (uint32_t e = x.fo0 + lane; e < x.fo1; e += 64) {
                            const uint32_t c = d.fo[e];
                            atomicOr(&bm[c >> 6], 1ull << (c & 63));
                            if ((c >> 6) == w) same = true;
                            else atomicOr(&sm[c >> 12], 1ull << ((c >> 6) & 63));
                        }
                        for (uint32_t e = x.rfo0; e < x.rfo1; ++e) {
                            const uint32_t r = d.rfo[e];
                            const size_t ri = (size_t)q * R + r;
                            rval[ri * 64 + lane] = v;
                            if (lane == 0) {
                                rmask[ri] = LaneMask{dm, stamp + 1};
                                rn[r >> 6] |= 1ull << (r & 63);
                            }
                            rpend = true;
                        }
                        lds_order();
                        if (__ballot(same)) {
                            // users in the word being walked (higher bits)
                            uint64_t more = 0;
                            if (lane == 0) {
                                more = bm[w];
                                bm[w] = 0;
                            }
                            cur |= lane0_u64(more);
                            lds_order();
                        }
                    }
                }
            }
            ++t;
            if (drop) {
                if (det != RIROS_UNDETECTED) active = false;
                if (__ballot(active) == 0) break;
            }
        }
        if (pos < F) {
            detect[fi] = det;
            if (events) events[fi] = ev;
            const uint64_t cycles = (drop && det != RIROS_UNDETECTED) ? (uint64_t)det + 1u : (uint64_t)T;
            words[fi] = wk + cycles * (d.uwidth[faults[fi].site] > 32 ? 2u : 1u);
        }
        base += (uint64_t)T + 1;
    }
    if (lane == 0) st.base[slot] = base;
}

__global__ void k_site_keys(const riros_fault* __restrict__ faults, uint32_t F, uint32_t* __restrict__ keys,
                            uint32_t* __restrict__ idx)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < F) {
        keys[i] = faults[i].site;
        idx[i] = i;
    }
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SimLayout {
    size_t tickets, base, mask, rmask, val, rval, total;
};

SimLayout sim_layout(uint32_t slots, uint32_t N, uint32_t R)
{
    SimLayout l;
    l.tickets = 0;
    l.base = 256;
    l.mask = l.base + align256((size_t)slots * 8);
    l.rmask = l.mask + align256((size_t)slots * N * sizeof(LaneMask));
    l.val = l.rmask + align256((size_t)slots * 2 * R * sizeof(LaneMask));
    l.rval = l.val + align256((size_t)slots * N * 64 * 8);
    l.total = l.rval + align256((size_t)slots * 2 * R * 64 * 8);
    return l;
}

}  // namespace

void conc_free(ConcWorkspace& ws)
{
    if (ws.sim) (void)hipFree(ws.sim);
    if (ws.sort) (void)hipFree(ws.sort);
    ws = ConcWorkspace{};
}

size_t conc_lds_bytes(uint32_t N, uint32_t R)
{
    const size_t NW = (N + 63) / 64, NS = (NW + 63) / 64, RW = (R + 63) / 64;
    return (NW + NS + RW) * sizeof(uint64_t);
}

size_t conc_slot_bytes(uint32_t N, uint32_t R)
{
    return ((size_t)N + 2 * (size_t)R) * (sizeof(LaneMask) + 64 * sizeof(uint64_t)) + sizeof(uint64_t);
}

int run_concurrent(const DevDesign& d, ConcWorkspace& ws, const GoldenView& gv, const riros_fault* faults,
                   uint32_t F, int drop, int waves_per_cu, int num_cu, uint32_t* detect, uint64_t* events,
                   uint64_t* words,
                   hipEvent_t ev0, hipEvent_t ev1, hipStream_t s, std::string& err)
{
    const size_t lds = conc_lds_bytes(d.N, d.R);
    if (lds > 160 * 1024) { err = "design too large for the concurrent kernel's LDS frontier"; return RIROS_EINVAL; }
    if (hipFuncSetAttribute((const void*)k_concurrent, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess) {
        err = "concurrent kernel attribute";
        return RIROS_EDEVICE;
    }
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_concurrent, 64, lds) != hipSuccess || occ < 1) {
        err = "concurrent kernel occupancy";
        return RIROS_EDEVICE;
    }
    const int wpc = waves_per_cu > 0 ? std::min(waves_per_cu, occ) : occ;
    const uint64_t groups = ((uint64_t)F + 63) / 64;
    // Dense faulty state decides how many groups are resident, and
    // residency hides a node's latency: the budget is large, but never more
    // than 60% of the free memory (with the current state counted as free).
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { err = "device memory query"; return RIROS_EDEVICE; }
    const size_t held = (ws.sim && ws.N == d.N && ws.R == d.R) ? ws.sim_bytes : 0;
    const size_t budget = std::min(kConcMaxSimBytes, (free_b + held) / 10 * 6);
    const uint64_t by_mem = budget / conc_slot_bytes(d.N, d.R);
    const uint32_t slots = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(groups, (uint64_t)num_cu * wpc), by_mem);
    if (slots == 0) { err = "design too large for the concurrent mode's faulty state"; return RIROS_ENOMEM; }

    // Faulty state: grown (and its stamps cleared) when a call needs more slots.
    if (!ws.sim || ws.slots < slots || ws.N != d.N || ws.R != d.R) {
        if (hipStreamSynchronize(s) != hipSuccess) { err = "concurrent workspace sync"; return RIROS_EDEVICE; }
        if (ws.sim) (void)hipFree(ws.sim);
        ws.sim = nullptr;
        ws.sim_bytes = 0;
        const SimLayout l = sim_layout(slots, d.N, d.R);
        if (hipMalloc(&ws.sim, l.total) != hipSuccess) {
            ws.sim = nullptr;
            err = "concurrent workspace allocation";
            return RIROS_ENOMEM;
        }
        // stamps and stamp counters start at zero; values need no clearing
        if (hipMemsetAsync(ws.sim, 0, l.val, s) != hipSuccess) { err = "concurrent workspace clear"; return RIROS_EDEVICE; }
        ws.sim_bytes = l.total;
        ws.slots = slots;
        ws.N = d.N;
        ws.R = d.R;
    }
    const SimLayout l = sim_layout(ws.slots, d.N, d.R);
    char* sb = (char*)ws.sim;
    ConcState st{(uint32_t*)(sb + l.tickets), (uint64_t*)(sb + l.base), (LaneMask*)(sb + l.mask),
                 (LaneMask*)(sb + l.rmask), (uint64_t*)(sb + l.val), (uint64_t*)(sb + l.rval)};

    // Fault order: by site, so that faults on one node (and, in the
    // caller's numbering, on nearby nodes) share a group and its frontier.
    size_t temp = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)F, 0, 32, s) !=
        hipSuccess) {
        err = "sort size query failed";
        return RIROS_EDEVICE;
    }
    const size_t fb = align256((size_t)F * 4);
    const size_t need = 4 * fb + align256(temp);
    if (ws.sort_bytes < need) {
        if (ws.sort) (void)hipFree(ws.sort);
        ws.sort = nullptr;
        ws.sort_bytes = 0;
        if (hipMalloc(&ws.sort, need) != hipSuccess) {
            ws.sort = nullptr;
            err = "concurrent sort allocation";
            return RIROS_ENOMEM;
        }
        ws.sort_bytes = need;
    }
    char* ob = (char*)ws.sort;
    uint32_t* keys_in = (uint32_t*)ob;
    uint32_t* keys_out = (uint32_t*)(ob + fb);
    uint32_t* idx = (uint32_t*)(ob + 2 * fb);
    uint32_t* order = (uint32_t*)(ob + 3 * fb);
    if (hipEventRecord(ev0, s) != hipSuccess) { err = "event record"; return RIROS_EDEVICE; }
    if (hipMemsetAsync(st.tickets, 0, sizeof(uint32_t), s) != hipSuccess) { err = "ticket clear"; return RIROS_EDEVICE; }
    hipLaunchKernelGGL(k_site_keys, dim3((F + 255) / 256), dim3(256), 0, s, faults, F, keys_in, idx);
    if (hipcub::DeviceRadixSort::SortPairs(ob + 4 * fb, temp, keys_in, keys_out, idx, order, (int)F, 0, 32, s) !=
        hipSuccess) {
        err = "site sort failed";
        return RIROS_EDEVICE;
    }
    hipLaunchKernelGGL(k_concurrent, dim3(slots), dim3(64), lds, s, d, gv.Gn, gv.Bp, gv.T, gv.TW, faults,
                       (const uint32_t*)order, F, drop, st, detect, events, words);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { err = std::string("concurrent kernel: ") + hipGetErrorString(e); return RIROS_EDEVICE; }
    if (hipEventRecord(ev1, s) != hipSuccess) { err = "event record"; return RIROS_EDEVICE; }
    return RIROS_OK;
}

}  // namespace riros
