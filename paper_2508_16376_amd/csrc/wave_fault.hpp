// One faulty machine simulated by one wavefront, or by a whole workgroup of
// two or four wavefronts, the divergent frontier of each level split across
// their lanes (the structural parallelism of the paper, Sec. IV-C, applied to
// a single fault: one fault's load spread over many workers).
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace riros {

// Schedule words read per pass (one per lane, 64 or 16) fill a compacted
// list of up to 32 nodes a word.  The list takes 8 KB of LDS at 64 words and
// 2 KB at 16; with the bitmaps it decides how many structural wavefronts fit
// on a compute unit, so the host takes 16 when 64 would cap the wavefronts it
// wants resident (a dense level then takes more passes of up to 512 nodes).
constexpr uint32_t kWordsWide = 64, kWordsNarrow = 16;
// Any other value is taken as the narrow pass (a pass of zero words would
// never advance).
__host__ __device__ constexpr uint32_t norm_wpp(uint32_t wpp) { return wpp == kWordsWide ? kWordsWide : kWordsNarrow; }

// LDS of one structural workspace (a wavefront, or a workgroup that runs one
// fault): sched[N/32] nodes to evaluate this cycle, with ssum one bit per
// non-empty sched word (a sparse frontier in a wide level is found without
// scanning the level's words); lvlm[L/32] levels holding scheduled nodes;
// rcur/rnext[R/32] registers whose state diverges in this / the next cycle,
// with summaries rcsum/rnsum; list[32 * wpp] compacted node ids; flags[8]
// (an output was divergent, then the values a workgroup's first wavefront
// hands to the others); lvloff[L+1] the design's level offsets (read once per
// fault, not per level).
constexpr uint32_t kFlagWords = 8;
enum : uint32_t { kFlagPo = 0, kFlagAnyReg, kFlagLevel, kFlagWord, kFlagTotal, kFlagQueue };
struct WaveLds {
    uint32_t* sched;
    uint32_t* ssum;
    uint32_t* lvlm;
    uint32_t* rcur;
    uint32_t* rnext;
    uint32_t* rcsum;
    uint32_t* rnsum;
    uint32_t* list;
    uint32_t* flags;
    uint32_t* lvloff;
    uint32_t wpp;   // schedule words per pass
};

__host__ __device__ inline size_t wave_lds_words(uint32_t N, uint32_t L, uint32_t R, uint32_t wpp)
{
    const size_t W = (N + 31) / 32, WR = (R + 31) / 32;
    return W + (W + 31) / 32 + (L + 31) / 32 + 2 * WR + 2 * ((WR + 31) / 32) + 32 * (size_t)norm_wpp(wpp) +
           kFlagWords + (L + 1);
}

// Words per pass for a design: the wide pass unless its LDS would keep fewer
// than `want` structural wavefronts resident per compute unit.
inline uint32_t words_per_pass(uint32_t N, uint32_t L, uint32_t R, uint32_t want)
{
    constexpr size_t kLdsPerCu = 160 * 1024;
    const size_t wide = wave_lds_words(N, L, R, kWordsWide) * sizeof(uint32_t);
    return kLdsPerCu / wide >= want ? kWordsWide : kWordsNarrow;
}

__device__ inline WaveLds wave_lds_carve(uint32_t* base, uint32_t N, uint32_t L, uint32_t R, uint32_t wpp)
{
    const uint32_t W = (N + 31) / 32, WL = (L + 31) / 32, WR = (R + 31) / 32;
    WaveLds s;
    s.sched = base;
    s.ssum = s.sched + W;
    s.lvlm = s.ssum + (W + 31) / 32;
    s.rcur = s.lvlm + WL;
    s.rnext = s.rcur + WR;
    s.rcsum = s.rnext + WR;
    s.rnsum = s.rcsum + (WR + 31) / 32;
    s.list = s.rnsum + (WR + 31) / 32;
    s.flags = s.list + 32 * norm_wpp(wpp);
    s.lvloff = s.flags + kFlagWords;
    s.wpp = norm_wpp(wpp);
    return s;
}

__device__ inline void wave_lds_clear(const WaveLds& s, uint32_t N, uint32_t L, uint32_t R)
{
    const uint32_t W = (N + 31) / 32, WL = (L + 31) / 32, WR = (R + 31) / 32;
    const uint32_t lane = threadIdx.x & 63;
    // sched, ssum and lvlm are contiguous, and so are rcur, rnext, rcsum, rnsum
    const uint32_t a = W + (W + 31) / 32 + WL, b = 2 * WR + 2 * ((WR + 31) / 32);
    for (uint32_t i = lane; i < a; i += 64) s.sched[i] = 0;
    for (uint32_t i = lane; i < b; i += 64) s.rcur[i] = 0;
}

// Orders the LDS (and workgroup-local global) accesses of the lanes that run
// one fault: a wave-level fence for one wavefront (other wavefronts of its
// workgroup may run other work), a workgroup barrier for a whole workgroup.
template <bool GROUP>
__device__ __forceinline__ void struct_sync()
{
    if constexpr (GROUP) __syncthreads();
    else wave_lds_sync();
}

// Simulate fault f from cycle 0 (drop: stop after the detect cycle).  slots
// is the workspace's [N] faulty-value array, regs its [2][R] register
// next-state ping-pong; stamp0 advances by T.  Returns the detect cycle
// (uniform), the event count and the byte-model words (totals over the
// lanes; the words count each event's NodeRec::words, a register event with
// divergent state twice, and the site's golden word once per simulated
// cycle).
//
// GROUP = false: called by all 64 lanes of one wavefront; other wavefronts
// of its workgroup may run other work (LDS accesses are ordered with
// wave_lds_sync, never a workgroup barrier).
// GROUP = true: called by every thread of the workgroup (2 or 4 wavefronts).
// The first wavefront keeps the schedule (register sets, level and word
// search, compaction of each pass) and hands its decisions to the others
// through flags; every pass's frontier is then evaluated by all the
// workgroup's lanes, with a barrier after it.  Every loop bound the threads
// test is read after a barrier from the same LDS word, so all threads reach
// the same barriers.
template <bool GROUP>
__device__ inline void struct_sim_fault(const DevDesign& d, const uint64_t* __restrict__ Gr,
                                        const uint64_t* __restrict__ Gn,
                                        const uint64_t* __restrict__ Bp, uint32_t T, uint32_t TW,
                                        const riros_fault f, int drop, const WaveLds& s,
                                        Slot* __restrict__ slots, uint64_t* __restrict__ regs,
                                        uint64_t& stamp0, uint32_t& det_out, uint64_t& ev_out,
                                        uint64_t& words_out)
{
    // The LDS arrays as local values rather than fields read through a
    // reference: code that chooses between two of them then selects
    // registers, where a choice between two fields' addresses would keep the
    // structure in scratch memory and reload a pointer on every use.
    uint32_t* const sched = s.sched;
    uint32_t* const ssum = s.ssum;
    uint32_t* const lvlm = s.lvlm;
    uint32_t* const rcur = s.rcur;
    uint32_t* const rnext = s.rnext;
    uint32_t* const rcsum = s.rcsum;
    uint32_t* const rnsum = s.rnsum;
    uint32_t* const list = s.list;
    uint32_t* const flags = s.flags;
    uint32_t* const lvloff = s.lvloff;
    const uint32_t wpp = s.wpp;
    const uint32_t R = d.R;
    const uint32_t WL = (d.L + 31) / 32, WR = (R + 31) / 32, WRS = (WR + 31) / 32;
    const uint32_t lane = threadIdx.x & 63;
    // Thread index and count among the lanes that run this fault; lead: the
    // wavefront that keeps the schedule.
    const uint32_t gtid = GROUP ? threadIdx.x : lane;
    const uint32_t gsize = GROUP ? blockDim.x : 64u;
    const bool lead = GROUP ? threadIdx.x < 64 : true;
    const uint32_t site = d.u2i[f.site];
    const uint32_t site_lvl = d.level[site];
    const uint32_t fbit = f.bit, fval = f.stuck, ft0 = f.t0;
    const uint64_t* __restrict__ srow = Bp + (size_t)(d.bp_off[site] + fbit) * TW;   // the site bit, 64 cycles a word
    // Register state left by the previous fault on this workspace: clear the
    // words the summaries point at.
    if (lead) {
        for (uint32_t j = lane; j < WRS; j += 64) {
            for (uint32_t m = rcsum[j]; m; m &= m - 1) rcur[j * 32 + __ffs(m) - 1] = 0;
            for (uint32_t m = rnsum[j]; m; m &= m - 1) rnext[j * 32 + __ffs(m) - 1] = 0;
            rcsum[j] = 0;
            rnsum[j] = 0;
        }
    }
    for (uint32_t i = gtid; i <= d.L; i += gsize) lvloff[i] = d.lvl_off[i];
    uint32_t ev = 0, wk = 0;
    uint32_t det = RIROS_UNDETECTED;
    struct_sync<GROUP>();
    for (uint32_t t = 0; t < T; ++t) {
        // Cycle start: registers whose D diverged last cycle are scheduled.
        // Lane j of the lead wavefront owns summary word j, hence register
        // words 32j..32j+31 and the sched summary word j (registers have the
        // lowest ids).
        uint32_t any = 0;
        if (lead) {
            for (uint32_t j = lane; j < WRS; j += 64) {
                for (uint32_t m = rcsum[j]; m; m &= m - 1) rcur[j * 32 + __ffs(m) - 1] = 0;
                const uint32_t nm = rnsum[j];
                for (uint32_t m = nm; m; m &= m - 1) {
                    const uint32_t i = j * 32 + __ffs(m) - 1;
                    const uint32_t v = rnext[i];
                    rcur[i] = v;
                    rnext[i] = 0;
                    sched[i] |= v;
                    any |= v;
                }
                rcsum[j] = nm;
                rnsum[j] = 0;
                ssum[j] |= nm;
            }
        }
        bool anyreg;
        if constexpr (GROUP) {
            if (lead) {
                const bool b = __ballot(any != 0) != 0;
                if (lane == 0) flags[kFlagAnyReg] = b ? 1u : 0u;
            }
            struct_sync<GROUP>();
            anyreg = flags[kFlagAnyReg] != 0;
        } else {
            anyreg = __ballot(any != 0) != 0;
        }
        if (!anyreg) {
            // No divergent state: the machine equals the golden one until the
            // site is next excited (its golden bit differs from the stuck
            // value; a flip, only in its cycle), so jump there; no event and
            // no detection in between.  Every thread reads the same words.
            bool found = false;
            if (fval == RIROS_FAULT_FLIP) {
                found = t <= ft0 && ft0 < T;
                t = ft0;
            }
            while (fval != RIROS_FAULT_FLIP && t < T) {
                const uint32_t wb = t >> 6;
                uint64_t w = srow[wb];
                if (fval) w = ~w;
                const uint32_t valid = T - (wb << 6);
                if (valid < 64) w &= (1ull << valid) - 1ull;
                const uint64_t m = w >> (t & 63);
                if (m) {
                    t += (uint32_t)__builtin_ctzll(m);
                    found = true;
                    break;
                }
                t = (wb + 1) << 6;
            }
            if (!found) break;
        }
        const uint64_t stamp = stamp0 + t + 1;
        const uint64_t* rst = regs + (size_t)(t & 1) * R;
        uint64_t* rnx = regs + (size_t)((t + 1) & 1) * R;
        if (gtid == 0) flags[kFlagPo] = 0;
        struct_sync<GROUP>();
        if (gtid == 0) {
            sched[site >> 5] |= 1u << (site & 31);
            ssum[site >> 10] |= 1u << ((site >> 5) & 31);
            lvlm[site_lvl >> 5] |= 1u << (site_lvl & 31);
            if (anyreg) lvlm[0] |= 1u;
        }
        struct_sync<GROUP>();
        for (;;) {
            // Lowest level with scheduled nodes (users are always at higher levels).
            int lv = -1;
            if (lead) {
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
            }
            if constexpr (GROUP) {
                if (gtid == 0) flags[kFlagLevel] = (uint32_t)lv;
                struct_sync<GROUP>();
                lv = (int)flags[kFlagLevel];
            }
            if (lv < 0) break;
            struct_sync<GROUP>();
            if (gtid == 0) lvlm[lv >> 5] &= ~(1u << (lv & 31));
            const uint32_t lo = lvloff[lv], hi = lvloff[lv + 1];
            const uint32_t w0 = lo >> 5, w1 = (hi - 1) >> 5, s1 = w1 >> 5;
            uint32_t wb = w0;
            for (;;) {
                // Next non-empty sched word at or after wb, from the summary
                // (64 summary words, 65,536 nodes, per probe).
                uint32_t nw = 0xFFFFFFFFu;
                if (lead) {
                    for (uint32_t sb = wb >> 5; sb <= s1; sb += 64) {
                        const uint32_t sw = sb + lane;
                        uint32_t sm = sw <= s1 ? ssum[sw] : 0u;
                        if (sw == (wb >> 5)) sm &= ~0u << (wb & 31);
                        const uint64_t bal = __ballot(sm != 0);
                        if (bal) {
                            const int first = __ffsll((unsigned long long)bal) - 1;
                            const uint32_t mw = __shfl(sm, first, 64);
                            nw = (sb + (uint32_t)first) * 32 + (uint32_t)(__ffs(mw) - 1);
                            break;
                        }
                    }
                }
                if constexpr (GROUP) {
                    if (gtid == 0) flags[kFlagWord] = nw;
                    struct_sync<GROUP>();
                    nw = flags[kFlagWord];
                }
                if (nw > w1) break;
                wb = nw;
                // Words wb..wb+wpp-1 of this level: one per lane of the lead
                // wavefront, compacted into list.
                const uint32_t w = wb + lane;
                uint32_t bits = 0;
                if (lead && lane < wpp && w <= w1) {
                    uint32_t m = ~0u;
                    if (w == w0) m &= ~0u << (lo & 31);
                    if (w == w1 && (hi & 31)) m &= (1u << (hi & 31)) - 1u;
                    const uint32_t word = sched[w];
                    bits = word & m;
                    if (bits) {
                        sched[w] = word & ~m;
                        if ((word & ~m) == 0) atomicAnd(&ssum[w >> 5], ~(1u << (w & 31)));
                    }
                }
                wb += wpp;
                uint32_t total = 0;
                if constexpr (GROUP) {
                    if (lead) {
                        const uint32_t cnt = __popc(bits);
                        const uint32_t incl = wave_incl_scan(cnt);
                        total = __shfl(incl, 63, 64);
                        uint32_t off = incl - cnt;
                        while (bits) {
                            const int b = __ffs(bits) - 1;
                            bits &= bits - 1;
                            list[off++] = w * 32 + (uint32_t)b;
                        }
                        if (lane == 0) flags[kFlagTotal] = total;
                    }
                    struct_sync<GROUP>();
                    total = flags[kFlagTotal];
                    if (total == 0) continue;   // only other levels' nodes in these words
                } else {
                    if (__ballot(bits != 0) == 0) continue;   // only other levels' nodes in these words
                    const uint32_t cnt = __popc(bits);
                    const uint32_t incl = wave_incl_scan(cnt);
                    total = __shfl(incl, 63, 64);
                    uint32_t off = incl - cnt;
                    while (bits) {
                        const int b = __ffs(bits) - 1;
                        bits &= bits - 1;
                        list[off++] = w * 32 + (uint32_t)b;
                    }
                    wave_lds_sync();
                }
                // A dense pass (more nodes than lanes) reads golden values from
                // the cycle-major trace, where a level's nodes are neighbours
                // and the cycle's row is shared by every fault near that
                // cycle; a sparse one from the node-major trace, where a node
                // keeps its line for sixteen cycles.
                const bool dense = total > 64;
                auto goldp = [&](uint32_t n) { return dense ? Gr[(size_t)t * d.N + n] : Gn[(size_t)n * T + t]; };
                for (uint32_t i = gtid; i < total; i += gsize) {
                    const uint32_t n = list[i];
                    // Two dependent round trips per node: the record (descriptor + fan-out ranges,
                    // with the node's own golden value beside it), then everything the record
                    // points at, issued together and combined with selects rather than branches,
                    // so that no load waits for another: operand slots and golden values (an
                    // operand slot the operator does not read repeats the first operand, or the
                    // node itself), and the first fan-out entries (the tables end in padding).
                    // (A per-wave LDS cache of records and of the active set's golden and faulty
                    // values was measured slower: the LDS it takes costs more occupancy than it
                    // saves latency.)
                    const NodeRec x = d.rec[n];
                    const uint64_t gv = goldp(n);
                    const bool comb = x.op != RIROS_OP_REG && x.op != RIROS_OP_PI && x.op != RIROS_OP_CONST;
                    const int ar = comb ? dev_arity(x.op) : 0;
                    const uint32_t i0 = ar > 0 ? x.a : n;
                    const uint32_t i1 = ar > 1 ? x.b : i0;
                    const uint32_t i2 = ar > 2 ? x.c : i0;
                    const Slot s0 = slots[i0], s1 = slots[i1], s2 = slots[i2];
                    const uint64_t g0 = goldp(i0), g1 = goldp(i1), g2 = goldp(i2);
                    const uint64_t pk0 = d.fo_pk[x.fo0], pk1 = d.fo_pk[x.fo0 + 1];
                    const uint64_t pk2 = d.fo_pk[x.fo0 + 2], pk3 = d.fo_pk[x.fo0 + 3];
                    const uint32_t rf0 = d.rfo[x.rfo0];
                    const bool d0 = ar > 0 && s0.stamp == stamp;
                    const bool d1 = ar > 1 && s1.stamp == stamp;
                    const bool d2 = ar > 2 && s2.stamp == stamp;
                    bool din = d0 || d1 || d2;
                    uint64_t v = apply_opw(x.op, x.width, x.b, x.c, d0 ? s0.v : g0, d1 ? s1.v : g1, d2 ? s2.v : g2);
                    if (!comb) {
                        v = gv;
                        if (x.op == RIROS_OP_REG) {
                            din = (rcur[n >> 5] >> (n & 31)) & 1u;
                            if (din) v = rst[n];
                        }
                    }
                    if (n == site) v = apply_fault(v, fbit, fval, t, ft0);
                    const bool dout = v != gv;
                    ev += (din || dout) ? 1u : 0u;
                    const uint32_t ew = (din || dout) ? (uint32_t)x.words : 0u;
                    wk += (x.op == RIROS_OP_REG && din) ? 2u * ew : ew;
                    if (dout) {
                        Slot sl;
                        sl.v = v;
                        sl.stamp = stamp;
                        slots[n] = sl;
                        if (x.flags & DF_PO) flags[kFlagPo] = 1;
                        for (uint32_t e = x.fo0; e < x.fo1; ++e) {
                            const uint32_t k = e - x.fo0;
                            const uint64_t pk = k == 0 ? pk0 : k == 1 ? pk1 : k == 2 ? pk2 : k == 3 ? pk3 : d.fo_pk[e];
                            const uint32_t c = (uint32_t)pk, lc = (uint32_t)(pk >> 32);
                            atomicOr(&sched[c >> 5], 1u << (c & 31));
                            atomicOr(&ssum[c >> 10], 1u << ((c >> 5) & 31));
                            atomicOr(&lvlm[lc >> 5], 1u << (lc & 31));
                        }
                        for (uint32_t e = x.rfo0; e < x.rfo1; ++e) {
                            const uint32_t r = e == x.rfo0 ? rf0 : d.rfo[e];
                            rnx[r] = v;
                            atomicOr(&rnext[r >> 5], 1u << (r & 31));
                            atomicOr(&rnsum[r >> 10], 1u << ((r >> 5) & 31));
                        }
                    }
                }
                struct_sync<GROUP>();
            }
        }
        if (flags[kFlagPo] && det == RIROS_UNDETECTED) det = t;
        struct_sync<GROUP>();
        if (drop && det != RIROS_UNDETECTED) break;
    }
    stamp0 += T;
    det_out = det;
    uint64_t evs = wave_sum_u64((uint64_t)ev), wks = wave_sum_u64((uint64_t)wk);
    if constexpr (GROUP) {
        // Sum the wavefronts' totals through the (idle) list array.
        const uint32_t wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
        if (lane == 0) {
            list[4 * wave] = (uint32_t)evs;
            list[4 * wave + 1] = (uint32_t)(evs >> 32);
            list[4 * wave + 2] = (uint32_t)wks;
            list[4 * wave + 3] = (uint32_t)(wks >> 32);
        }
        __syncthreads();
        evs = 0;
        wks = 0;
        for (uint32_t k = 0; k < nwaves; ++k) {
            evs += make_u64(list[4 * k], list[4 * k + 1]);
            wks += make_u64(list[4 * k + 2], list[4 * k + 3]);
        }
        __syncthreads();
    }
    ev_out = evs;
    const uint64_t cycles = (drop && det != RIROS_UNDETECTED) ? (uint64_t)det + 1u : (uint64_t)T;
    words_out = wks + cycles * (d.uwidth[f.site] > 32 ? 2u : 1u);
}

// One fault on one wavefront.
__device__ __forceinline__ void wave_sim_fault(const DevDesign& d, const uint64_t* __restrict__ Gr,
                                               const uint64_t* __restrict__ Gn,
                                               const uint64_t* __restrict__ Bp, uint32_t T, uint32_t TW,
                                               const riros_fault f, int drop, const WaveLds& s,
                                               Slot* __restrict__ slots, uint64_t* __restrict__ regs,
                                               uint64_t& stamp0, uint32_t& det_out, uint64_t& ev_out,
                                               uint64_t& words_out)
{
    struct_sim_fault<false>(d, Gr, Gn, Bp, T, TW, f, drop, s, slots, regs, stamp0, det_out, ev_out, words_out);
}

}  // namespace riros
