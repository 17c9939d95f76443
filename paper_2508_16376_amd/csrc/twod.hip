// Two-dimensional fault simulation (the paper's two-dimensional parallelism,
// Sec. III and IV-C, transposed for a GPU).  Two persistent launches; every
// wavefront takes work from atomic queues:
//   launch A, phase 1: heavy faults placed up front (largest predicted load
//      first), one fault per wavefront, each level's divergent frontier split
//      across the lanes (wave_sim_fault, the structural dimension);
//   launch A, phase 2: light faults, one per lane, each lane walking its own
//      fault's frontier at its own cycle and taking a new fault when it
//      finishes (the fault dimension).  A lane hands its fault over to the
//      structural path when the frontier outgrows the lane's capacity, or when
//      the fault's events per cycle exceed a threshold (a monitor in the spirit
//      of the paper's execution-time-share monitor, Sec. IV-C);
//   launch A, phase 3 (unified schedule, optional): a wavefront whose lanes
//      have run out of light work takes handed-over faults while the other
//      wavefronts are still in phase 2, so long faults start on the
//      structural path as soon as they are handed over (the paper overlaps
//      phases by letting idle workers steal across them, Sec. IV-D);
//   launch B: the handed-over faults nobody took in launch A, one per
//      wavefront, from cycle 0.
// No wavefront waits for another's work, only (boundedly) for new work to
// appear.  Where a fault runs never changes its result.
#include <hipcub/hipcub.hpp>

#include <type_traits>

#include "device_common.hpp"
#include "twod.hpp"
#include "wave_fault.hpp"

namespace riros {

constexpr uint32_t kNone = 0xFFFFFFFFu;

// Counters that different parties hammer sit on separate 128-byte lines, so
// that phase-3 polling never slows the light lanes' atomics.
struct TwoDCounters {
    alignas(128) uint32_t light_head;   // next index into the light queue
    uint32_t heavy_head;                // next index into the up-front heavy queue
    uint32_t n_heavy;                   // faults placed on the heavy queue up front
    alignas(128) uint32_t esc_count;    // faults handed from light lanes to the heavy path
    alignas(128) uint32_t esc_head;     // launch B: next handed-over fault to look at
    uint32_t inflight;                  // light faults taken by a lane and not yet finished or handed over
    uint32_t error;                     // unused (kept zero)
    alignas(128) uint32_t esc_take;     // phase-3 tickets (launch A)
    // Per-XCD light queues (xcd mode): segment x of the light order holds the
    // faults whose site falls to XCD x, [seg_begin[x], seg_end[x]) relative to
    // the light part; seg_head[x] is its next position, one 128-byte line each.
    uint32_t seg_begin[8], seg_end[8];
    struct alignas(128) Head {
        uint32_t v;
    } seg_head[8];
};

// XCD of a fault's site in xcd mode: blocks of 64 consecutive node ids (a
// template's nodes are numbered together) go round-robin to the 8 XCDs.
__host__ __device__ __forceinline__ uint32_t site_xcd(uint32_t site)
{
    return (site >> 6) & 7u;
}

// Lane-private sets, held in registers: every index below is a compile-time
// constant after unrolling, so no array leaves the register file.
template <int C>
struct SortedIds {
    uint32_t v[C];
    uint32_t n;
    // Insert keeping ascending order; duplicates are dropped.  false = full.
    __device__ __forceinline__ bool insert(uint32_t u)
    {
        bool dup = false;
#pragma unroll
        for (int k = 0; k < C; ++k) dup |= ((uint32_t)k < n) && v[k] == u;
        if (dup) return true;
        if (n >= (uint32_t)C) return false;
        uint32_t x = u;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if ((uint32_t)k < n) {
                if (v[k] > x) {
                    const uint32_t tmp = v[k];
                    v[k] = x;
                    x = tmp;
                }
            } else if ((uint32_t)k == n) {
                v[k] = x;
            }
        }
        n++;
        return true;
    }
    __device__ __forceinline__ uint32_t pop_min()
    {
        const uint32_t u = v[0];
#pragma unroll
        for (int k = 0; k + 1 < C; ++k) v[k] = v[k + 1];
        n--;
        return u;
    }
};

// (node id, faulty ^ golden) pairs; V is the value word (uint32_t when no
// node of the design is wider than 32 bits).
template <int C, typename V = uint64_t>
struct DeltaSet {
    uint32_t id[C];
    V dx[C];
    uint32_t n;
    __device__ __forceinline__ bool add(uint32_t i, V x)
    {
        if (n >= (uint32_t)C) return false;
#pragma unroll
        for (int k = 0; k < C; ++k)
            if ((uint32_t)k == n) {
                id[k] = i;
                dx[k] = x;
            }
        n++;
        return true;
    }
    __device__ __forceinline__ V find(uint32_t i, bool& hit) const
    {
        V r = 0;
#pragma unroll
        for (int k = 0; k < C; ++k)
            if (((uint32_t)k < n) && id[k] == i) {
                r = dx[k];
                hit = true;
            }
        return r;
    }
};

__device__ __forceinline__ uint32_t pick4(uint32_t k, uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    return k == 0 ? a : (k == 1 ? b : (k == 2 ? c : d));
}

// A node's golden value in cycle t from the node-major trace: the 64-bit
// word, or (32-bit lanes, every node at most 32 bits wide) the 32-bit copy,
// whose lines hold twice the cycles.
template <typename V>
__device__ __forceinline__ V gold_at(const uint64_t* __restrict__ Gn, const uint32_t* __restrict__ Gn32, size_t i)
{
    if constexpr (sizeof(V) == 8) return Gn[i];
    else return Gn32[i];
}

// The operator table on 32-bit words (every operand and result at most 32
// bits wide): the same results as apply_opw on their zero-extended values.
__device__ __forceinline__ uint32_t apply_opw32(uint32_t op, uint32_t width, uint32_t pb, uint32_t pc, uint32_t x0,
                                                uint32_t x1, uint32_t x2)
{
    uint32_t r;
    switch (op) {
    case RIROS_OP_ADD: r = x0 + x1; break;
    case RIROS_OP_SUB: r = x0 - x1; break;
    case RIROS_OP_AND: r = x0 & x1; break;
    case RIROS_OP_OR: r = x0 | x1; break;
    case RIROS_OP_XOR: r = x0 ^ x1; break;
    case RIROS_OP_NOT: r = ~x0; break;
    case RIROS_OP_MUX: r = x0 != 0 ? x2 : x1; break;
    case RIROS_OP_SHL: r = pb >= 32 ? 0u : (x0 << pb); break;
    case RIROS_OP_SHR:
    case RIROS_OP_SLICE: r = pb >= 32 ? 0u : (x0 >> pb); break;
    case RIROS_OP_EQ: r = x0 == x1; break;
    case RIROS_OP_NE: r = x0 != x1; break;
    case RIROS_OP_ULT: r = x0 < x1; break;
    case RIROS_OP_CONCAT: r = (pc >= 32 ? 0u : (x0 << pc)) | x1; break;
    case RIROS_OP_MUL: r = x0 * x1; break;
    default: r = 0; break;
    }
    return width >= 32 ? r : (r & ((1u << width) - 1u));
}

template <typename V>
__device__ __forceinline__ V apply_op_v(uint32_t op, uint32_t width, uint32_t pb, uint32_t pc, V x0, V x1, V x2)
{
    if constexpr (sizeof(V) == 8) return apply_opw(op, width, pb, pc, x0, x1, x2);
    else return apply_opw32(op, width, pb, pc, x0, x1, x2);
}

template <typename V>
__device__ __forceinline__ V apply_fault_v(V v, uint32_t bit, uint32_t stuck, uint32_t t, uint32_t t0)
{
    const V m = (V)1 << bit;
    if (stuck == RIROS_FAULT_FLIP) return t == t0 ? (v ^ m) : v;
    return stuck ? (v | m) : (v & ~m);
}

// Per-lane view of a fault's design: everything the light path reads.
struct LaneDesign {
    const uint32_t* u2i;
    const LaneRec* rec;
    const uint32_t* fo;
    const uint32_t* rfo;
    const uint32_t* bp_off;
    const uint64_t* Gn;
    const uint64_t* Bp;
    uint32_t T, TW;
    const uint32_t* Gn32;
};

__device__ __forceinline__ LaneDesign lane_design(const DevDesign& d, const GoldenView& g)
{
    return LaneDesign{d.u2i, d.lrec, d.fo, d.rfo, d.bp_off, g.Gn, g.Bp, g.T, g.TW, g.Gn32};
}

// Where a fault's design comes from: the launch's one design, or (batched
// campaigns) a device table indexed by the fault's design id.
struct DesignSrc {
    DevDesign d;
    GoldenView g;
    const DevDesign* td;
    const GoldenView* tg;
    const uint16_t* did;
};

// The site's golden word (one or two words) once per simulated cycle: the
// fault-cycle term of the byte model.
__device__ __forceinline__ uint64_t site_words(int drop, uint32_t det, uint32_t T, uint32_t width)
{
    const uint64_t cycles = (drop && det != RIROS_UNDETECTED) ? (uint64_t)det + 1u : (uint64_t)T;
    return cycles * (width > 32 ? 2u : 1u);
}

// How light lanes take and run their faults (all of it only changes the
// schedule, never a result).
struct LanePolicy {
    int lockstep;          // a lane about to start a cycle waits while another lane of its wavefront is inside one
    uint32_t deal;         // 0, or the group size g of the dealt queue head (a power of two, 4 to 32)
    uint32_t head_lanes;   // 0, or the size of a wavefront's first take, after which it takes nothing until
                           // that batch is finished
    uint32_t xcd;          // 1: per-XCD light queues (the order was partitioned by site_xcd), 0: one queue
};

// Light-queue position p -> the queue index it takes, when the head of the
// queue is dealt out (gshift = log2 of the group size g).  The first
// 64 x chunks positions are read as chunks rows of 64 (a row is what one
// wavefront takes first: its 64 lanes): lane l of row c takes group
// (l / g) * chunks + c of the queue, element l % g.  Row c thus holds group c
// of each of the 64 / g strata of chunks x g consecutive faults, so the
// heaviest faults of a descending order spread over every wavefront instead
// of filling the first ones.  A bijection of [0, 64 x chunks); later
// positions, and every position when chunks = 0, map to themselves.
__device__ __forceinline__ uint32_t dealt(uint32_t p, uint32_t gshift, uint32_t chunks)
{
    if (p >= chunks * 64u) return p;
    const uint32_t c = p >> 6, l = p & 63u;
    return (((l >> gshift) * chunks + c) << gshift) | (l & ((1u << gshift) - 1u));
}

// Phase 2: light faults one per lane.  A lane with no divergent register
// skips straight to the next cycle in which its site is excited (the site's
// bit differs from the stuck value), reading 64 cycles of that bit with one
// load of its bit-plane; only the site can diverge in such a cycle, with
// faulty = golden ^ (1 << bit).  Otherwise the lane evaluates its pending
// nodes in increasing id order (a topological order) from the node-major
// golden values of the operands xor their divergence deltas.  V: the value
// word, uint32_t when no node of the design(s) is wider than 32 bits (half
// the registers and vector instructions per value), else uint64_t.
template <int C, bool BATCH, typename V>
__device__ void light_phase(const DesignSrc& src, const riros_fault* __restrict__ faults,
                            uint32_t nlight, const uint32_t* __restrict__ lorder, TwoDCounters* ctr,
                            uint32_t* __restrict__ esc, int drop, uint32_t* __restrict__ detect_out,
                            uint64_t* __restrict__ events_out, uint64_t* __restrict__ words_out,
                            uint32_t lanes, uint32_t rate_num, LanePolicy lp)
{
    // Register next-state deltas: a pipeline keeps one per divergent stage.
    // Batched lanes hold their design's pointers in registers, so they keep
    // fewer (occupancy stays at three or four wavefronts per SIMD).
    constexpr int CR = BATCH ? C / 2 : (C == 4 ? 4 : (C == 8 ? 6 : 8));
    constexpr uint32_t kPre = 4;
    const uint32_t lane = threadIdx.x & 63;
    // Dealing (deal = g > 0): one row of 64 queue positions per wavefront of
    // the launch, as far as the queue reaches.
    const uint32_t chunks = lp.deal ? min(gridDim.x * (blockDim.x >> 6), nlight >> 6) : 0u;
    const uint32_t gshift = lp.deal ? (uint32_t)__builtin_ctz(lp.deal) : 0u;
    // Head batch (head_lanes = h > 0): the wavefront's first take is h faults
    // (with priorities, h of the heaviest), and it takes no more until all of
    // them are finished, so the heaviest faults run h to a wavefront, beside
    // faults of their own kind only, on up to 64 / h times more wavefronts.
    // 0: first take; 1: holding the head batch; 2: refilling freely.
    uint32_t hstate = lp.head_lanes ? 0u : 2u;
    // Per-XCD queues (xcd mode): workgroups are dispatched to the 8 XCDs
    // round-robin, so this wavefront runs on XCD blockIdx.x % 8 and takes
    // faults from that XCD's segment first, whose sites share that XCD's L2;
    // when a segment runs dry it moves on to the next XCD's (stealing).
    // cseg counts the segments this wavefront has found empty.
    const uint32_t home = blockIdx.x & 7u;
    uint32_t cseg = 0;
    // One design: uniform for the whole wave.  Batched: per lane, per fault.
    LaneDesign d = lane_design(src.d, src.g);

    uint32_t fi = kNone, site = 0, fbit = 0, fval = 0, ft0 = 0, t = 0, det = RIROS_UNDETECTED;
    uint32_t rk = 0;   // next entry of rcur to evaluate in this cycle
    uint64_t ev = 0, wk = 0;   // events and byte-model words of the lane's fault
    bool in_cycle = false;
    uint64_t exw = 0;
    uint32_t ewb = kNone;
    size_t bprow = 0;
    LaneRec srec{};
    bool exhausted = nlight == 0;
    SortedIds<C> pend;
    DeltaSet<C, V> div;
    DeltaSet<CR, V> rcur, rnxt;
    pend.n = div.n = rcur.n = rnxt.n = 0;

    bool finished = false;   // this lane finished or handed over a fault in the last iteration
    // Lanes with 32-bit values and capacity 4 evaluate two nodes per
    // iteration (see below) and keep the record of the last register they
    // evaluated (creg): when that register is the first divergent one of the
    // next cycle, as a latent accumulator's is in every cycle, it is
    // evaluated at the cycle start without loading its record (only its
    // golden word when it is the fault site), and its users go into the same
    // iteration's pair.  Wider values or larger sets leave
    // no registers for either.
    constexpr bool kPair = sizeof(V) == 4 && C <= 4;
    uint32_t creg = kNone;
    LaneRec crec{};
    for (;;) {
        // Count the faults finished in the last iteration out of flight (one
        // atomic per wave), after their hand-overs were performed.
        const uint64_t finm = __ballot(finished);
        if (finm && (int)lane == __ffsll((unsigned long long)finm) - 1) atomicSub(&ctr->inflight, (uint32_t)__popcll(finm));
        finished = false;
        // Refill idle lanes from the light queue (one atomic per wave); only
        // the first `lanes` lanes take work, so that light faults spread over
        // every wavefront of the grid.
        if (hstate == 1 && __ballot(fi != kNone) == 0) hstate = 2;
        const uint32_t cap = hstate == 2 ? lanes : min(lanes, lp.head_lanes);
        const bool need = fi == kNone && lane < cap && hstate != 1;
        const uint64_t needm = __ballot(need && !exhausted);
        if (needm) {
            const uint32_t k = (uint32_t)__popcll(needm);
            const int leader = __ffsll((unsigned long long)needm) - 1;
            uint32_t base = 0, got = 0;
            if ((int)lane == leader) {
                // In flight before taken (the fence waits for the increment),
                // so that a taken fault is always counted: phase 3 ends when
                // the queue is empty and nothing is in flight.
                atomicAdd(&ctr->inflight, k);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                uint32_t taken = 0;
                if (lp.xcd) {
                    while (cseg < 8u) {
                        const uint32_t sg = (home + cseg) & 7u;
                        const uint32_t len = ctr->seg_end[sg] - ctr->seg_begin[sg];
                        const uint32_t b = atomicAdd(&ctr->seg_head[sg].v, k);
                        if (b < len) {
                            taken = min(k, len - b);
                            base = ctr->seg_begin[sg] + b;
                            if (b + k >= len) cseg++;
                            break;
                        }
                        cseg++;
                    }
                    // light_head counts the faults taken (phase 3 ends on it).
                    if (taken) atomicAdd(&ctr->light_head, taken);
                } else {
                    base = atomicAdd(&ctr->light_head, k);
                    taken = base >= nlight ? 0u : min(k, nlight - base);
                }
                if (taken < k) atomicSub(&ctr->inflight, k - taken);
                got = taken;
            }
            base = __shfl(base, leader, 64);
            got = __shfl(got, leader, 64);
            if (lp.xcd) {
                cseg = __shfl(cseg, leader, 64);
                if (cseg >= 8u) exhausted = true;
            } else if (base + k >= nlight) {
                exhausted = true;
            }
            if (need) {
                const uint32_t rank = (uint32_t)__popcll(needm & ((1ull << lane) - 1ull));
                const uint32_t idx = base + rank;
                if (rank < got) {
                    const uint32_t q = lp.xcd ? idx : dealt(idx, gshift, chunks);
                    fi = lorder ? lorder[q] : q;
                    if (BATCH) {
                        const uint32_t k = src.did[fi];
                        d = lane_design(src.td[k], src.tg[k]);
                    }
                    const riros_fault f = faults[fi];
                    site = d.u2i[f.site];
                    fbit = f.bit;
                    fval = f.stuck;
                    ft0 = f.t0;
                    srec = d.rec[site];
                    bprow = (size_t)(d.bp_off[site] + fbit) * d.TW;
                    t = 0;
                    det = RIROS_UNDETECTED;
                    ev = 0;
                    wk = 0;
                    creg = kNone;
                    pend.n = div.n = rcur.n = rnxt.n = 0;
                    rk = 0;
                    in_cycle = false;
                    ewb = kNone;
                }
            }
        }
        if (hstate == 0) hstate = 1;
        if (__ballot(fi != kNone) == 0) break;
        if (fi == kNone) continue;
        // Lockstep (optional): a lane about to start a cycle waits while
        // another lane of the wavefront is still inside one, so that the
        // lanes start their cycles together and walk frontiers of the same
        // shape (faults of one node, or of one template) in step: the same
        // branches, and records and golden lines shared between lanes.
        const uint64_t inside = __ballot(in_cycle);
        if (lp.lockstep && !in_cycle && inside != 0) continue;

        bool esc_now = false;
        // Record a divergent node: keep its delta, schedule its users, stage
        // register next states, note output mismatches.  The first four users
        // and the first register fed come with the node's record.
        auto on_divergent = [&](uint32_t n, V delta, const LaneRec& r) {
            if (!div.add(n, delta)) { esc_now = true; return; }
            if ((r.flags & DF_PO) && det == RIROS_UNDETECTED) det = t;
            for (uint32_t e = r.fo0; e < r.fo1; ++e) {
                const uint32_t k = e - r.fo0;
                const uint32_t u = k < kPre ? pick4(k, r.u[0], r.u[1], r.u[2], r.u[3]) : d.fo[e];
                if (!pend.insert(u)) { esc_now = true; return; }
            }
            for (uint32_t e = r.rfo0; e < r.rfo1; ++e)
                if (!rnxt.add(e == r.rfo0 ? r.r0 : d.rfo[e], delta)) { esc_now = true; return; }
        };

        bool evaluated = false;
        if (!in_cycle) {
            if (rcur.n == 0) {
                // Skip to the next cycle in which the site is excited (a flip:
                // its own cycle only).
                bool found = false;
                const uint32_t T = d.T;
                if (fval == RIROS_FAULT_FLIP) {
                    found = t <= ft0 && ft0 < T;
                    t = ft0;
                }
                while (fval != RIROS_FAULT_FLIP && t < T) {
                    const uint32_t wb = t >> 6;
                    if (wb != ewb) {
                        uint64_t w = d.Bp[bprow + wb];
                        if (fval) w = ~w;
                        const uint32_t valid = T - (wb << 6);
                        if (valid < 64) w &= (1ull << valid) - 1ull;
                        exw = w;
                        ewb = wb;
                    }
                    const uint64_t m = exw >> (t & 63);
                    if (m) {
                        t += (uint32_t)__builtin_ctzll(m);
                        found = true;
                        break;
                    }
                    t = (wb + 1) << 6;
                }
                if (!found) {
                    detect_out[fi] = det;
                    if (events_out) events_out[fi] = ev;
                    words_out[fi] = wk + site_words(drop, det, d.T, srec.width);
                    fi = kNone;
                    finished = true;
                    continue;
                }
                ev++;
                wk += srec.words;
                on_divergent(site, (V)1 << fbit, srec);
                evaluated = true;
            } else {
                // Divergent registers are evaluated first, straight from
                // rcur (registers have the lowest ids, and their order among
                // themselves does not matter); the site joins the pending
                // set unless it is one of them.
                rk = 0;
                bool site_reg = false;
                (void)rcur.find(site, site_reg);
                if (!site_reg && !pend.insert(site)) esc_now = true;
                if (kPair && !esc_now && creg != kNone && rcur.id[0] == creg) {
                    // A register's evaluation: its delta is its staged next
                    // state (an event with a divergent input), and when the
                    // register is the site, that state with the fault
                    // applied to it (which may mask it).
                    V delta = rcur.dx[0];
                    if (creg == site) {
                        const V gv = gold_at<V>(d.Gn, d.Gn32, (size_t)creg * d.T + t);
                        delta = apply_fault_v<V>(gv ^ delta, fbit, fval, t, ft0) ^ gv;
                    }
                    ev++;
                    wk += 2u * crec.words;
                    if (delta != 0) on_divergent(creg, delta, crec);
                    rk = 1;
                }
            }
            in_cycle = true;
        }
        // The cycle-start evaluation of the site's own register can leave
        // nothing to evaluate (no other divergent register, nothing pending).
        if (!evaluated && !esc_now && (rk < rcur.n || pend.n > 0)) {
            // Evaluate the next node (registers of the cycle first, then the
            // lowest pending node: users always have larger ids) and, in the
            // same iteration, the node after it, when that one is still the
            // next once the first's users are scheduled: two registers of a
            // cycle never depend on each other, and a pending node depends on
            // no node other than smaller pending ones and the registers.  For
            // both: the record (with the node's first users) and the node's
            // golden value, then the operands' golden values in one round
            // trip, from the record's operand slots (a slot the operator does
            // not read repeats the first operand, or the node itself), so no
            // load waits for another.
            uint32_t n0 = 0, n1 = kNone;
            bool n1_reg = false;
            if (rk < rcur.n) {
#pragma unroll
                for (int k = 0; k < CR; ++k) {
                    if ((uint32_t)k == rk) n0 = rcur.id[k];
                    if (kPair && (uint32_t)k == rk + 1 && rk + 1 < rcur.n) {
                        n1 = rcur.id[k];
                        n1_reg = true;
                    }
                }
                if (kPair && !n1_reg && pend.n > 0) n1 = pend.v[0];
                rk++;
            } else {
                n0 = pend.pop_min();
                if (kPair && pend.n > 0) n1 = pend.v[0];
            }
            const uint32_t T = d.T;
            const uint32_t m1 = n1 != kNone ? n1 : n0;
            const LaneRec r0 = d.rec[n0];
            const LaneRec r1 = d.rec[m1];
            auto gold = [&](uint32_t m) { return gold_at<V>(d.Gn, d.Gn32, (size_t)m * T + t); };
            const V g0 = gold(n0), g1 = gold(m1);
            const V x00 = gold(r0.o[0]), x01 = gold(r0.o[1]), x02 = gold(r0.o[2]);
            const V x10 = gold(r1.o[0]), x11 = gold(r1.o[1]), x12 = gold(r1.o[2]);
            auto evaluate = [&](uint32_t n, const LaneRec& r, V gv, V x0, V x1, V x2) {
                const bool comb = r.op != RIROS_OP_REG && r.op != RIROS_OP_PI && r.op != RIROS_OP_CONST;
                V delta = 0;
                bool din = false;
                if (r.op == RIROS_OP_REG) {
                    delta = rcur.find(n, din);
                    if (kPair) {
                        creg = n;
                        crec = r;
                    }
                } else if (comb) {
                    // A repeated slot finds what the first one found: din and
                    // the operands the operator reads are exact.
                    x0 ^= div.find(r.o[0], din);
                    x1 ^= div.find(r.o[1], din);
                    x2 ^= div.find(r.o[2], din);
                    delta = apply_op_v<V>(r.op, r.width, r.b, r.c, x0, x1, x2) ^ gv;
                }
                if (n == site) delta = apply_fault_v<V>(gv ^ delta, fbit, fval, t, ft0) ^ gv;
                const bool dout = delta != 0;
                if (din || dout) {
                    ev++;
                    wk += (r.op == RIROS_OP_REG && din) ? 2u * r.words : r.words;
                }
                if (dout) on_divergent(n, delta, r);
            };
            evaluate(n0, r0, g0, x00, x01, x02);
            if (kPair && n1 != kNone && !esc_now && (n1_reg || (rk >= rcur.n && pend.n > 0 && pend.v[0] == n1))) {
                if (n1_reg) rk++;
                else (void)pend.pop_min();
                evaluate(n1, r1, g1, x10, x11, x12);
            }
        }

        // Monitor: a fault averaging more than rate_num/4 events per cycle after
        // its first 8 cycles belongs on the structural path.
        if (!esc_now && rate_num && t >= 8 && ev * 4 > (uint64_t)rate_num * (t + 1)) esc_now = true;
        if (esc_now) {
            const uint32_t slot = atomicAdd(&ctr->esc_count, 1u);
            // A phase-3 wavefront may be waiting for this entry (kNone until
            // written).  The entry itself is the whole message, so a relaxed
            // device-scope store suffices; release or acquire at device scope
            // would write back or invalidate the whole L2 on every access.
            __hip_atomic_store(&esc[slot], fi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            fi = kNone;
            finished = true;
            continue;
        }
        if (in_cycle && pend.n == 0 && rk >= rcur.n) {
            // End of cycle t.
            bool done = drop && det != RIROS_UNDETECTED;
            if (!done) {
                t++;
                div.n = 0;
                rcur = rnxt;
                rnxt.n = 0;
                in_cycle = false;
                done = t >= d.T;
            }
            if (done) {
                detect_out[fi] = det;
                if (events_out) events_out[fi] = ev;
                words_out[fi] = wk + site_words(drop, det, d.T, srec.width);
                fi = kNone;
                finished = true;
            }
        }
    }
}

// Structural path for one fault, on the fault's design: one wavefront, or
// (GROUP) every wavefront of the workgroup.
template <bool BATCH, bool GROUP = false>
__device__ __forceinline__ void heavy_one(const DesignSrc& src, uint32_t fi, const riros_fault* __restrict__ faults,
                                          int drop, const WaveLds& s, Slot* slots, uint64_t* regs,
                                          uint64_t& stamp0, uint32_t* __restrict__ detect_out,
                                          uint64_t* __restrict__ events_out, uint64_t* __restrict__ words_out)
{
    uint32_t det;
    uint64_t ev, wk;
    if (BATCH) {
        const uint32_t k = src.did[fi];
        const DevDesign dd = src.td[k];
        const GoldenView gg = src.tg[k];
        struct_sim_fault<GROUP>(dd, gg.G, gg.Gn, gg.Bp, gg.T, gg.TW, faults[fi], drop, s, slots, regs, stamp0, det, ev,
                                wk);
    } else {
        struct_sim_fault<GROUP>(src.d, src.g.G, src.g.Gn, src.g.Bp, src.g.T, src.g.TW, faults[fi], drop, s, slots, regs,
                                stamp0, det, ev, wk);
    }
    if (GROUP ? threadIdx.x == 0 : (threadIdx.x & 63) == 0) {
        detect_out[fi] = det;
        if (events_out) events_out[fi] = ev;
        words_out[fi] = wk;
    }
}

// Phase 3: take handed-over faults while launch A runs.  A wavefront whose
// lanes have run out of light work takes a ticket: the ticket-th handed-over
// fault is its next one.  It waits (polling its own entry, with backoff) until
// that fault is published, and simulates it; or until light work is over (the
// queue is empty and no lane holds a light fault) and the list ended before
// its ticket (then it leaves); or until a bounded idle time has passed (then
// it leaves its ticket, and launch B simulates the fault if it comes).  A
// simulated entry is overwritten with kDone, which launch B skips.
constexpr uint32_t kDone = 0xFFFFFFFEu;
// Tickets never exceed the hand-overs plus one per workgroup of launch A
// (only its first wavefront takes tickets, and holds at most one unfilled
// ticket), and launch A never has more than kTicketPad workgroups: the list
// has F + kTicketPad entries, all kNone at the start of a run.
constexpr uint32_t kTicketPad = 8192;
// Idle polls back off from one to 32 maximal sleeps (about 3 to 100 us); the
// limit counts sleeps (about a second in all).
constexpr uint32_t kIdleLimit = 1u << 18;

template <bool BATCH>
__device__ void drain_handover(const DesignSrc& src, const riros_fault* __restrict__ faults, uint32_t F,
                               uint32_t nlight, TwoDCounters* ctr, uint32_t* esc, int drop, const WaveLds& s, Slot* slots,
                               uint64_t* regs, uint64_t& stamp0, uint32_t* __restrict__ detect_out,
                               uint64_t* __restrict__ events_out, uint64_t* __restrict__ words_out)
{
    const uint32_t lane = threadIdx.x & 63;
    uint32_t idle = 0;
    for (;;) {
        uint32_t fi = kNone, ticket = 0;
        bool leave = false;
        if (lane == 0) {
            ticket = atomicAdd(&ctr->esc_take, 1u);
            uint32_t backoff = 1;
            // (ticket >= F + kTicketPad cannot happen; leave rather than read past the list.)
            leave = ticket >= F + kTicketPad;
            while (!leave) {
                // Device-scope relaxed atomics throughout: the entry itself is
                // the message, and acquire or release at device scope would
                // write back or invalidate the L2 on every poll.
                const uint32_t v = __hip_atomic_load(&esc[ticket], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (v != kNone) {
                    fi = v;
                    break;
                }
                // Light work is over when the queue is empty and no lane holds
                // a light fault; then esc_count read after it is final.  (Each
                // load completes before the next is issued: the fences only
                // wait.)  This does not depend on every wavefront of the
                // launch being resident.
                const uint32_t lh = __hip_atomic_load(&ctr->light_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const uint32_t inf = __hip_atomic_load(&ctr->inflight, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const uint32_t c = __hip_atomic_load(&ctr->esc_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (ticket < c) continue;   // reserved: the store follows at once
                if (lh >= nlight && inf == 0) {
                    leave = true;
                    break;
                }
                idle += backoff;
                if (idle > kIdleLimit) {
                    leave = true;
                    break;
                }
                for (uint32_t k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(127);
                backoff = min(backoff * 2, 32u);
            }
        }
        fi = __shfl(fi, 0, 64);
        ticket = __shfl(ticket, 0, 64);
        if (__shfl((int)leave, 0, 64)) break;
        heavy_one<BATCH>(src, fi, faults, drop, s, slots, regs, stamp0, detect_out, events_out, words_out);
        if (lane == 0) __hip_atomic_store(&esc[ticket], kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        idle = 0;
    }
}

// Shapes of the largest design of a launch (LDS and workspace are sized by it).
struct MaxShape {
    uint32_t N, L, R;
    uint32_t wpp;   // structural schedule words per pass
};

// STRUCT = false: the launch has no structural work (no heavy prefix and no
// phase 3), so it needs no LDS and its occupancy is bounded by registers
// alone; one wavefront per workgroup.  STRUCT = true: workgroups of 1, 2 or 4
// wavefronts share one structural workspace (the LDS and faulty-value slots
// of one wavefront): wavefront 0 runs phase 1 over the heavy prefix (possibly
// empty), light faults, then phase 3 when `unified`; the others run light
// faults only.  Sharing keeps light lanes resident when the structural LDS of
// a large design would otherwise cap the wavefronts per compute unit.
constexpr uint32_t kMaxShare = 4;

// Capacities up to 8 are held to three wavefronts per SIMD (at most 168
// registers per lane; checked free of spills).  W32: every node of the
// launch's designs is at most 32 bits wide, so light lanes keep 32-bit values.
template <int C, bool BATCH, bool STRUCT, bool W32>
__global__ __launch_bounds__(STRUCT ? 64 * kMaxShare : 64) __attribute__((amdgpu_waves_per_eu(C <= 8 ? 3 : 1)))
void k_twod_a(
    DesignSrc src, MaxShape mx, const riros_fault* __restrict__ faults, uint32_t F,
    const uint32_t* __restrict__ order, TwoDCounters* ctr, uint32_t* __restrict__ esc, int drop, PlainWorkspace ws,
    uint32_t rate_num, int unified, int group_heavy, LanePolicy lp, uint32_t* __restrict__ detect_out,
    uint64_t* __restrict__ events_out, uint64_t* __restrict__ words_out)
{
    if constexpr (STRUCT) {
        extern __shared__ uint32_t lds[];
        const WaveLds s = wave_lds_carve(lds, mx.N, mx.L, mx.R, mx.wpp);
        const uint32_t wave = threadIdx.x >> 6;
        if (wave == 0) wave_lds_clear(s, mx.N, mx.L, mx.R);
        __syncthreads();
        Slot* slots = ws.slots + (size_t)blockIdx.x * mx.N;
        uint64_t* regs = ws.regs + (size_t)blockIdx.x * 2 * mx.R;
        uint64_t stamp0 = *ws.stamp_dev;
        const uint32_t nh = ctr->n_heavy;
        // Phase 1: heavy faults placed up front, each on every wavefront of
        // the workgroup (group_heavy) or on its first wavefront.
        if (group_heavy && blockDim.x > 64) {
            for (;;) {
                if (threadIdx.x == 0) s.flags[kFlagQueue] = atomicAdd(&ctr->heavy_head, 1u);
                __syncthreads();
                const uint32_t idx = s.flags[kFlagQueue];
                __syncthreads();
                if (idx >= nh) break;
                heavy_one<BATCH, true>(src, order ? order[idx] : idx, faults, drop, s, slots, regs, stamp0, detect_out,
                                       events_out, words_out);
            }
        } else if (wave == 0) {
            for (;;) {
                uint32_t idx = 0;
                if (threadIdx.x == 0) idx = atomicAdd(&ctr->heavy_head, 1u);
                idx = __shfl(idx, 0, 64);
                if (idx >= nh) break;
                heavy_one<BATCH>(src, order ? order[idx] : idx, faults, drop, s, slots, regs, stamp0, detect_out,
                                 events_out, words_out);
            }
        }
        // Phase 2: light faults, one per lane; each wavefront takes at most
        // its share of lanes so that light faults spread over every wavefront.
        const uint32_t nlight = F - nh;
        const uint32_t waves = gridDim.x * (blockDim.x >> 6);
        const uint32_t lanes = min(64u, max(1u, (nlight + waves - 1) / waves));
        light_phase<C, BATCH, std::conditional_t<W32, uint32_t, uint64_t>>(
            src, faults, nlight, order ? order + nh : nullptr, ctr, esc, drop, detect_out, events_out, words_out, lanes,
            rate_num, lp);
        if (unified && wave == 0)
            drain_handover<BATCH>(src, faults, F, nlight, ctr, esc, drop, s, slots, regs, stamp0, detect_out,
                                  events_out, words_out);
    } else {
        const uint32_t lanes = min(64u, max(1u, (F + gridDim.x - 1) / gridDim.x));
        light_phase<C, BATCH, std::conditional_t<W32, uint32_t, uint64_t>>(src, faults, F, order, ctr, esc, drop,
                                                                          detect_out, events_out, words_out, lanes,
                                                                          rate_num, lp);
    }
}

// Launch B: the faults handed over in launch A (their list is complete), one
// per workgroup of 64 threads, or of 128 or 256 (GROUP: every wavefront of
// the workgroup on the same fault).  Stamps continue above the largest range
// launch A can have used (span).
template <bool BATCH, bool GROUP>
__global__ __launch_bounds__(GROUP ? 256 : 64) void k_twod_b(DesignSrc src, MaxShape mx,
                                                            const riros_fault* __restrict__ faults,
                                                            TwoDCounters* ctr, const uint32_t* __restrict__ esc,
                                                            int drop, PlainWorkspace ws, uint64_t span,
                                                            uint32_t* __restrict__ detect_out,
                                                            uint64_t* __restrict__ events_out,
                                                            uint64_t* __restrict__ words_out)
{
    extern __shared__ uint32_t lds[];
    const WaveLds s = wave_lds_carve(lds, mx.N, mx.L, mx.R, mx.wpp);
    if (threadIdx.x < 64) wave_lds_clear(s, mx.N, mx.L, mx.R);
    __syncthreads();
    Slot* slots = ws.slots + (size_t)blockIdx.x * mx.N;
    uint64_t* regs = ws.regs + (size_t)blockIdx.x * 2 * mx.R;
    uint64_t stamp0 = *ws.stamp_dev + span;
    const uint32_t n = ctr->esc_count;
    for (;;) {
        uint32_t idx = 0;
        if constexpr (GROUP) {
            if (threadIdx.x == 0) s.flags[kFlagQueue] = atomicAdd(&ctr->esc_head, 1u);
            __syncthreads();
            idx = s.flags[kFlagQueue];
            __syncthreads();
        } else {
            if (threadIdx.x == 0) idx = atomicAdd(&ctr->esc_head, 1u);
            idx = __shfl(idx, 0, 64);
        }
        if (idx >= n) break;
        const uint32_t fi = esc[idx];
        if (fi == kDone) continue;   // simulated in launch A (phase 3)
        heavy_one<BATCH, GROUP>(src, fi, faults, drop, s, slots, regs, stamp0, detect_out, events_out, words_out);
    }
}

// Order: fault indexes sorted by descending priority; the prefix with
// priority > theta is the up-front heavy queue.  The sort key is
//   bit 63      priority > theta (the heavy prefix stays exact),
//   bits 32-62  the priority, ordered, with the low 19 bits of its IEEE
//               pattern dropped (bands about 6% wide: the longest-first order
//               is kept to that resolution),
//   bits 0-31   the complement of the fault's site,
// so that within a band faults on one node, and on nodes numbered together,
// sit next to each other: a wavefront's lanes then take faults whose
// frontiers walk the same nodes (the same records and golden lines, and the
// same branches).
__global__ void k_iota(uint32_t* __restrict__ v, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

__global__ void k_order_keys(const float* __restrict__ priority, const riros_fault* __restrict__ faults, uint32_t n,
                             float theta, int xcd, uint64_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float p = priority[i];
    uint32_t u = __float_as_uint(p);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // IEEE order as unsigned order
    const uint64_t heavy = p > theta ? 1ull : 0ull;
    const uint32_t site = faults[i].site;
    const uint64_t part = xcd ? (uint64_t)site_xcd(site) << 60 : 0ull;
    keys[i] = (heavy << 63) | part | ((uint64_t)(u >> 19) << 32) | (uint64_t)(~site);
    idx[i] = i;
}

// Segment bounds of the per-XCD light queues in a descending order whose keys
// carry site_xcd in bits 60-62 below the heavy bit (after k_count_heavy).
__global__ void k_seg_bounds(const uint64_t* __restrict__ sorted_desc, uint32_t n, TwoDCounters* ctr)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nh = ctr->n_heavy;
    if (i >= n || i < nh) return;
    const uint32_t x = (uint32_t)(sorted_desc[i] >> 60) & 7u;
    if (i == nh || ((uint32_t)(sorted_desc[i - 1] >> 60) & 7u) != x) ctr->seg_begin[x] = i - nh;
    if (i + 1 == n || ((uint32_t)(sorted_desc[i + 1] >> 60) & 7u) != x) ctr->seg_end[x] = i + 1 - nh;
}

__global__ void k_fill_u32(uint32_t* __restrict__ v, uint32_t n, uint32_t x)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = x;
}

__global__ void k_count_heavy(const uint64_t* __restrict__ sorted_desc, uint32_t n, TwoDCounters* ctr)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const bool h = (sorted_desc[i] >> 63) != 0;
        const bool next_h = (i + 1 < n) && (sorted_desc[i + 1] >> 63) != 0;
        if (h && !next_h) ctr->n_heavy = i + 1;
    }
}

__global__ void k_zero_counters(TwoDCounters* ctr)
{
    for (uint32_t i = threadIdx.x; i < sizeof(TwoDCounters) / 4; i += blockDim.x) ((uint32_t*)ctr)[i] = 0;
}

// Reset the per-run counters, keeping the heavy-queue length fixed when the
// campaign was ordered.
__global__ void k_reset_run_counters(TwoDCounters* ctr)
{
    if (threadIdx.x == 0) {
        ctr->light_head = 0;
        ctr->esc_count = 0;
        ctr->heavy_head = 0;
        ctr->esc_head = 0;
        ctr->error = 0;
        ctr->inflight = 0;
        ctr->esc_take = 0;
    }
    if (threadIdx.x < 8) ctr->seg_head[threadIdx.x].v = 0;
}

// Coverage of each design of a campaign: workgroup k reduces faults
// off[k]..off[k+1] with that design's cycle count.
__global__ __launch_bounds__(256) void k_batch_coverage(const uint32_t* __restrict__ detect,
                                                        const uint64_t* __restrict__ events,
                                                        const uint64_t* __restrict__ words,
                                                        const uint32_t* __restrict__ off,
                                                        const GoldenView* __restrict__ tg,
                                                        riros_coverage* __restrict__ cov)
{
    __shared__ unsigned long long red[4][4];
    const uint32_t k = blockIdx.x;
    const uint32_t T = tg[k].T;
    unsigned long long det = 0, fc = 0, ev = 0, wk = 0;
    for (uint32_t i = off[k] + threadIdx.x; i < off[k + 1]; i += blockDim.x) {
        const uint32_t dc = detect[i];
        det += dc != RIROS_UNDETECTED;
        fc += dc != RIROS_UNDETECTED ? (unsigned long long)dc + 1 : T;
        ev += events[i];
        wk += words[i];
    }
    det = wave_sum_u64(det);
    fc = wave_sum_u64(fc);
    ev = wave_sum_u64(ev);
    wk = wave_sum_u64(wk);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = det;
        red[1][w] = fc;
        red[2][w] = ev;
        red[3][w] = wk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cov[k].detected = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        cov[k].total = off[k + 1] - off[k];
        cov[k].fault_cycles = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        cov[k].events = red[2][0] + red[2][1] + red[2][2] + red[2][3];
        cov[k].words = red[3][0] + red[3][1] + red[3][2] + red[3][3];
    }
}

struct TwoDLayout {
    size_t ctr, esc, order, idx, keys_in, keys_out, temp, total;
    size_t temp_bytes;
};

static TwoDLayout layout_for(uint32_t F, size_t temp_bytes)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    TwoDLayout l{};
    size_t o = 0;
    l.ctr = o; o += up(sizeof(TwoDCounters));
    l.esc = o; o += up(((size_t)F + kTicketPad) * 4);
    l.order = o; o += up((size_t)F * 4);
    l.idx = o; o += up((size_t)F * 4);
    l.keys_in = o; o += up((size_t)F * 8);
    l.keys_out = o; o += up((size_t)F * 8);
    l.temp = o; o += up(temp_bytes);
    l.total = o;
    l.temp_bytes = temp_bytes;
    return l;
}

// LDS of the structural path (launch A with structural work, launch B).
static size_t lds_bytes_a(const MaxShape& mx)
{
    return wave_lds_words(mx.N, mx.L, mx.R, mx.wpp) * sizeof(uint32_t);
}
static size_t lds_bytes_b(const MaxShape& mx)
{
    return wave_lds_words(mx.N, mx.L, mx.R, mx.wpp) * sizeof(uint32_t);
}

// Persistent launches never exceed what can be resident at once: the lane
// quota assumes every wavefront of the launch runs from the start.
static uint32_t resident_blocks(const void* kern, size_t lds, uint32_t want, uint32_t threads = 64)
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)threads, lds) != hipSuccess || per_cu <= 0 ||
        cus <= 0)
        return std::max(1u, std::min(want, kTicketPad));
    return std::max(1u, std::min<uint32_t>(std::min(want, kTicketPad), (uint32_t)per_cu * (uint32_t)cus));
}

template <int C, bool BATCH, bool W32>
static const void* kernel_a(bool structural)
{
    return structural ? (const void*)k_twod_a<C, BATCH, true, W32> : (const void*)k_twod_a<C, BATCH, false, W32>;
}

// 32-bit light lanes exist for capacities 4 and 8 (capacity 16 keeps 64-bit
// values).
static const void* kernel_a_any(int cap, bool batch, bool structural, bool w32)
{
    if (batch) {
        if (cap == 16) return kernel_a<16, true, false>(structural);
        if (cap == 4) return w32 ? kernel_a<4, true, true>(structural) : kernel_a<4, true, false>(structural);
        return w32 ? kernel_a<8, true, true>(structural) : kernel_a<8, true, false>(structural);
    }
    if (cap == 16) return kernel_a<16, false, false>(structural);
    if (cap == 4) return w32 ? kernel_a<4, false, true>(structural) : kernel_a<4, false, false>(structural);
    return w32 ? kernel_a<8, false, true>(structural) : kernel_a<8, false, false>(structural);
}

// Launch A's grid for `want` wavefronts: workgroups of 64 * share threads
// (share 0 with structural work: the smallest of 1, 2, 4 that keeps want
// wavefronts resident despite the structural LDS, else 4).
struct GridA {
    uint32_t blocks = 1, threads = 64;
};

static GridA twod_grid_a(int cap, bool batch, bool structural, bool w32, const MaxShape& mx, uint32_t want,
                         int share)
{
    GridA g;
    const void* k = kernel_a_any(cap, batch, structural, w32);
    if (!structural) {
        g.blocks = resident_blocks(k, 0, want);
        return g;
    }
    const size_t lds = lds_bytes_a(mx);
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        g.blocks = std::max(1u, std::min(want, kTicketPad));
        return g;
    }
    uint32_t sh = (uint32_t)share;
    if (sh == 0) {
        sh = kMaxShare;
        for (uint32_t c = 1; c < kMaxShare; c *= 2) {
            const uint32_t wb = (want + c - 1) / c;
            if (resident_blocks(k, lds, wb, 64 * c) * c >= want) {
                sh = c;
                break;
            }
        }
    }
    g.threads = 64 * sh;
    g.blocks = resident_blocks(k, lds, (want + sh - 1) / sh, g.threads);
    return g;
}

// Launch B's kernel for a structural workgroup of `wg` threads (64 = one
// wavefront per fault).
template <bool BATCH>
static const void* kernel_b(uint32_t wg)
{
    return wg > 64 ? (const void*)k_twod_b<BATCH, true> : (const void*)k_twod_b<BATCH, false>;
}

template <bool BATCH>
static void launch_b(uint32_t wg, uint32_t blocks, size_t lds, hipStream_t s, const DesignSrc& src,
                     const MaxShape& mx, const riros_fault* faults, TwoDCounters* ctr, const uint32_t* esc, int drop,
                     const PlainWorkspace& ws, uint64_t span, uint32_t* detect, uint64_t* events, uint64_t* words)
{
    if (wg > 64)
        hipLaunchKernelGGL((k_twod_b<BATCH, true>), dim3(blocks), dim3(wg), lds, s, src, mx, faults, ctr, esc, drop,
                           ws, span, detect, events, words);
    else
        hipLaunchKernelGGL((k_twod_b<BATCH, false>), dim3(blocks), dim3(64), lds, s, src, mx, faults, ctr, esc, drop,
                           ws, span, detect, events, words);
}

template <int C, bool BATCH, bool W32>
static hipError_t launch_twod_c(const DesignSrc& src, const MaxShape& mx, const riros_fault* faults, uint32_t F,
                                const uint32_t* order, bool heavy, int unified, int share, uint32_t heavy_wg,
                                LanePolicy lp, TwoDCounters* ctr, uint32_t* esc, int drop,
                                const PlainWorkspace& ws, uint64_t span, uint32_t blocks, uint32_t rate_num,
                                uint32_t* detect, uint64_t* events,
                                uint64_t* words, hipStream_t s)
{
    const size_t lds = lds_bytes_a(mx), ldsb = lds_bytes_b(mx);
    hipError_t e = hipFuncSetAttribute(kernel_b<BATCH>(heavy_wg), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)ldsb);
    if (e != hipSuccess) return e;
    const bool structural = heavy || unified;
    const GridA ga = twod_grid_a(C, BATCH, structural, W32, mx, blocks, share);
    if (unified)
        hipLaunchKernelGGL(k_fill_u32, dim3((F + kTicketPad + 255) / 256), dim3(256), 0, s, esc, F + kTicketPad, kNone);
    if (structural) {
        hipLaunchKernelGGL((k_twod_a<C, BATCH, true, W32>), dim3(ga.blocks), dim3(ga.threads), lds, s, src, mx, faults, F,
                           order, ctr, esc, drop, ws, rate_num, unified, heavy_wg > 64 ? 1 : 0, lp, detect,
                           events, words);
    } else {
        hipLaunchKernelGGL((k_twod_a<C, BATCH, false, W32>), dim3(ga.blocks), dim3(64), 0, s, src, mx, faults, F, order,
                           ctr, esc, drop, ws, rate_num, 0, 0, lp, detect, events, words);
    }
    const uint32_t wgb = heavy_wg > 64 ? heavy_wg : 64u;
    const uint32_t bb = resident_blocks(kernel_b<BATCH>(wgb), ldsb, blocks, wgb);
    launch_b<BATCH>(wgb, bb, ldsb, s, src, mx, faults, ctr, esc, drop, ws, span, detect, events, words);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_advance_stamp(ws.stamp_dev, 2 * span, s);
}

template <bool BATCH>
static hipError_t launch_twod_any(int cap, bool w32, const DesignSrc& src, const MaxShape& mx,
                                  const riros_fault* faults, uint32_t F, const uint32_t* order, bool heavy, int unified,
                                  int share, uint32_t heavy_wg, LanePolicy lp, TwoDCounters* ctr,
                                  uint32_t* esc, int drop,
                                  const PlainWorkspace& ws, uint64_t span, uint32_t blocks, uint32_t rate_num,
                                  uint32_t* detect, uint64_t* events, uint64_t* words, hipStream_t s)
{
#define RIROS_TWOD_C(CAP, W)                                                                                       \
    launch_twod_c<CAP, BATCH, W>(src, mx, faults, F, order, heavy, unified, share, heavy_wg, lp, ctr, esc,               \
                                 drop,                                                                                \
                                 ws, span,                                                                            \
                                 blocks, rate_num, detect, events, words, s)
    switch (cap) {
    case 4: return w32 ? RIROS_TWOD_C(4, true) : RIROS_TWOD_C(4, false);
    case 16: return RIROS_TWOD_C(16, false);
    default: return w32 ? RIROS_TWOD_C(8, true) : RIROS_TWOD_C(8, false);
    }
#undef RIROS_TWOD_C
}

// Ordering by priority (descending) and the heavy prefix count; outside any
// graph (the sort may use library-internal memory operations).
static int order_by_priority(TwoDWorkspace& ws, const TwoDLayout& lay, const float* priority,
                             const riros_fault* faults, uint32_t F, float theta, int xcd, TwoDCounters* ctr,
                             hipStream_t s, std::string& err)
{
    char* base = (char*)ws.mem;
    uint32_t* idx = (uint32_t*)(base + lay.idx);
    uint64_t* keys_in = (uint64_t*)(base + lay.keys_in);
    uint64_t* keys_out = (uint64_t*)(base + lay.keys_out);
    uint32_t* order = (uint32_t*)(base + lay.order);
    hipLaunchKernelGGL(k_order_keys, dim3((F + 255) / 256), dim3(256), 0, s, priority, faults, F, theta, xcd, keys_in,
                       idx);
    size_t tb = lay.temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(base + lay.temp, tb, keys_in, keys_out, idx, order,
                                                               (int)F, 0, 64, s);
    if (e != hipSuccess) { err = "priority sort failed"; return RIROS_EDEVICE; }
    if (!(theta > 3.0e38f))
        hipLaunchKernelGGL(k_count_heavy, dim3((F + 255) / 256), dim3(256), 0, s, keys_out, F, ctr);
    if (xcd) hipLaunchKernelGGL(k_seg_bounds, dim3((F + 255) / 256), dim3(256), 0, s, keys_out, F, ctr);
    return RIROS_OK;
}

static int ensure_twod_ws(TwoDWorkspace& ws, uint32_t F, bool with_sort, TwoDLayout& lay, std::string& err,
                          hipStream_t s)
{
    size_t temp_bytes = 0;
    if (with_sort) {
        hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, temp_bytes, (const uint64_t*)nullptr,
                                                                   (uint64_t*)nullptr, (const uint32_t*)nullptr,
                                                                   (uint32_t*)nullptr, (int)F, 0, 64, s);
        if (e != hipSuccess) { err = "sort size query failed"; return RIROS_EDEVICE; }
    }
    lay = layout_for(F, temp_bytes);
    if (ws.bytes < lay.total) {
        if (ws.mem) (void)hipFree(ws.mem);
        ws.mem = nullptr;
        ws.bytes = 0;
        if (hipMalloc(&ws.mem, lay.total) != hipSuccess) { err = "two-dimensional workspace allocation"; return RIROS_ENOMEM; }
        ws.bytes = lay.total;
    }
    ws.ctr = ws.mem;
    return RIROS_OK;
}

int run_twod(const DevDesign& d, TwoDWorkspace& ws, const GoldenView& gw, const riros_fault* faults,
             const float* priority, uint32_t F, int drop, const TwoDParams& p, PlainWorkspace heavy_ws,
             uint32_t blocks, uint32_t* detect, uint64_t* events, uint64_t* words, hipEvent_t ev0, hipEvent_t ev1,
             hipStream_t s, std::string& err)
{
    TwoDLayout lay;
    int rc = ensure_twod_ws(ws, F, priority != nullptr, lay, err, s);
    if (rc) return rc;
    char* base = (char*)ws.mem;
    TwoDCounters* ctr = (TwoDCounters*)(base + lay.ctr);
    uint32_t* esc = (uint32_t*)(base + lay.esc);
    if (hipEventRecord(ev0, s) != hipSuccess) { err = "event record"; return RIROS_EDEVICE; }
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, ctr);
    const uint32_t* order = nullptr;
    if (priority) {
        rc = order_by_priority(ws, lay, priority, faults, F, p.theta, p.xcd ? 1 : 0, ctr, s, err);
        if (rc) return rc;
        order = (const uint32_t*)(base + lay.order);
    }
    const uint32_t rate_num = p.monitor_rate > 0.f ? (uint32_t)std::min(4.0e9f, p.monitor_rate * 4.f + 0.5f) : 0u;
    DesignSrc src{d, gw, nullptr, nullptr, nullptr};
    const MaxShape mx{d.N, d.L, d.R, words_per_pass(d.N, d.L, d.R, (uint32_t)std::max(1, p.waves_per_cu))};
    const uint64_t span = (uint64_t)F * gw.T + 1;
    const bool heavy = priority != nullptr && !(p.theta > 3.0e38f);
    hipError_t e = launch_twod_any<false>(p.light_cap, p.w32, src, mx, faults, F, order, heavy, p.unified, p.share,
                                          (uint32_t)p.heavy_wg, LanePolicy{p.lockstep, p.deal, p.head_lanes, p.xcd && priority ? 1u : 0u}, ctr,
                                          esc, drop, heavy_ws, span,
                                          blocks,
                                          rate_num,
                                          detect, events, words, s);
    if (e != hipSuccess) { err = std::string("two-dimensional kernels: ") + hipGetErrorString(e); return RIROS_EDEVICE; }
    if (hipEventRecord(ev1, s) != hipSuccess) { err = "event record"; return RIROS_EDEVICE; }
    return RIROS_OK;
}

hipError_t prepare_twod_batch(BatchPlan& b)
{
    const MaxShape mx{b.Nmax, b.Lmax, b.Rmax, b.wpp};
    hipError_t e = hipSuccess;
    auto attr = [&](const void* f, size_t lds) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
    attr((const void*)k_twod_a<4, true, true, false>, lds_bytes_a(mx));
    attr((const void*)k_twod_a<8, true, true, false>, lds_bytes_a(mx));
    attr((const void*)k_twod_a<16, true, true, false>, lds_bytes_a(mx));
    attr((const void*)k_twod_a<4, true, true, true>, lds_bytes_a(mx));
    attr((const void*)k_twod_a<8, true, true, true>, lds_bytes_a(mx));
    attr((const void*)k_twod_b<true, false>, lds_bytes_b(mx));
    attr((const void*)k_twod_b<true, true>, lds_bytes_b(mx));
    if (e == hipSuccess) {
        const GridA ga = twod_grid_a(b.light_cap, true, b.heavy || b.unified, b.w32 && b.light_cap != 16, mx, b.blocks,
                                     b.share);
        b.blocks_a = ga.blocks;
        b.threads_a = ga.threads;
        const uint32_t wgb = b.heavy_wg > 64 ? b.heavy_wg : 64u;
        b.blocks_b = resident_blocks(kernel_b<true>(wgb), lds_bytes_b(mx), b.blocks, wgb);
    }
    return e;
}

int order_batch(TwoDWorkspace& ws, const float* priority, const riros_fault* faults, uint32_t F, float theta, int xcd,
                const uint32_t** order, hipStream_t s, std::string& err)
{
    TwoDLayout lay;
    int rc = ensure_twod_ws(ws, F, priority != nullptr, lay, err, s);
    if (rc) return rc;
    char* base = (char*)ws.mem;
    TwoDCounters* ctr = (TwoDCounters*)(base + lay.ctr);
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, ctr);
    *order = nullptr;
    if (priority) {
        rc = order_by_priority(ws, lay, priority, faults, F, theta, xcd, ctr, s, err);
        if (rc) return rc;
        *order = (const uint32_t*)(base + lay.order);
    }
    return RIROS_OK;
}

hipError_t launch_twod_batch(const BatchPlan& b, TwoDWorkspace& ws, hipStream_t s)
{
    const TwoDLayout lay = layout_for(b.F, 0);
    char* base = (char*)ws.mem;
    TwoDCounters* ctr = (TwoDCounters*)(base + lay.ctr);
    uint32_t* esc = (uint32_t*)(base + lay.esc);
    hipLaunchKernelGGL(k_reset_run_counters, dim3(1), dim3(64), 0, s, ctr);
    DesignSrc src{b.td_host0, b.tg_host0, b.td, b.tg, b.did};
    const MaxShape mx{b.Nmax, b.Lmax, b.Rmax, b.wpp};
    const size_t lds = lds_bytes_a(mx), ldsb = lds_bytes_b(mx);
#define RIROS_LAUNCH_A(CAP, HV, L, W)                                                                        \
    hipLaunchKernelGGL((k_twod_a<CAP, true, HV, W>), dim3(b.blocks_a), dim3(HV ? b.threads_a : 64), L, s, src, mx,  \
                       b.faults, b.F, b.order,                                                                   \
                       ctr, esc, b.drop, b.ws, b.rate_num, b.unified, b.heavy_wg > 64 ? 1 : 0,                       \
                       LanePolicy{b.lockstep, b.deal, b.head_lanes, b.xcd && b.order ? 1u : 0u},                                             \
                       b.detect,                                                                                  \
                       b.events,                                                                                  \
                       b.words)
    if (b.unified)
        hipLaunchKernelGGL(k_fill_u32, dim3((b.F + kTicketPad + 255) / 256), dim3(256), 0, s, esc, b.F + kTicketPad,
                           kNone);
    if (b.heavy || b.unified) {
        switch (b.light_cap) {
        case 4: if (b.w32) RIROS_LAUNCH_A(4, true, lds, true); else RIROS_LAUNCH_A(4, true, lds, false); break;
        case 16: RIROS_LAUNCH_A(16, true, lds, false); break;
        default: if (b.w32) RIROS_LAUNCH_A(8, true, lds, true); else RIROS_LAUNCH_A(8, true, lds, false); break;
        }
    } else {
        switch (b.light_cap) {
        case 4: if (b.w32) RIROS_LAUNCH_A(4, false, 0, true); else RIROS_LAUNCH_A(4, false, 0, false); break;
        case 16: RIROS_LAUNCH_A(16, false, 0, false); break;
        default: if (b.w32) RIROS_LAUNCH_A(8, false, 0, true); else RIROS_LAUNCH_A(8, false, 0, false); break;
        }
    }
#undef RIROS_LAUNCH_A
    launch_b<true>(b.heavy_wg > 64 ? b.heavy_wg : 64u, b.blocks_b, ldsb, s, src, mx, b.faults, ctr, esc, b.drop, b.ws,
                   b.span, b.detect, b.events, b.words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_advance_stamp(b.ws.stamp_dev, 2 * b.span, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_coverage, dim3(b.n), dim3(256), 0, s, b.detect, b.events, b.words, b.off, b.tg, b.cov);
    return hipGetLastError();
}

int twod_check(const TwoDWorkspace& ws, hipStream_t s, std::string& err)
{
    TwoDCounters c;
    if (hipMemcpyAsync(&c, ws.ctr, sizeof c, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        err = "counter read";
        return RIROS_EDEVICE;
    }
    if (c.esc_head < c.esc_count) {
        err = "handed-over faults left unsimulated";
        return RIROS_EDEVICE;
    }
    return RIROS_OK;
}

void twod_free(TwoDWorkspace& ws)
{
    if (ws.mem) (void)hipFree(ws.mem);
    ws.mem = nullptr;
    ws.bytes = 0;
    ws.ctr = nullptr;
}

}  // namespace riros
