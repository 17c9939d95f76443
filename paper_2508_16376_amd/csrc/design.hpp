// Host-side design compiler: validation, levelisation, level-major
// renumbering and the fan-out tables the kernels walk.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "riros.h"

namespace riros {

// 16-byte node descriptor in internal (level-major) numbering.
//   comb ops    a, b, c = operand ids (per arity); SHL/SHR/SLICE: b = shift
//               (clamped to 64); CONCAT: c = width of operand b
//   PI          a = stimulus column
//   CONST       a, b = value (low, high word)
//   REG         a = D node; b, c = reset value (low, high word)
struct Desc {
    uint8_t op, width, flags, pad;
    uint32_t a, b, c;
};
static_assert(sizeof(Desc) == 16, "descriptor layout");

enum : uint8_t { DF_PO = 1, DF_REGFO = 2, DF_COMBFO = 4 };

// Zero entries after the last fan-out entry of fo, fo_pk and rfo.
constexpr uint32_t kFanoutPad = 4;

// 32-byte node record for per-lane walks: the descriptor plus the node's
// fan-out ranges, so one load gives everything needed to evaluate a node and
// schedule its users.  `words` is the node's share of the byte model (memory
// words an evaluation of the node must touch, counted per event; see
// event_words).
struct NodeRec {
    uint8_t op, width, flags, words;
    uint32_t a, b, c;
    uint32_t fo0, fo1;     // combinational users: fo[fo0..fo1)
    uint32_t rfo0, rfo1;   // registers fed: rfo[rfo0..rfo1)
};
static_assert(sizeof(NodeRec) == 32, "record layout");

// 64-byte record of the light (one fault per lane) path: the node record
// plus the first four entries of the node's combinational fan-out and the
// first register it feeds (the tables' padding where the lists are
// shorter), so that a lane evaluating the node gets its users in the same
// round trip as its operands' ids, and only the operands' golden values take
// a second one.  o[3] are the nodes whose golden values the evaluation reads
// as operands x0, x1, x2: the operands an operator has, the first operand
// again in the slots it does not read, and the node itself for a register,
// input or constant (so the three loads need no decision).
struct LaneRec {
    uint8_t op, width, flags, words;
    uint32_t a, b, c;
    uint32_t fo0, fo1;
    uint32_t rfo0, rfo1;
    uint32_t u[4];     // fo[fo0 .. fo0 + 3]
    uint32_t r0;       // rfo[rfo0]
    uint32_t o[3];
};
static_assert(sizeof(LaneRec) == 64, "lane record layout");

struct Image {
    uint32_t N = 0, L = 0, R = 0, npi = 0;
    std::vector<uint32_t> u2i, i2u;         // user id <-> internal id
    std::vector<uint32_t> lvl_off;          // L+1 node offsets per level
    std::vector<uint32_t> level;            // per internal node
    std::vector<Desc> desc;
    std::vector<uint32_t> fo_off, fo, fo_lvl;   // combinational users (deduplicated)
    std::vector<uint64_t> fo_pk;                // user id | level << 32
    std::vector<uint32_t> rfo_off, rfo;         // registers whose D is this node
    // fo, fo_pk and rfo end in kFanoutPad zero entries (fo_lvl does not).
    std::vector<uint32_t> po;                   // internal ids, deduplicated
    std::vector<NodeRec> rec;                   // per internal node
    std::vector<LaneRec> lrec;                  // per internal node, for the light path
    std::vector<uint32_t> bp_off;               // first bit-plane row of each node (prefix sum of widths)
    uint32_t bp_rows = 0;                       // total bit-plane rows (sum of widths)
    uint32_t max_width = 0;                     // widest node
};

// Independent parts of a design for the golden machine.  The non-source
// nodes (not inputs or constants) fall into connected components (a register
// joined to its D input, an operator to its operands); components are packed
// into parts of at most kGoldenPartCap local nodes, each part with copies of
// the inputs and constants it reads, so that one workgroup can simulate a
// part for every cycle with its values in LDS and no other part's values.
// A local node is the design's descriptor with its operand ids (operands of
// an operator, the D input of a register) replaced by local indexes; gid is
// the internal id whose trace column the part writes, or kNoGid for a copied
// source another part owns.
constexpr uint32_t kGoldenPartCap = 4096;
constexpr uint32_t kNoGid = 0xFFFFFFFFu;
struct GNode {
    uint8_t op, width, pad0, pad1;
    uint32_t a, b, c;
    uint32_t gid;
};
static_assert(sizeof(GNode) == 20, "golden part node layout");
struct GoldenParts {
    std::vector<GNode> node;          // every part's local nodes, part after part, in level order
    std::vector<uint32_t> part_off;   // P+1 offsets into node
    std::vector<uint32_t> lvl;        // per part, the local offsets where its levels start, and its size
    std::vector<uint32_t> lvl_off;    // P+1 offsets into lvl
    uint32_t max_nodes = 0;           // largest part
};

// Fills gp and returns true when every component fits a part; false (gp
// empty) when a component is larger, the design then runs on one workgroup.
bool build_golden_parts(const Image& img, uint32_t max_parts, GoldenParts& gp);

// Per-node graph features of the load predictor (internal numbering):
// log2(1 + forward cone, capped), level / deepest level, fewest registers to
// an output (capped, -1 when none), log2(width).
constexpr uint32_t kConeCap = 1024;
constexpr int kDepthCap = 16;
void node_features(const Image& img, std::vector<float>& out /* [N][4] */);

// Registers take internal ids 0..R-1, then the other level-0 nodes (PI,
// CONST), then levels 1..L-1.  Returns RIROS_OK or an error code with `err`.
int build_image(const riros_design_desc& desc, Image& img, std::string& err);

int op_arity(uint8_t op);
// Algorithmic memory words of one event at a node (the byte model of the
// fault-simulation pass): its k operands (k = 0 for registers, inputs and
// constants), its own golden word and its faulty value, each two words when
// the node is wider than 32 bits.  A register whose state diverges moves its
// state too (read and written): twice this for a register event with a
// divergent state.  Per simulated cycle the site's golden word (1 or 2 words)
// is added once per fault.
uint8_t event_words(uint8_t op, uint8_t width);
bool op_is_comb(uint8_t op);

}  // namespace riros
