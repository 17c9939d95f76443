/*
 * riros.h -- C interface of the MI355X word-level RTL fault simulator.
 *
 * The simulator runs many faulty copies of a word-level RTL design cycle by
 * cycle against a golden (fault-free) trace and reports, for every injected
 * single stuck-at fault, the first cycle in which any primary output differs
 * from the golden value, or that the fault stayed undetected (paper, Sec. II-B:
 * a fault is injected, the faulty machine is simulated, and the fault is
 * detected by comparing faulty against good values).  Faults on wires sit on
 * the node that drives the wire, faults on registers on the register's node
 * (Sec. IV-A, unified fault injection).
 *
 * Conventions shared by every entry point:
 *   - Return value: RIROS_OK (0) on success, a negative RIROS_E* code on
 *     failure; riros_last_error() then returns a message (thread-local).  On
 *     failure no output buffer has been written.
 *   - Every input array is owned by the caller and is only read during the
 *     call.  Handles are owned by the library until the matching riros_free_*.
 *   - `stream` arguments are a hipStream_t owned by the caller, or NULL for
 *     the null stream.  Host-side outputs are complete when the call returns.
 *   - Values are two-state and unsigned; each node's value is kept masked to
 *     its width (1..64 bits).
 */
#ifndef RIROS_H
#define RIROS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RIROS_OK 0
#define RIROS_EINVAL (-1)   /* malformed design, fault, option or argument */
#define RIROS_ECYCLE (-2)   /* combinational loop (a cycle not cut by a register) */
#define RIROS_ENOMEM (-3)   /* host or device allocation failed */
#define RIROS_EDEVICE (-4)  /* HIP runtime error */

#define RIROS_UNDETECTED 0xFFFFFFFFu

/* Node operators.  Operands are zero-extended, results masked to the width.
 *   CONST  value = param
 *   PI     value = stimulus[t][param]
 *   REG    value = state; state(0) = param, state(t+1) = value(in[0], t)
 *          (end-of-cycle update of non-blocking assignments, Sec. II-B);
 *          in[0] must have the register's width
 *   ADD SUB AND OR XOR MUL            in[0] op in[1] (ADD/SUB/MUL modulo 2^width)
 *   NOT                                ~in[0]
 *   MUX                                in[0] != 0 ? in[2] : in[1]
 *   SHL SHR                            in[0] << param, in[0] >> param (logical)
 *   EQ NE ULT                          in[0] == / != / < in[1], as 0 or 1
 *   SLICE                              in[0] >> param
 *   CONCAT                             (in[0] << width(in[1])) | in[1]       */
enum {
    RIROS_OP_CONST = 0, RIROS_OP_PI, RIROS_OP_REG, RIROS_OP_ADD, RIROS_OP_SUB,
    RIROS_OP_AND, RIROS_OP_OR, RIROS_OP_XOR, RIROS_OP_NOT, RIROS_OP_MUX,
    RIROS_OP_SHL, RIROS_OP_SHR, RIROS_OP_EQ, RIROS_OP_NE, RIROS_OP_ULT,
    RIROS_OP_SLICE, RIROS_OP_CONCAT, RIROS_OP_MUL, RIROS_NUM_OPS
};

/* One RTL node (24 bytes).  Operand slots a node's operator does not read are
 * ignored.  Node ids are indexes into the node array. */
typedef struct {
    uint8_t op;
    uint8_t width;       /* 1..64 */
    uint16_t reserved;
    uint32_t in[3];      /* operand node ids */
    uint64_t param;      /* CONST value, PI column, REG reset value, shift amount or SLICE low bit */
} riros_node;

/* A single fault on bit `bit` of node `site` (a wire fault sits on the node
 * driving the wire, a register fault on the register's node, Sec. IV-A).
 * stuck 0 or 1: stuck-at, the bit is forced to `stuck` in every cycle.
 * stuck RIROS_FAULT_FLIP: the bit is inverted in cycle t0 only; on a register
 * this is a single-event upset of the stored state, which then evolves
 * normally (the paper's unified injection admits other fault models through
 * the faulty-value function, Sec. IV-A and V-A).  Either way the effect
 * applies to the node's value as seen by its users and by output comparison;
 * a register's next-state write is not altered. */
#define RIROS_FAULT_FLIP 2
typedef struct {
    uint32_t site;
    uint8_t bit;         /* < width(site) */
    uint8_t stuck;       /* 0, 1 or RIROS_FAULT_FLIP */
    uint16_t t0;         /* RIROS_FAULT_FLIP: the cycle of the flip (no effect if >= T); else ignored */
} riros_fault;

typedef struct {
    uint32_t num_nodes;
    const riros_node* nodes;
    uint32_t num_pi;     /* stimulus columns; every PI's param is < num_pi */
    uint32_t num_po;
    const uint32_t* po;  /* primary-output node ids */
} riros_design_desc;

typedef struct riros_design_s* riros_design;
typedef struct riros_golden_s* riros_golden;

/* Validate a design, levelise it (registers cut every combinational cycle) and
 * upload its levelised image to the current HIP device.  This is the compile
 * step that turns RTL into a graph of nodes and the node graph into schedulable
 * work (Sec. IV, Steps 1 and 4).  Errors: RIROS_EINVAL for a bad operator,
 * width, operand id, PI column, PO id or a register whose D input has another
 * width; RIROS_ECYCLE for a combinational loop; RIROS_ENOMEM; RIROS_EDEVICE.
 * On success *out is a new handle (free with riros_free_design). */
int riros_load_design(const riros_design_desc* desc, riros_design* out);
void riros_free_design(riros_design d);

/* Simulate the fault-free machine for cycles 0..T-1 and keep the golden trace
 * resident in device memory (the "good gate" values every bad gate is compared
 * against, Sec. II-B).  `stimulus` is a host array uint64[T][num_pi], row t =
 * primary-input values of cycle t (masked to each PI's width on use).  The
 * trace is kept in three layouts (cycle-major, node-major and one bit-plane
 * per node bit), about 16*T*num_nodes + T*sum(widths)/8 bytes of device
 * memory, plus 4*T*num_nodes for a 32-bit node-major copy when no node is
 * wider than 32 bits.  A design whose non-input nodes fall into independent
 * components of at most 4,096 nodes (with the inputs and constants they
 * read) runs by parts, one workgroup per part with the part's values in LDS;
 * otherwise one workgroup walks the whole design.  Errors: RIROS_EINVAL
 * (T == 0, NULL pointers), RIROS_ENOMEM, RIROS_EDEVICE.  *out is a new handle. */
int riros_golden_sim(riros_design d, const uint64_t* stimulus, uint32_t T, void* stream,
                     riros_golden* out);
void riros_free_golden(riros_golden g);

/* riros_golden_sim for n designs at once: one kernel launch simulates the
 * fault-free machines of every design in fewer than two parts, one workgroup
 * per design (the designs are independent), a second one the parts of the
 * others, one workgroup per part; then each trace gets its other layouts.  stimulus[i] and T[i]
 * as for riros_golden_sim; out[i] receives design i's handle.  Errors as for
 * riros_golden_sim (nothing is returned on failure). */
int riros_golden_sim_many(uint32_t n, const riros_design* designs, const uint64_t* const* stimulus,
                          const uint32_t* T, void* stream, riros_golden* out);

/* Copy cycles [t0, t0+nt) of a golden trace to host memory as
 * uint64[nt][num_nodes], in the caller's node numbering. */
int riros_golden_read(riros_golden g, uint32_t t0, uint32_t nt, uint64_t* out);

/* Scheduling mode of riros_fault_sim. */
#define RIROS_MODE_PLAIN 0     /* one fault per wavefront, static fault order */
#define RIROS_MODE_TWO_D 1     /* light faults one per lane, heavy faults split
                                  structurally; persistent work queue */
#define RIROS_MODE_CONCURRENT 2 /* node-major concurrent simulation (good gate and
                                  bad gates of a node together, Sec. II-B and
                                  Sec. IV-B): faults ordered by site, 64 to a
                                  wavefront, one per lane, walking the union of
                                  their divergent frontiers; each frontier node is
                                  fetched once for all 64.  Takes up to 128 GiB,
                                  and at most 60% of the free device memory, for
                                  faulty state (about 528 * (num_nodes + 2 *
                                  registers) bytes per resident wavefront);
                                  waves_per_cu bounds the wavefronts; priority
                                  and the TWO_D fields are ignored */

typedef struct {
    int32_t mode;          /* RIROS_MODE_* */
    int32_t drop;          /* 1: stop a fault at its detect cycle; 0: run all T cycles */
    int32_t io_on_device;  /* 1: faults, detect, events and coverage are device pointers
                              and the call is asynchronous on `stream` */
    int32_t waves_per_cu;  /* resident wavefronts per compute unit (0 = default) */
    const float* priority; /* optional per-fault predicted load (device pointer when
                              io_on_device, else host); higher runs first.  Only
                              changes the schedule, never a result */
    float theta;           /* TWO_D: priority above which a fault starts on the
                              structural (heavy) path; +inf = all light */
    int32_t light_cap;     /* TWO_D: per-lane divergent-node capacity, 4, 8 or 16
                              (0 = 8); a lane that overflows hands its fault to
                              the structural path */
    int32_t unified;       /* TWO_D: 1 = a wavefront whose lanes have run out of
                              light work takes handed-over faults while the
                              others still run light work (the structural path
                              then needs LDS in every wavefront of launch A);
                              0 = handed-over faults wait for launch B */
    float monitor_rate;    /* TWO_D: a light fault averaging more than this many
                              events per cycle after its first 8 cycles moves to
                              the structural path (0 = never) */
    int32_t struct_share;  /* TWO_D, when launch A has structural work (a heavy
                              prefix or unified): wavefronts of launch A per
                              structural workspace (the LDS and faulty-value
                              slots of one wavefront), 1, 2 or 4; the first
                              takes the structural work, the others run light
                              faults only.  0 = the smallest that keeps
                              waves_per_cu wavefronts resident despite the
                              structural LDS of the design, else 4 */
    void* stream;
    uint64_t* words;       /* optional per-fault output [F] (same memory space as detect):
                              the memory words the method must touch for the fault
                              (the byte model of the measurement): per simulated cycle
                              the site's golden word; per event at a node with k
                              operands (k = 0 for a register, input or constant),
                              k + 2 words (operands, the node's golden word, its
                              faulty value); a register whose state diverges, 2 words
                              more (state read and written); every word counts twice
                              for a node wider than 32 bits.  4 bytes a word. */
    int32_t campaign_golden; /* riros_batch_create only: 1 = every launch of the
                              campaign also recomputes each design's golden trace
                              (one workgroup per design, one kernel) before its fault
                              simulation, inside the same graph; 0 = the traces
                              riros_golden_sim computed are used as they are */
    int32_t heavy_wg;      /* TWO_D: threads that simulate one fault on the structural
                              path in launch B (handed-over faults) and, when launch A
                              runs workgroups of several wavefronts (struct_share), in
                              its heavy prefix: 64 (one wavefront), 128 or 256 (the
                              fault's frontier split across 2 or 4 wavefronts, one
                              barrier per pass: the paper spreads a high-load node
                              over many workers, Sec. IV-C); 0 = 64 */
    int32_t lockstep;      /* TWO_D: 1 = a light lane about to start a cycle waits while
                              another lane of its wavefront is still inside one, so the
                              lanes of a wavefront (faults of one node or one template,
                              when ordered by priority) walk their frontiers in step; 0 =
                              every lane runs on.  Never changes a result */
    int32_t deal;          /* TWO_D: 0 = light faults are taken in queue order (with
                              priorities: descending, so the first wavefronts take
                              the heaviest 64 each); 4, 8, 16 or 32 = the first
                              64 x (resident wavefronts) queue positions are dealt
                              out in groups of `deal` consecutive faults, so that a
                              wavefront's first 64 lanes take one group of each of
                              64 / deal priority strata: the heavy head of the
                              order spreads over every wavefront of the launch
                              (the longest-first deal of the paper's load
                              balancing, Sec. IV-C).  Never changes a result */
    int32_t head_lanes;    /* TWO_D: 0 = a wavefront refills any idle lane (up to its
                              share of the list) at once; 1..64 = its first take is
                              head_lanes faults, and it takes no more until all of
                              them are finished (its other lanes idle meanwhile), so
                              the head of a descending order (the faults predicted
                              heaviest) runs head_lanes to a wavefront, beside faults
                              of its own kind only, on up to 64 / head_lanes times
                              more wavefronts.  Never changes a result */
    int32_t xcd_queues;    /* TWO_D with priorities: 1 = one light queue per XCD (the
                              chip's 8 dies, each with its own L2): the descending
                              order is partitioned by the fault site's XCD (blocks
                              of 64 consecutive node ids round-robin over the 8),
                              each part keeping its longest-first order, and a
                              wavefront takes faults from its own XCD's part first,
                              then from the others' once its own is empty, so faults
                              on nearby nodes share one L2; deal is ignored.  0 = one
                              queue.  Never changes a result */
} riros_sim_opts;

typedef struct {
    uint64_t detected;      /* faults with a detect cycle */
    uint64_t total;         /* faults simulated */
    uint64_t fault_cycles;  /* sum over faults of (detect + 1), or T if undetected */
    uint64_t events;        /* sum of per-fault event counts */
    uint64_t words;         /* sum of per-fault byte-model words (riros_sim_opts.words) */
} riros_coverage;

/* Fault-simulate F single faults (stuck-at or bit flip) against the golden trace.
 * detect[F] receives the first cycle in which any primary output of the
 * faulty machine differs from the golden trace, or RIROS_UNDETECTED.
 * events[F] (may be NULL) receives the fault's bad-gate evaluations: node n in
 * cycle t counts when one of its inputs (for a register: its state) or its own
 * value differs from the golden machine (Sec. II-B, concurrent fault
 * simulation); with drop = 1 the count stops after the detect cycle.
 * cov (may be NULL) receives totals.  Results do not depend on mode, priority,
 * theta, light_cap, unified, monitor_rate or waves_per_cu.  Errors: RIROS_EINVAL (site >= num_nodes,
 * bit >= width, stuck > 2, unknown mode, design/golden mismatch, a design
 * whose frontier bitmaps exceed a compute unit's 160 KB of LDS), RIROS_ENOMEM
 * (also: CONCURRENT when one wavefront's faulty state exceeds its budget),
 * RIROS_EDEVICE.  Calls on one design share its workspace: issue them on one
 * stream, or wait for one before the next. */
int riros_fault_sim(riros_design d, riros_golden g, const riros_fault* faults, uint32_t F,
                    const riros_sim_opts* opts, uint32_t* detect, uint64_t* events,
                    riros_coverage* cov);

/* ------------------------------------------------------------------------ */
/* Learned load predictor.  It only orders faults and picks their starting   */
/* path (the paper marks high-load nodes with an execution-time monitor,      */
/* Sec. IV-C; here a small network predicts each fault's load up front), so   */
/* no result depends on it.                                                   */
/* ------------------------------------------------------------------------ */

#define RIROS_NUM_FEATURES 6
#define RIROS_MLP_PARAMS 4673          /* 6-64-64-1: W1[64][6] b1[64] W2[64][64] b2[64] W3[64] b3 */
#define RIROS_MLP_WEIGHTS (4673 + 12)  /* parameters, then input mean[6] and std[6] */

/* Per-fault features, float32[F][6]: log2(1 + forward combinational cone of
 * the site, registers fed counted but not crossed, capped at 1024); site
 * level / deepest level; fewest registers from the site to an output (capped
 * at 16, -1 if none); log2(site width); toggle rate of the site bit over the
 * golden trace (changes / (T-1)); fraction of cycles in which the site bit
 * differs from the stuck value (a flip: 1/T if t0 < T, else 0).  faults/out are device pointers when
 * io_on_device (asynchronous on stream), else host pointers.  Errors as for
 * riros_fault_sim. */
int riros_features(riros_design d, riros_golden g, const riros_fault* faults, uint32_t F, float* out,
                   int32_t io_on_device, void* stream);

typedef struct {
    uint32_t epochs;   /* passes over the samples, in the given order */
    uint32_t batch;    /* minibatch size (the last one of a pass may be smaller) */
    float lr, beta1, beta2, eps;   /* Adam (Kingma and Ba, 2015) */
} riros_train_cfg;

/* Train the predictor with minibatch Adam on mean squared error.  Host
 * arrays: feats float32[S][6], y float32[S] (target, e.g. log2(1 + events)),
 * weights float32[RIROS_MLP_WEIGHTS]: on entry the initial parameters (the
 * normalisation part is ignored), on return the trained parameters with the
 * mean and standard deviation of each feature over the samples.  losses
 * (may be NULL) receives the loss of every step, epochs * ceil(S / batch)
 * floats.  Errors: RIROS_EINVAL (S, epochs or batch zero, NULL pointers),
 * RIROS_ENOMEM, RIROS_EDEVICE. */
int riros_mlp_train(const float* feats, const float* y, uint32_t S, const riros_train_cfg* cfg, float* weights,
                    float* losses, void* stream);

/* Predicted load for F feature rows with trained weights.  feats/out are
 * device pointers when io_on_device (asynchronous), else host pointers. */
int riros_mlp_predict(const float* weights, const float* feats, uint32_t F, float* out, int32_t io_on_device,
                      void* stream);

/* Gradient of the mean squared error over one batch of B samples (host
 * arrays; weights include the normalisation): grad float32[RIROS_MLP_PARAMS],
 * loss float32[1].  The same kernels as training; for checking them. */
int riros_mlp_grad(const float* weights, const float* feats, const float* y, uint32_t B, float* grad,
                   float* loss, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched campaigns: many designs, each with its own golden trace and fault  */
/* list, simulated by one persistent two-dimensional launch over a single     */
/* work queue of all their faults, captured once as a HIP graph and replayed. */
/* ------------------------------------------------------------------------ */

typedef struct riros_batch_s* riros_batch;

/* Build a campaign of n designs (all loaded on the current device; goldens[i]
 * belongs to designs[i]).  faults[i] is a host array of F[i] faults of design
 * i; priority (may be NULL, and entries may be NULL for zero priority) gives
 * per-fault predicted loads; the whole campaign is ordered by them, and
 * faults above opts->theta start on the structural path.  opts->mode must be
 * RIROS_MODE_TWO_D and opts->io_on_device 0; drop, waves_per_cu, light_cap
 * and monitor_rate apply.  Inputs are uploaded and the run is captured as a
 * graph.  Errors: RIROS_EINVAL (n == 0 or > 65536, mismatched goldens, invalid
 * faults or options), RIROS_ENOMEM, RIROS_EDEVICE. */
int riros_batch_create(uint32_t n, const riros_design* designs, const riros_golden* goldens,
                       const riros_fault* const* faults, const uint32_t* F, const float* const* priority,
                       const riros_sim_opts* opts, riros_batch* out);

/* Run the whole campaign: one graph launch on `stream` (asynchronous).
 * riros_last_kernel_ms then reports its duration. */
int riros_batch_launch(riros_batch b, void* stream);

/* Results of design i after the last launch (waits for it): detect[F[i]],
 * events[F[i]] and words[F[i]] (byte-model words as in riros_sim_opts.words;
 * both may be NULL), coverage (may be NULL); host arrays. */
int riros_batch_read(riros_batch b, uint32_t i, uint32_t* detect, uint64_t* events, uint64_t* words,
                     riros_coverage* cov);

void riros_batch_free(riros_batch b);

/* Number of nodes, levels and registers of a loaded design. */
int riros_design_info(riros_design d, uint32_t* num_nodes, uint32_t* num_levels, uint32_t* num_regs);

/* Duration in milliseconds of the fault-simulation kernels of the last
 * riros_fault_sim call on this thread (HIP events on its stream; the call must
 * have completed). */
int riros_last_kernel_ms(float* ms);

const char* riros_last_error(void);

/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate device memory: code under HIP graph       */
/* capture, tight serving loops, harnesses that forbid hipMalloc.             */
/* ------------------------------------------------------------------------ */

/* Bytes of the library's static scratch array, one per GPU it runs on, held
 * until the process ends. */
#define RIROS_NOALLOC_SCRATCH_BYTES (128u << 20)

/* riros_fault_sim in RIROS_MODE_PLAIN with device-resident inputs and outputs
 * (opts->io_on_device must be 1; opts->words may be NULL), calling no
 * hipMalloc, hipFree or allocating library routine: its workspace (each
 * wavefront's faulty-value slots and register ping-pong, 16 * num_nodes +
 * 16 * registers bytes) comes from the static scratch array, and the grid is
 * cut to the wavefronts whose workspace fits it.  A design whose one-wavefront
 * workspace exceeds RIROS_NOALLOC_SCRATCH_BYTES is rejected (RIROS_EINVAL,
 * with the sizes in the message), and so are other modes and host I/O.  Faults
 * are validated on the device; the call waits once for that check, then runs
 * asynchronously on opts->stream (riros_last_kernel_ms does not time it).
 * Every call on a GPU shares that GPU's array and keeps nothing in it between
 * calls (the slots it uses are cleared by a kernel first): calls that overlap
 * on one GPU race, so issue them on one stream.  Results equal riros_fault_sim's
 * in plain mode. */
int riros_fault_sim_noalloc(riros_design d, riros_golden g, const riros_fault* faults, uint32_t F,
                            const riros_sim_opts* opts, uint32_t* detect, uint64_t* events,
                            riros_coverage* cov);

/* ------------------------------------------------------------------------ */
/* Peak-rate probes for the roofline (measurement tools, not part of the      */
/* method): the rates a fault-simulation pass is compared against, measured   */
/* on the current device.                                                     */
/* ------------------------------------------------------------------------ */

/* HBM streaming rate: the best of `reps` device copies of `bytes` bytes (each
 * reads `bytes` and writes `bytes`), *gbs = 2 * bytes / time in GB/s.  Takes
 * 2 * bytes of device memory for the call.  Returns 0, -1 (bad argument), -3
 * (no memory) or -4 (HIP error). */
int riros_peak_hbm(uint64_t bytes, int reps, double* gbs, void* stream);

/* int32 vector-ALU rate: the best of `reps` launches of independent chains of
 * single-cycle integer instructions (v_add_u32, v_xor_b32) on every compute
 * unit, *ops_per_s = instructions per second counted per lane.  Returns 0,
 * -1, -3 or -4 as above. */
int riros_peak_valu(int reps, double* ops_per_s, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RIROS_H */
