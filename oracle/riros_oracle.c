/*
 * CPU oracle for word-level RTL stuck-at fault simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: it has its own
 * node layout (byte-identical to the C interface's riros_node because both
 * read the same input arrays), its own topological sort, its own evaluator.
 *
 * What it computes (paper Sec. II-B, Sec. IV-A):
 *   golden   the fault-free machine, every node, every cycle: G[t][n].
 *   O0       each fault simulated alone, from cycle 0, evaluating every node
 *            of the design in every cycle (the plain definition).
 *   O1       the same quantities, evaluating only the nodes with a divergent
 *            input ("bad gates" of concurrent fault simulation, Sec. II-B;
 *            the check of whether a task's inputs changed, Alg. 1), with its
 *            own level buckets and stamps.  Pinned against O0.
 *
 * Semantics (readings of the paper, which leaves them to Verilog):
 *   - two-state unsigned values, each node's value masked to its width;
 *   - in cycle t the stimulus row t is applied, combinational logic settles,
 *     primary outputs are compared, then every register takes its D value
 *     (the end-of-cycle synchronisation of non-blocking assignments, Sec. II-B);
 *   - a stuck-at fault (site s, bit b, value v) forces bit b of node s to v in
 *     every cycle (a wire fault sits on the node driving the wire, a register
 *     fault on the register's node, Sec. IV-A); a forced register is forced on
 *     read, its next-state write is never forced;
 *   - a bit flip (stuck == 2, cycle t0) inverts bit b of node s in cycle t0
 *     only: a transient fault model through the same injection point (the
 *     paper's unified injection supports other fault models by changing the
 *     faulty-value function, Sec. IV-A and V-A); on a register it is a
 *     single-event upset of the stored state, which then evolves normally;
 *   - a fault is detected in the first cycle in which any primary output
 *     differs from the golden value (Sec. II-B); otherwise it is undetected
 *     (0xFFFFFFFF);
 *   - an event is one bad-gate evaluation: node n in cycle t is an event of
 *     fault f when one of its inputs is divergent (for a register: its state,
 *     i.e. its D one cycle earlier) or its own faulty value is divergent.
 *     With dropping, events stop after the detect cycle (that cycle included);
 *     without, they run to the last cycle.  detect does not depend on drop.
 *   - statistics (optional outputs, for the benchmark's byte model and the
 *     workload calibration; they change no result):
 *       words    the algorithmic memory words the method must touch, with
 *                w(n) = 2 for a node wider than 32 bits, else 1: per
 *                simulated cycle w(site) (the site's golden word, read to see
 *                whether the fault is excited); per event at node n,
 *                (k + 2) * w(n), k = operand count of a combinational node
 *                (0 otherwise): its operands, its own golden word and its
 *                faulty value; per register whose state diverges, 2 * w(r)
 *                more (the divergent state is read and written);
 *       lastreg  the last cycle in which some register's state diverges
 *                (0xFFFFFFFF if none), within the simulated cycles.
 *
 * Parity pins: tests/test_oracle_*.py (closed forms, brute force against a
 * bit-blasted evaluator, invariants, O0 against O1).
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    O_CONST, O_PI, O_REG, O_ADD, O_SUB, O_AND, O_OR, O_XOR, O_NOT, O_MUX,
    O_SHL, O_SHR, O_EQ, O_NE, O_ULT, O_SLICE, O_CONCAT, O_MUL, O_NUM_OPS
};

typedef struct {
    uint8_t op, width;
    uint16_t pad;
    uint32_t in[3];
    uint64_t param;
} o_node;

typedef struct {
    uint32_t site;
    uint8_t bit, stuck;   /* stuck: 0 or 1 (stuck-at), O_FLIP (bit flip in cycle t0) */
    uint16_t t0;
} o_fault;

#define O_FLIP 2

#define O_UNDET 0xFFFFFFFFu

static const int o_arity[O_NUM_OPS] = {
    0, 0, 1, 2, 2, 2, 2, 2, 1, 3, 1, 1, 2, 2, 2, 1, 2, 2
};

static uint64_t o_mask(unsigned w) { return w >= 64 ? ~0ull : ((1ull << w) - 1ull); }

static int o_is_comb(uint8_t op) { return op != O_CONST && op != O_PI && op != O_REG; }

/* Result of a combinational operator on already-masked operand values. */
static uint64_t o_apply(const o_node* nd, const o_node* all, uint64_t a, uint64_t b, uint64_t c)
{
    uint64_t r = 0, k = nd->param;
    switch (nd->op) {
    case O_ADD: r = a + b; break;
    case O_SUB: r = a - b; break;
    case O_AND: r = a & b; break;
    case O_OR: r = a | b; break;
    case O_XOR: r = a ^ b; break;
    case O_NOT: r = ~a; break;
    case O_MUX: r = (a != 0) ? c : b; break;
    case O_SHL: r = k >= 64 ? 0 : (a << k); break;
    case O_SHR: r = k >= 64 ? 0 : (a >> k); break;
    case O_EQ: r = (a == b); break;
    case O_NE: r = (a != b); break;
    case O_ULT: r = (a < b); break;
    case O_SLICE: r = k >= 64 ? 0 : (a >> k); break;
    case O_CONCAT: {
        unsigned wb = all[nd->in[1]].width;
        r = (wb >= 64 ? 0 : (a << wb)) | b;
        break;
    }
    case O_MUL: r = a * b; break;
    default: r = 0; break;
    }
    return r & o_mask(nd->width);
}

/* The fault's effect on its site's value in cycle t. */
static uint64_t o_force(uint64_t v, const o_fault* f, uint32_t t)
{
    uint64_t bit = 1ull << f->bit;
    if (f->stuck == O_FLIP) return t == f->t0 ? (v ^ bit) : v;
    return f->stuck ? (v | bit) : (v & ~bit);
}

/* Words of a node's value: two for a node wider than 32 bits. */
static uint64_t o_ww(const o_node* x) { return x->width > 32 ? 2u : 1u; }

/* Words of one event at node x (operands, golden word, faulty value). */
static uint64_t o_event_words(const o_node* x)
{
    uint64_t k = o_is_comb(x->op) ? (uint64_t)o_arity[x->op] : 0u;
    return (k + 2u) * o_ww(x);
}

/* ------------------------------------------------------------------------- */
/* Design preparation: validation and a topological order (Kahn).            */
/* ------------------------------------------------------------------------- */

typedef struct {
    const o_node* nd;
    uint32_t N, npi, npo;
    const uint32_t* po;
    uint32_t* topo;     /* every node, inputs before users (registers cut edges) */
    uint32_t* regs;     /* register node ids */
    uint32_t nregs;
} o_design;

static int o_prepare(o_design* d, const void* nodes, uint32_t N, const uint32_t* po, uint32_t npo,
                     uint32_t npi)
{
    const o_node* nd = (const o_node*)nodes;
    memset(d, 0, sizeof(*d));
    d->nd = nd; d->N = N; d->npi = npi; d->po = po; d->npo = npo;
    for (uint32_t n = 0; n < N; ++n) {
        if (nd[n].op >= O_NUM_OPS || nd[n].width < 1 || nd[n].width > 64) return -1;
        for (int k = 0; k < o_arity[nd[n].op]; ++k)
            if (nd[n].in[k] >= N) return -1;
        if (nd[n].op == O_PI && nd[n].param >= npi) return -1;
        if (nd[n].op == O_REG && nd[nd[n].in[0]].width != nd[n].width) return -1;
    }
    for (uint32_t i = 0; i < npo; ++i)
        if (po[i] >= N) return -1;
    uint32_t* indeg = calloc(N, sizeof(uint32_t));
    uint32_t* cnt = calloc(N + 1, sizeof(uint32_t));
    uint32_t* users = NULL;
    d->topo = malloc((size_t)N * sizeof(uint32_t));
    d->regs = malloc((size_t)N * sizeof(uint32_t));
    if (!indeg || !cnt || !d->topo || !d->regs) goto oom;
    /* user lists of the combinational edges */
    for (uint32_t n = 0; n < N; ++n) {
        if (!o_is_comb(nd[n].op)) continue;
        for (int k = 0; k < o_arity[nd[n].op]; ++k) { cnt[nd[n].in[k] + 1]++; indeg[n]++; }
    }
    for (uint32_t n = 0; n < N; ++n) cnt[n + 1] += cnt[n];
    users = malloc((size_t)(cnt[N] + 1) * sizeof(uint32_t));
    if (!users) goto oom;
    {
        uint32_t* fill = calloc(N, sizeof(uint32_t));
        if (!fill) goto oom;
        for (uint32_t n = 0; n < N; ++n) {
            if (!o_is_comb(nd[n].op)) continue;
            for (int k = 0; k < o_arity[nd[n].op]; ++k) {
                uint32_t s = nd[n].in[k];
                users[cnt[s] + fill[s]++] = n;
            }
        }
        free(fill);
    }
    uint32_t head = 0, tail = 0;
    for (uint32_t n = 0; n < N; ++n)
        if (indeg[n] == 0) d->topo[tail++] = n;
    while (head < tail) {
        uint32_t s = d->topo[head++];
        for (uint32_t e = cnt[s]; e < cnt[s + 1]; ++e)
            if (--indeg[users[e]] == 0) d->topo[tail++] = users[e];
    }
    free(indeg); free(cnt); free(users);
    if (tail != N) { free(d->topo); free(d->regs); d->topo = d->regs = NULL; return -2; }
    for (uint32_t n = 0; n < N; ++n)
        if (nd[n].op == O_REG) d->regs[d->nregs++] = n;
    return 0;
oom:
    free(indeg); free(cnt); free(users); free(d->topo); free(d->regs);
    d->topo = d->regs = NULL;
    return -3;
}

static void o_release(o_design* d) { free(d->topo); free(d->regs); }

/* Value of node n in cycle t given the current values, register states and
 * stimulus (no fault forcing). */
static uint64_t o_value(const o_design* d, uint32_t n, const uint64_t* val, const uint64_t* state,
                        const uint64_t* stim_row)
{
    const o_node* x = &d->nd[n];
    switch (x->op) {
    case O_CONST: return x->param & o_mask(x->width);
    case O_PI: return stim_row[x->param] & o_mask(x->width);
    case O_REG: return state[n];
    default: {
        uint64_t a = 0, b = 0, c = 0;
        int ar = o_arity[x->op];
        if (ar > 0) a = val[x->in[0]];
        if (ar > 1) b = val[x->in[1]];
        if (ar > 2) c = val[x->in[2]];
        return o_apply(x, d->nd, a, b, c);
    }
    }
}

int oracle_golden(const void* nodes, uint32_t N, const uint32_t* po, uint32_t npo, uint32_t npi,
                  const uint64_t* stim, uint32_t T, uint64_t* G)
{
    o_design d;
    int rc = o_prepare(&d, nodes, N, po, npo, npi);
    if (rc) return rc;
    uint64_t* val = calloc(N ? N : 1, sizeof(uint64_t));
    uint64_t* state = calloc(N ? N : 1, sizeof(uint64_t));
    if (!val || !state) { free(val); free(state); o_release(&d); return -3; }
    for (uint32_t i = 0; i < d.nregs; ++i) {
        uint32_t r = d.regs[i];
        state[r] = d.nd[r].param & o_mask(d.nd[r].width);
    }
    for (uint32_t t = 0; t < T; ++t) {
        const uint64_t* row = stim + (size_t)t * npi;
        for (uint32_t i = 0; i < N; ++i) {
            uint32_t n = d.topo[i];
            val[n] = o_value(&d, n, val, state, row);
        }
        memcpy(G + (size_t)t * N, val, (size_t)N * sizeof(uint64_t));
        for (uint32_t i = 0; i < d.nregs; ++i) {
            uint32_t r = d.regs[i];
            state[r] = val[d.nd[r].in[0]] & o_mask(d.nd[r].width);
        }
    }
    free(val); free(state); o_release(&d);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* O0: every node, every cycle.                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint64_t* val;
    uint64_t* state;
} o0_scratch;

static void o0_one(const o_design* d, const uint64_t* stim, uint32_t T, const uint64_t* G,
                   const o_fault* f, int drop, o0_scratch* s, uint32_t* detect_out,
                   uint64_t* events_out, uint64_t* words_out, uint32_t* lastreg_out)
{
    const uint32_t N = d->N;
    uint64_t* val = s->val;
    uint64_t* state = s->state;
    uint32_t detect = O_UNDET, lastreg = O_UNDET, cycles = 0;
    uint64_t ev = 0, words = 0;
    for (uint32_t i = 0; i < d->nregs; ++i) {
        uint32_t r = d->regs[i];
        state[r] = d->nd[r].param & o_mask(d->nd[r].width);
    }
    for (uint32_t t = 0; t < T; ++t) {
        const uint64_t* row = stim + (size_t)t * d->npi;
        const uint64_t* g = G + (size_t)t * N;
        for (uint32_t i = 0; i < N; ++i) {
            uint32_t n = d->topo[i];
            uint64_t v = o_value(d, n, val, state, row);
            if (n == f->site) v = o_force(v, f, t);
            val[n] = v;
        }
        cycles = t + 1;
        for (uint32_t n = 0; n < N; ++n) {
            const o_node* x = &d->nd[n];
            int div_in = 0;
            if (x->op == O_REG) {
                div_in = state[n] != g[n];
                if (div_in) { words += 2u * o_ww(x); lastreg = t; }
            } else if (o_is_comb(x->op)) {
                for (int k = 0; k < o_arity[x->op]; ++k)
                    div_in |= val[x->in[k]] != g[x->in[k]];
            }
            if (div_in || val[n] != g[n]) { ev++; words += o_event_words(x); }
        }
        for (uint32_t i = 0; i < d->npo; ++i)
            if (val[d->po[i]] != g[d->po[i]] && detect == O_UNDET) detect = t;
        if (drop && detect != O_UNDET) break;
        for (uint32_t i = 0; i < d->nregs; ++i) {
            uint32_t r = d->regs[i];
            state[r] = val[d->nd[r].in[0]] & o_mask(d->nd[r].width);
        }
    }
    *detect_out = detect;
    if (events_out) *events_out = ev;
    if (words_out) *words_out = words + (uint64_t)cycles * o_ww(&d->nd[f->site]);
    if (lastreg_out) *lastreg_out = lastreg;
}

/* ------------------------------------------------------------------------- */
/* O1: only nodes with a divergent input, in level order.                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint32_t* level;       /* level of each node */
    uint32_t nlevels;
    uint32_t* fo_off;      /* combinational users, CSR */
    uint32_t* fo;
    uint32_t* rfo_off;     /* registers whose D is this node, CSR */
    uint32_t* rfo;
    uint8_t* is_po;
} o1_graph;

static int o1_build(const o_design* d, o1_graph* g)
{
    const uint32_t N = d->N;
    memset(g, 0, sizeof(*g));
    g->level = calloc(N ? N : 1, sizeof(uint32_t));
    g->fo_off = calloc(N + 1, sizeof(uint32_t));
    g->rfo_off = calloc(N + 1, sizeof(uint32_t));
    g->is_po = calloc(N ? N : 1, 1);
    if (!g->level || !g->fo_off || !g->rfo_off || !g->is_po) return -3;
    uint32_t maxl = 0;
    for (uint32_t i = 0; i < N; ++i) {
        uint32_t n = d->topo[i];
        const o_node* x = &d->nd[n];
        uint32_t l = 0;
        if (o_is_comb(x->op)) {
            for (int k = 0; k < o_arity[x->op]; ++k)
                if (g->level[x->in[k]] + 1 > l) l = g->level[x->in[k]] + 1;
        }
        g->level[n] = l;
        if (l > maxl) maxl = l;
    }
    g->nlevels = maxl + 1;
    for (uint32_t n = 0; n < N; ++n) {
        const o_node* x = &d->nd[n];
        if (o_is_comb(x->op))
            for (int k = 0; k < o_arity[x->op]; ++k) g->fo_off[x->in[k] + 1]++;
        if (x->op == O_REG) g->rfo_off[x->in[0] + 1]++;
    }
    for (uint32_t n = 0; n < N; ++n) {
        g->fo_off[n + 1] += g->fo_off[n];
        g->rfo_off[n + 1] += g->rfo_off[n];
    }
    g->fo = malloc((size_t)(g->fo_off[N] + 1) * sizeof(uint32_t));
    g->rfo = malloc((size_t)(g->rfo_off[N] + 1) * sizeof(uint32_t));
    uint32_t* f1 = calloc(N ? N : 1, sizeof(uint32_t));
    uint32_t* f2 = calloc(N ? N : 1, sizeof(uint32_t));
    if (!g->fo || !g->rfo || !f1 || !f2) { free(f1); free(f2); return -3; }
    for (uint32_t n = 0; n < N; ++n) {
        const o_node* x = &d->nd[n];
        if (o_is_comb(x->op))
            for (int k = 0; k < o_arity[x->op]; ++k) {
                uint32_t s = x->in[k];
                g->fo[g->fo_off[s] + f1[s]++] = n;
            }
        if (x->op == O_REG) {
            uint32_t s = x->in[0];
            g->rfo[g->rfo_off[s] + f2[s]++] = n;
        }
    }
    free(f1); free(f2);
    for (uint32_t i = 0; i < d->npo; ++i) g->is_po[d->po[i]] = 1;
    return 0;
}

static void o1_free(o1_graph* g)
{
    free(g->level); free(g->fo_off); free(g->fo); free(g->rfo_off); free(g->rfo); free(g->is_po);
}

typedef struct {
    uint64_t* fval;       /* faulty value, valid when fstamp == current stamp */
    uint32_t* fstamp;
    uint32_t* qstamp;     /* queued in the current cycle */
    uint64_t* rstate;     /* divergent register state, valid when rstamp == stamp */
    uint32_t* rstamp;
    uint32_t* bucket;     /* per-level lists, each with capacity of the level's size */
    uint32_t* bfill;
    uint32_t* boff;
    uint32_t* rnext;      /* (reg, value) pairs produced this cycle */
    uint64_t* rnextv;
} o1_scratch;

static void o1_one(const o_design* d, const o1_graph* gr, const uint64_t* stim, uint32_t T,
                   const uint64_t* G, const o_fault* f, int drop, o1_scratch* s,
                   uint32_t* detect_out, uint64_t* events_out, uint64_t* words_out, uint32_t* lastreg_out)
{
    const uint32_t N = d->N;
    uint32_t detect = O_UNDET, lastreg = O_UNDET, cycles = 0;
    uint64_t ev = 0, words = 0;
    uint32_t nnext = 0;
    /* stamps are cycle+1 offset by a per-call base so that scratch need not be cleared */
    for (uint32_t t = 0; t < T; ++t) {
        uint32_t stamp = t + 1;
        const uint64_t* row = stim + (size_t)t * d->npi;
        const uint64_t* g = G + (size_t)t * N;
        for (uint32_t l = 0; l < gr->nlevels; ++l) s->bfill[l] = 0;
#define O1_PUSH(node)                                                              \
    do {                                                                           \
        uint32_t _n = (node);                                                      \
        if (s->qstamp[_n] != stamp) {                                              \
            s->qstamp[_n] = stamp;                                                 \
            uint32_t _l = gr->level[_n];                                           \
            s->bucket[s->boff[_l] + s->bfill[_l]++] = _n;                          \
        }                                                                          \
    } while (0)
        cycles = t + 1;
        /* registers whose D diverged in the previous cycle */
        for (uint32_t i = 0; i < nnext; ++i) {
            uint32_t r = s->rnext[i];
            s->rstate[r] = s->rnextv[i];
            s->rstamp[r] = stamp;
            words += 2u * o_ww(&d->nd[r]);
            lastreg = t;
            O1_PUSH(r);
        }
        nnext = 0;
        O1_PUSH(f->site);
        for (uint32_t l = 0; l < gr->nlevels; ++l) {
            for (uint32_t j = 0; j < s->bfill[l]; ++j) {
                uint32_t n = s->bucket[s->boff[l] + j];
                const o_node* x = &d->nd[n];
                int div_in = 0;
                uint64_t v;
                if (x->op == O_CONST) {
                    v = x->param & o_mask(x->width);
                } else if (x->op == O_PI) {
                    v = row[x->param] & o_mask(x->width);
                } else if (x->op == O_REG) {
                    div_in = s->rstamp[n] == stamp;
                    v = div_in ? s->rstate[n] : g[n];
                } else {
                    uint64_t op[3] = {0, 0, 0};
                    for (int k = 0; k < o_arity[x->op]; ++k) {
                        uint32_t in = x->in[k];
                        if (s->fstamp[in] == stamp) { op[k] = s->fval[in]; div_in = 1; }
                        else op[k] = g[in];
                    }
                    v = o_apply(x, d->nd, op[0], op[1], op[2]);
                }
                if (n == f->site) v = o_force(v, f, t);
                int div_out = v != g[n];
                if (div_in || div_out) { ev++; words += o_event_words(x); }
                if (!div_out) continue;
                s->fval[n] = v;
                s->fstamp[n] = stamp;
                for (uint32_t e = gr->fo_off[n]; e < gr->fo_off[n + 1]; ++e) O1_PUSH(gr->fo[e]);
                for (uint32_t e = gr->rfo_off[n]; e < gr->rfo_off[n + 1]; ++e) {
                    uint32_t r = gr->rfo[e];
                    s->rnext[nnext] = r;
                    s->rnextv[nnext] = v & o_mask(d->nd[r].width);
                    nnext++;
                }
                if (gr->is_po[n] && detect == O_UNDET) detect = t;
            }
        }
#undef O1_PUSH
        if (drop && detect != O_UNDET) break;
    }
    *detect_out = detect;
    if (events_out) *events_out = ev;
    if (words_out) *words_out = words + (uint64_t)cycles * o_ww(&d->nd[f->site]);
    if (lastreg_out) *lastreg_out = lastreg;
}

/* ------------------------------------------------------------------------- */
/* Thread pool over faults.                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int variant;
    const o_design* d;
    const o1_graph* gr;
    const uint64_t* stim;
    uint32_t T;
    const uint64_t* G;
    const o_fault* faults;
    uint32_t F;
    int drop;
    uint32_t* detect;
    uint64_t* events;
    uint64_t* words;
    uint32_t* lastreg;
    atomic_uint next;
    atomic_int failed;
} o_job;

static void* o_worker(void* arg)
{
    o_job* j = (o_job*)arg;
    const uint32_t N = j->d->N;
    const size_t n1 = N ? N : 1;
    if (j->variant == 0) {
        o0_scratch s;
        s.val = calloc(n1, sizeof(uint64_t));
        s.state = calloc(n1, sizeof(uint64_t));
        if (!s.val || !s.state) { atomic_store(&j->failed, 1); free(s.val); free(s.state); return NULL; }
        for (;;) {
            uint32_t i = atomic_fetch_add(&j->next, 1u);
            if (i >= j->F) break;
            o0_one(j->d, j->stim, j->T, j->G, &j->faults[i], j->drop, &s, &j->detect[i],
                   j->events ? &j->events[i] : NULL, j->words ? &j->words[i] : NULL,
                   j->lastreg ? &j->lastreg[i] : NULL);
        }
        free(s.val); free(s.state);
    } else {
        o1_scratch s;
        const o1_graph* gr = j->gr;
        memset(&s, 0, sizeof(s));
        s.fval = calloc(n1, sizeof(uint64_t));
        s.fstamp = calloc(n1, sizeof(uint32_t));
        s.qstamp = calloc(n1, sizeof(uint32_t));
        s.rstate = calloc(n1, sizeof(uint64_t));
        s.rstamp = calloc(n1, sizeof(uint32_t));
        s.bucket = calloc(n1, sizeof(uint32_t));
        s.bfill = calloc(gr->nlevels, sizeof(uint32_t));
        s.boff = calloc(gr->nlevels + 1, sizeof(uint32_t));
        s.rnext = calloc(n1, sizeof(uint32_t));
        s.rnextv = calloc(n1, sizeof(uint64_t));
        if (!s.fval || !s.fstamp || !s.qstamp || !s.rstate || !s.rstamp || !s.bucket || !s.bfill ||
            !s.boff || !s.rnext || !s.rnextv) {
            atomic_store(&j->failed, 1);
        } else {
            for (uint32_t n = 0; n < N; ++n) s.boff[gr->level[n] + 1]++;
            for (uint32_t l = 0; l < gr->nlevels; ++l) s.boff[l + 1] += s.boff[l];
            for (;;) {
                uint32_t i = atomic_fetch_add(&j->next, 1u);
                if (i >= j->F) break;
                /* fresh stamps per fault: clear the stamp arrays */
                memset(s.fstamp, 0, n1 * sizeof(uint32_t));
                memset(s.qstamp, 0, n1 * sizeof(uint32_t));
                memset(s.rstamp, 0, n1 * sizeof(uint32_t));
                o1_one(j->d, gr, j->stim, j->T, j->G, &j->faults[i], j->drop, &s, &j->detect[i],
                       j->events ? &j->events[i] : NULL, j->words ? &j->words[i] : NULL,
                       j->lastreg ? &j->lastreg[i] : NULL);
            }
        }
        free(s.fval); free(s.fstamp); free(s.qstamp); free(s.rstate); free(s.rstamp);
        free(s.bucket); free(s.bfill); free(s.boff); free(s.rnext); free(s.rnextv);
    }
    return NULL;
}

/*
 * Fault simulation of F faults.  variant 0 = O0, 1 = O1.  G is the golden trace
 * from oracle_golden.  detect[F] and events[F], words[F] and lastreg[F] (the
 * last three may be NULL) are written.  nthreads <= 0 means 1.  Returns 0, or
 * a negative code for an invalid design (-1), a combinational cycle (-2),
 * memory (-3) or an invalid fault (-4).
 */
int oracle_fault_sim_ex(int variant, const void* nodes, uint32_t N, const uint32_t* po, uint32_t npo,
                        uint32_t npi, const uint64_t* stim, uint32_t T, const uint64_t* G,
                        const void* faults, uint32_t F, int drop, int nthreads, uint32_t* detect,
                        uint64_t* events, uint64_t* words, uint32_t* lastreg)
{
    o_design d;
    int rc = o_prepare(&d, nodes, N, po, npo, npi);
    if (rc) return rc;
    const o_fault* fl = (const o_fault*)faults;
    for (uint32_t i = 0; i < F; ++i)
        if (fl[i].site >= N || fl[i].bit >= d.nd[fl[i].site].width || fl[i].stuck > O_FLIP) {
            o_release(&d);
            return -4;
        }
    o1_graph gr;
    memset(&gr, 0, sizeof(gr));
    if (variant == 1 && (rc = o1_build(&d, &gr)) != 0) { o1_free(&gr); o_release(&d); return rc; }
    o_job j;
    j.variant = variant; j.d = &d; j.gr = &gr; j.stim = stim; j.T = T; j.G = G; j.faults = fl;
    j.F = F; j.drop = drop; j.detect = detect; j.events = events; j.words = words; j.lastreg = lastreg;
    atomic_init(&j.next, 0u);
    atomic_init(&j.failed, 0);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 1; i < nthreads; ++i)
        if (pthread_create(&th[started], NULL, o_worker, &j) == 0) started++;
    o_worker(&j);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    if (variant == 1) o1_free(&gr);
    o_release(&d);
    return atomic_load(&j.failed) ? -3 : 0;
}

/* detect and events only. */
int oracle_fault_sim(int variant, const void* nodes, uint32_t N, const uint32_t* po, uint32_t npo,
                     uint32_t npi, const uint64_t* stim, uint32_t T, const uint64_t* G,
                     const void* faults, uint32_t F, int drop, int nthreads, uint32_t* detect,
                     uint64_t* events)
{
    return oracle_fault_sim_ex(variant, nodes, N, po, npo, npi, stim, T, G, faults, F, drop, nthreads,
                               detect, events, NULL, NULL);
}
