// Design compiler: turns the caller's node list into the levelised image the
// kernels use.  The paper compiles RTL into a graph of RTL nodes and maps the
// graph one-to-one onto tasks (Sec. IV, Steps 1 and 4); here the graph is
// validated, cut at registers, levelised (level 0 = registers, inputs,
// constants; a combinational node sits one level above its deepest operand)
// and renumbered level by level so that each level is a contiguous id range.
#include "design.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <deque>
#include <thread>

namespace riros {

uint8_t event_words(uint8_t op, uint8_t width)
{
    const uint32_t k = op_is_comb(op) ? (uint32_t)op_arity(op) : 0u;
    return (uint8_t)((k + 2u) * (width > 32 ? 2u : 1u));
}

int op_arity(uint8_t op)
{
    switch (op) {
    case RIROS_OP_CONST: case RIROS_OP_PI: return 0;
    case RIROS_OP_REG: case RIROS_OP_NOT: case RIROS_OP_SHL: case RIROS_OP_SHR:
    case RIROS_OP_SLICE: return 1;
    case RIROS_OP_MUX: return 3;
    default: return 2;
    }
}

bool op_is_comb(uint8_t op)
{
    return op != RIROS_OP_CONST && op != RIROS_OP_PI && op != RIROS_OP_REG;
}

static int fail(std::string& err, int code, const char* fmt, unsigned a = 0, unsigned b = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    err = buf;
    return code;
}

int build_image(const riros_design_desc& d, Image& img, std::string& err)
{
    const uint32_t N = d.num_nodes;
    if (N == 0 || d.nodes == nullptr) return fail(err, RIROS_EINVAL, "design has no nodes");
    if (N >= 0x7FFFFFFFu) return fail(err, RIROS_EINVAL, "too many nodes");
    if (d.num_po > 0 && d.po == nullptr) return fail(err, RIROS_EINVAL, "po is NULL");
    const riros_node* nd = d.nodes;
    for (uint32_t n = 0; n < N; ++n) {
        const riros_node& x = nd[n];
        if (x.op >= RIROS_NUM_OPS) return fail(err, RIROS_EINVAL, "node %u: unknown operator %u", n, x.op);
        if (x.width < 1 || x.width > 64) return fail(err, RIROS_EINVAL, "node %u: width %u not in 1..64", n, x.width);
        for (int k = 0; k < op_arity(x.op); ++k)
            if (x.in[k] >= N) return fail(err, RIROS_EINVAL, "node %u: operand id %u out of range", n, x.in[k]);
        if (x.op == RIROS_OP_PI && x.param >= d.num_pi)
            return fail(err, RIROS_EINVAL, "node %u: PI column %u >= num_pi", n, (unsigned)x.param);
        if (x.op == RIROS_OP_REG && nd[x.in[0]].width != x.width)
            return fail(err, RIROS_EINVAL, "register %u: D input width %u differs", n, nd[x.in[0]].width);
    }
    for (uint32_t i = 0; i < d.num_po; ++i)
        if (d.po[i] >= N) return fail(err, RIROS_EINVAL, "po[%u] = %u out of range", i, d.po[i]);

    // Levels by Kahn's algorithm over combinational edges.
    std::vector<uint32_t> indeg(N, 0), uoff(N + 1, 0), lvl(N, 0);
    for (uint32_t n = 0; n < N; ++n)
        if (op_is_comb(nd[n].op))
            for (int k = 0; k < op_arity(nd[n].op); ++k) { uoff[nd[n].in[k] + 1]++; indeg[n]++; }
    for (uint32_t n = 0; n < N; ++n) uoff[n + 1] += uoff[n];
    std::vector<uint32_t> users(uoff[N]), fill(N, 0);
    for (uint32_t n = 0; n < N; ++n)
        if (op_is_comb(nd[n].op))
            for (int k = 0; k < op_arity(nd[n].op); ++k) {
                uint32_t s = nd[n].in[k];
                users[uoff[s] + fill[s]++] = n;
            }
    std::vector<uint32_t> q;
    q.reserve(N);
    for (uint32_t n = 0; n < N; ++n)
        if (indeg[n] == 0) q.push_back(n);
    for (size_t h = 0; h < q.size(); ++h) {
        uint32_t s = q[h];
        for (uint32_t e = uoff[s]; e < uoff[s + 1]; ++e) {
            uint32_t u = users[e];
            lvl[u] = std::max(lvl[u], lvl[s] + 1);
            if (--indeg[u] == 0) q.push_back(u);
        }
    }
    if (q.size() != N) return fail(err, RIROS_ECYCLE, "combinational loop through %u nodes", (unsigned)(N - q.size()));

    uint32_t L = 0;
    for (uint32_t n = 0; n < N; ++n) L = std::max(L, lvl[n] + 1);

    // Level-major numbering; inside level 0 registers come first.
    auto rank = [&](uint32_t n) -> uint32_t {
        if (lvl[n] != 0) return 3;
        return nd[n].op == RIROS_OP_REG ? 0 : (nd[n].op == RIROS_OP_PI ? 1 : 2);
    };
    std::vector<uint32_t> order(N);
    for (uint32_t n = 0; n < N; ++n) order[n] = n;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (lvl[a] != lvl[b]) return lvl[a] < lvl[b];
        return rank(a) < rank(b);
    });
    img.N = N;
    img.L = L;
    img.npi = d.num_pi;
    img.u2i.assign(N, 0);
    img.i2u = order;
    for (uint32_t i = 0; i < N; ++i) img.u2i[order[i]] = i;
    img.R = 0;
    for (uint32_t n = 0; n < N; ++n) img.R += nd[n].op == RIROS_OP_REG;
    img.lvl_off.assign(L + 1, 0);
    img.level.assign(N, 0);
    for (uint32_t i = 0; i < N; ++i) {
        img.level[i] = lvl[order[i]];
        img.lvl_off[img.level[i] + 1]++;
    }
    for (uint32_t l = 0; l < L; ++l) img.lvl_off[l + 1] += img.lvl_off[l];

    img.desc.assign(N, Desc{});
    for (uint32_t i = 0; i < N; ++i) {
        const riros_node& x = nd[order[i]];
        Desc& o = img.desc[i];
        o.op = x.op;
        o.width = x.width;
        uint64_t m = x.width >= 64 ? ~0ull : ((1ull << x.width) - 1);
        switch (x.op) {
        case RIROS_OP_CONST:
            o.a = (uint32_t)(x.param & m);
            o.b = (uint32_t)((x.param & m) >> 32);
            break;
        case RIROS_OP_PI:
            o.a = (uint32_t)x.param;
            break;
        case RIROS_OP_REG:
            o.a = img.u2i[x.in[0]];
            o.b = (uint32_t)(x.param & m);
            o.c = (uint32_t)((x.param & m) >> 32);
            break;
        case RIROS_OP_SHL: case RIROS_OP_SHR: case RIROS_OP_SLICE:
            o.a = img.u2i[x.in[0]];
            o.b = x.param >= 64 ? 64u : (uint32_t)x.param;
            break;
        case RIROS_OP_NOT:
            o.a = img.u2i[x.in[0]];
            break;
        case RIROS_OP_CONCAT:
            o.a = img.u2i[x.in[0]];
            o.b = img.u2i[x.in[1]];
            o.c = nd[x.in[1]].width;
            break;
        case RIROS_OP_MUX:
            o.a = img.u2i[x.in[0]];
            o.b = img.u2i[x.in[1]];
            o.c = img.u2i[x.in[2]];
            break;
        default:
            o.a = img.u2i[x.in[0]];
            o.b = img.u2i[x.in[1]];
            break;
        }
    }

    // Fan-out tables in internal numbering; a user that reads a node twice is listed once.
    std::vector<std::vector<uint32_t>> fo(N), rfo(N);
    for (uint32_t i = 0; i < N; ++i) {
        const Desc& o = img.desc[i];
        if (o.op == RIROS_OP_REG) {
            rfo[o.a].push_back(i);
            continue;
        }
        if (!op_is_comb(o.op)) continue;
        int ar = op_arity(o.op);
        uint32_t ins[3] = {o.a, o.b, o.c};
        for (int k = 0; k < ar; ++k) {
            bool dup = false;
            for (int j = 0; j < k; ++j) dup |= ins[j] == ins[k];
            if (!dup) fo[ins[k]].push_back(i);
        }
    }
    img.fo_off.assign(N + 1, 0);
    img.rfo_off.assign(N + 1, 0);
    for (uint32_t i = 0; i < N; ++i) {
        img.fo_off[i + 1] = img.fo_off[i] + (uint32_t)fo[i].size();
        img.rfo_off[i + 1] = img.rfo_off[i] + (uint32_t)rfo[i].size();
    }
    img.fo.clear();
    img.fo_lvl.clear();
    img.fo_pk.clear();
    img.rfo.clear();
    for (uint32_t i = 0; i < N; ++i) {
        std::sort(fo[i].begin(), fo[i].end());
        for (uint32_t u : fo[i]) {
            img.fo.push_back(u);
            img.fo_lvl.push_back(img.level[u]);
            img.fo_pk.push_back((uint64_t)u | ((uint64_t)img.level[u] << 32));
        }
        for (uint32_t r : rfo[i]) img.rfo.push_back(r);
        if (!fo[i].empty()) img.desc[i].flags |= DF_COMBFO;
        if (!rfo[i].empty()) img.desc[i].flags |= DF_REGFO;
    }
    // Each table ends in kFanoutPad zero entries, so that a kernel may read
    // the first kFanoutPad entries of any node's list without a bounds check
    // (issuing them together with the operand loads) and use those in range.
    for (uint32_t k = 0; k < kFanoutPad; ++k) {
        img.fo.push_back(0);
        img.fo_pk.push_back(0);
        img.rfo.push_back(0);
    }
    std::vector<uint8_t> seen(N, 0);
    img.po.clear();
    img.rec.assign(N, NodeRec{});
    img.bp_off.assign(N, 0);
    uint32_t rows = 0;
    for (uint32_t i = 0; i < d.num_po; ++i) {
        uint32_t p = img.u2i[d.po[i]];
        if (!seen[p]) { seen[p] = 1; img.po.push_back(p); img.desc[p].flags |= DF_PO; }
    }
    for (uint32_t i = 0; i < N; ++i) {
        const Desc& o = img.desc[i];
        NodeRec& r = img.rec[i];
        r.op = o.op;
        r.width = o.width;
        r.flags = o.flags;
        r.a = o.a;
        r.b = o.b;
        r.c = o.c;
        r.fo0 = img.fo_off[i];
        r.fo1 = img.fo_off[i + 1];
        r.rfo0 = img.rfo_off[i];
        r.rfo1 = img.rfo_off[i + 1];
        r.words = event_words(o.op, o.width);
        img.bp_off[i] = rows;
        rows += o.width;
        img.max_width = std::max<uint32_t>(img.max_width, o.width);
    }
    img.bp_rows = rows;
    img.lrec.assign(N, LaneRec{});
    for (uint32_t i = 0; i < N; ++i) {
        const NodeRec& r = img.rec[i];
        LaneRec& l = img.lrec[i];
        l.op = r.op;
        l.width = r.width;
        l.flags = r.flags;
        l.words = r.words;
        l.a = r.a;
        l.b = r.b;
        l.c = r.c;
        l.fo0 = r.fo0;
        l.fo1 = r.fo1;
        l.rfo0 = r.rfo0;
        l.rfo1 = r.rfo1;
        for (uint32_t k = 0; k < 4; ++k) l.u[k] = img.fo[r.fo0 + k];   // padded: always in the table
        l.r0 = img.rfo[r.rfo0];
        const bool comb = r.op != RIROS_OP_REG && r.op != RIROS_OP_PI && r.op != RIROS_OP_CONST;
        const uint32_t ar = comb ? (uint32_t)op_arity(r.op) : 0u;
        l.o[0] = ar > 0 ? r.a : i;
        l.o[1] = ar > 1 ? r.b : l.o[0];
        l.o[2] = ar > 2 ? r.c : l.o[0];
    }
    return RIROS_OK;
}

// Golden-machine parts: union-find over the non-source nodes, components
// packed longest first into the emptiest part (LPT), then each part's local
// program in level order.
bool build_golden_parts(const Image& img, uint32_t max_parts, GoldenParts& gp)
{
    gp = GoldenParts{};
    const uint32_t N = img.N;
    auto source = [&](uint32_t n) { return img.desc[n].op == RIROS_OP_PI || img.desc[n].op == RIROS_OP_CONST; };
    std::vector<uint32_t> up(N);
    for (uint32_t i = 0; i < N; ++i) up[i] = i;
    auto find = [&](uint32_t x) {
        while (up[x] != x) {
            up[x] = up[up[x]];
            x = up[x];
        }
        return x;
    };
    auto operands = [&](uint32_t n, uint32_t* ops) -> uint32_t {
        const Desc& d = img.desc[n];
        if (d.op == RIROS_OP_REG) {
            ops[0] = d.a;
            return 1;
        }
        if (!op_is_comb(d.op)) return 0;
        const uint32_t k = (uint32_t)op_arity(d.op);
        ops[0] = d.a;
        if (k > 1) ops[1] = d.b;
        if (k > 2) ops[2] = d.c;
        return k;
    };
    for (uint32_t n = 0; n < N; ++n) {
        if (source(n)) continue;
        uint32_t ops[3];
        const uint32_t k = operands(n, ops);
        for (uint32_t j = 0; j < k; ++j)
            if (!source(ops[j])) {
                const uint32_t a = find(n), b = find(ops[j]);
                if (a != b) up[a] = b;
            }
    }
    // Components: their nodes and the sources they read.
    std::vector<uint32_t> comp_of(N, kNoGid);
    std::vector<std::vector<uint32_t>> members;
    for (uint32_t n = 0; n < N; ++n) {
        if (source(n)) continue;
        const uint32_t r = find(n);
        if (comp_of[r] == kNoGid) {
            comp_of[r] = (uint32_t)members.size();
            members.emplace_back();
        }
        members[comp_of[r]].push_back(n);
    }
    const uint32_t C = (uint32_t)members.size();
    std::vector<uint32_t> csize(C);
    for (uint32_t c = 0; c < C; ++c) {
        std::vector<uint32_t> src;
        for (uint32_t n : members[c]) {
            uint32_t ops[3];
            const uint32_t k = operands(n, ops);
            for (uint32_t j = 0; j < k; ++j)
                if (source(ops[j])) src.push_back(ops[j]);
        }
        std::sort(src.begin(), src.end());
        src.erase(std::unique(src.begin(), src.end()), src.end());
        csize[c] = (uint32_t)(members[c].size() + src.size());
        if (csize[c] > kGoldenPartCap) return false;
    }
    if (C == 0) return false;
    // LPT packing; more parts while one exceeds the cap (sources shared by
    // components of a part are counted once there, so the sum bounds it).
    std::vector<uint32_t> order(C);
    for (uint32_t c = 0; c < C; ++c) order[c] = c;
    std::sort(order.begin(), order.end(),
              [&](uint32_t x, uint32_t y) { return csize[x] > csize[y] || (csize[x] == csize[y] && x < y); });
    uint32_t P = std::max<uint32_t>(1, std::min(C, max_parts));
    std::vector<uint32_t> part_of(C);
    for (;;) {
        std::vector<uint64_t> load(P, 0);
        bool fits = true;
        for (uint32_t c : order) {
            uint32_t best = 0;
            for (uint32_t p = 1; p < P; ++p)
                if (load[p] < load[best]) best = p;
            part_of[c] = best;
            load[best] += csize[c];
            if (load[best] > kGoldenPartCap) fits = false;
        }
        if (fits) break;
        if (P >= C) return false;
        P = std::min(C, P * 2);
    }
    // Local programs.  Owned sources: a source belongs to the first part that
    // reads it; sources nobody reads go to parts of their own (at most
    // kGoldenPartCap each) after the others.
    std::vector<std::vector<uint32_t>> parts(P);
    for (uint32_t c = 0; c < C; ++c)
        for (uint32_t n : members[c]) parts[part_of[c]].push_back(n);
    {
        std::vector<uint8_t> read(N, 0);
        for (uint32_t n = 0; n < N; ++n) {
            if (source(n)) continue;
            uint32_t ops[3];
            const uint32_t k = operands(n, ops);
            for (uint32_t j = 0; j < k; ++j) read[ops[j]] = 1;
        }
        std::vector<uint32_t> unread;
        for (uint32_t n = 0; n < N; ++n)
            if (source(n) && !read[n]) unread.push_back(n);
        for (size_t i = 0; i < unread.size(); i += kGoldenPartCap)
            parts.emplace_back(unread.begin() + i,
                               unread.begin() + std::min(unread.size(), (size_t)i + kGoldenPartCap));
        P = (uint32_t)parts.size();
    }
    std::vector<uint8_t> owned_src(N, 0);
    std::vector<uint32_t> loc(N, kNoGid);
    gp.part_off.push_back(0);
    gp.lvl_off.push_back(0);
    for (uint32_t p = 0; p < P; ++p) {
        std::vector<uint32_t> nodes = parts[p];
        std::vector<uint32_t> src;
        for (uint32_t n : parts[p]) {
            uint32_t ops[3];
            const uint32_t k = operands(n, ops);
            for (uint32_t j = 0; j < k; ++j)
                if (source(ops[j])) src.push_back(ops[j]);
        }
        std::sort(src.begin(), src.end());
        src.erase(std::unique(src.begin(), src.end()), src.end());
        nodes.insert(nodes.end(), src.begin(), src.end());
        std::sort(nodes.begin(), nodes.end(), [&](uint32_t x, uint32_t y) {
            return img.level[x] < img.level[y] || (img.level[x] == img.level[y] && x < y);
        });
        for (uint32_t i = 0; i < nodes.size(); ++i) loc[nodes[i]] = i;
        uint32_t prev_level = 0xFFFFFFFFu;
        for (uint32_t i = 0; i < nodes.size(); ++i) {
            const uint32_t n = nodes[i];
            const Desc& d = img.desc[n];
            GNode g{d.op, d.width, 0, 0, d.a, d.b, d.c, n};
            if (source(n)) {
                if (owned_src[n]) g.gid = kNoGid;
                owned_src[n] = 1;
            } else if (d.op == RIROS_OP_REG) {
                g.a = loc[d.a];
            } else {
                const uint32_t k = (uint32_t)op_arity(d.op);
                g.a = loc[d.a];
                if (k > 1) g.b = loc[d.b];
                if (k > 2) g.c = loc[d.c];
            }
            if (img.level[n] != prev_level) {
                gp.lvl.push_back(i);
                prev_level = img.level[n];
            }
            gp.node.push_back(g);
        }
        gp.lvl.push_back((uint32_t)nodes.size());
        for (uint32_t n : nodes) loc[n] = kNoGid;
        gp.part_off.push_back((uint32_t)gp.node.size());
        gp.lvl_off.push_back((uint32_t)gp.lvl.size());
        gp.max_nodes = std::max<uint32_t>(gp.max_nodes, (uint32_t)nodes.size());
    }
    return true;
}

// Predictor graph features.  The cone of a node is the number of distinct
// nodes reached through combinational users, registers fed counted but not
// crossed, the node itself excluded, capped at kConeCap.  Register depth is a
// 0-1 breadth-first search backwards from the outputs: crossing a register
// from its output to its D input costs one.
void node_features(const Image& img, std::vector<float>& out)
{
    const uint32_t N = img.N;
    out.assign((size_t)N * 4, 0.f);
    const float maxl = (float)std::max<uint32_t>(1, img.L - 1);
    // register depth
    const int INF = 1 << 30;
    std::vector<int> dist(N, INF);
    std::deque<uint32_t> dq;
    for (uint32_t p : img.po) { dist[p] = 0; dq.push_back(p); }
    while (!dq.empty()) {
        const uint32_t u = dq.front();
        dq.pop_front();
        const Desc& x = img.desc[u];
        if (x.op == RIROS_OP_REG) {
            if (dist[u] + 1 < dist[x.a]) { dist[x.a] = dist[u] + 1; dq.push_back(x.a); }
        } else if (op_is_comb(x.op)) {
            const uint32_t ins[3] = {x.a, x.b, x.c};
            for (int k = 0; k < op_arity(x.op); ++k)
                if (dist[u] < dist[ins[k]]) { dist[ins[k]] = dist[u]; dq.push_front(ins[k]); }
        }
    }
    // cones, in parallel over nodes
    std::vector<uint32_t> cone(N, 0);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&](unsigned tid) {
        std::vector<uint32_t> seen(N, 0), q;
        q.reserve(kConeCap + 64);
        uint32_t mark = 0;
        for (uint32_t s = tid; s < N; s += nt) {
            ++mark;
            seen[s] = mark;
            q.clear();
            q.push_back(s);
            uint32_t count = 0;
            for (size_t h = 0; h < q.size() && count < kConeCap; ++h) {
                const uint32_t u = q[h];
                for (uint32_t e = img.fo_off[u]; e < img.fo_off[u + 1]; ++e) {
                    const uint32_t c = img.fo[e];
                    if (seen[c] != mark) { seen[c] = mark; ++count; q.push_back(c); }
                }
                for (uint32_t e = img.rfo_off[u]; e < img.rfo_off[u + 1]; ++e) {
                    const uint32_t r = img.rfo[e];
                    if (seen[r] != mark) { seen[r] = mark; ++count; }
                }
            }
            cone[s] = std::min(count, kConeCap);
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& t : th) t.join();
    for (uint32_t n = 0; n < N; ++n) {
        float* o = &out[(size_t)n * 4];
        o[0] = (float)std::log2(1.0 + (double)cone[n]);
        o[1] = (float)img.level[n] / maxl;
        o[2] = dist[n] >= INF ? -1.f : (float)std::min(dist[n], kDepthCap);
        o[3] = (float)std::log2((double)img.desc[n].width);
    }
}

}  // namespace riros
