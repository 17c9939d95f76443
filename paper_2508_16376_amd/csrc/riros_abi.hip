// C interface of the simulator: design and golden-trace handles, fault
// simulation entry point, errors and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "concurrent.hpp"
#include "design.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "riros.h"
#include "twod.hpp"
#include "wave_fault.hpp"

namespace {

thread_local std::string g_err;
thread_local hipEvent_t g_ev0 = nullptr, g_ev1 = nullptr;
thread_local bool g_ev_valid = false;

int set_err(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

bool valid_share(int32_t v)
{
    return v == 0 || v == 1 || v == 2 || v == 4;
}

bool valid_heavy_wg(int32_t v)
{
    return v == 0 || v == 64 || v == 128 || v == 256;
}

bool valid_deal(int32_t v)
{
    return v == 0 || v == 4 || v == 8 || v == 16 || v == 32;
}

bool valid_head_lanes(int32_t v)
{
    return v >= 0 && v <= 64;
}

int hip_err(hipError_t e, const char* what)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_err = buf;
    return e == hipErrorOutOfMemory ? RIROS_ENOMEM : RIROS_EDEVICE;
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t _e = (call);                     \
        if (_e != hipSuccess) return hip_err(_e, what); \
    } while (0)

template <class T>
hipError_t dev_upload(T** dst, const std::vector<T>& src)
{
    size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return hipSuccess;
}

// Device buffer freed on scope exit.
template <class T>
struct DevBuf {
    T* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc((void**)&p, std::max<size_t>(n, 1) * sizeof(T)); }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct riros_design_s {
    riros::Image img;
    int device = 0;
    int num_cu = 0;
    riros::DevDesign dev{};
    std::vector<void*> owned;
    // plain-kernel workspace (grow-only)
    riros::Slot* ws_slots = nullptr;
    size_t ws_slots_cap = 0;
    uint64_t* ws_regs = nullptr;
    size_t ws_regs_cap = 0;
    uint64_t* stamp_dev = nullptr;   // slot stamps above this are unused (advanced on the device by every run)
    uint64_t* ws_words = nullptr;    // per-fault byte-model words when the caller asks for none (grow-only)
    size_t ws_words_cap = 0;
    // golden machine by parts (P = 0: one workgroup for the whole design)
    riros::DevGoldenParts gparts{};
    // two-dimensional kernel workspace
    riros::TwoDWorkspace twod{};
    // concurrent (node-major) mode workspace
    riros::ConcWorkspace conc{};
    // staging for host-side inputs and outputs
    void* stage = nullptr;
    size_t stage_cap = 0;
    riros_coverage* d_cov = nullptr;
    uint32_t* d_bad = nullptr;
    float4* d_nodefeat = nullptr;   // predictor graph features, computed on first use
};

struct riros_golden_s {
    riros_design d = nullptr;
    uint32_t T = 0;
    uint64_t* G = nullptr;    // row-major [T][N]
    uint64_t* Gn = nullptr;   // node-major [N][T]
    uint64_t* Bp = nullptr;   // bit-planes [bp_rows][ceil(T/64)]
    uint32_t* Gn32 = nullptr; // node-major 32-bit copy [N][T] when no node is wider than 32 bits
    uint64_t* stim = nullptr; // the stimulus [T][npi] (a campaign graph may recompute the trace)
    riros::GoldenView view() const { return riros::GoldenView{G, Gn, Bp, T, (T + 63) / 64, Gn32}; }
};

static void free_golden_mem(riros_golden g)
{
    if (g->G) (void)hipFree(g->G);
    if (g->Gn) (void)hipFree(g->Gn);
    if (g->Bp) (void)hipFree(g->Bp);
    if (g->Gn32) (void)hipFree(g->Gn32);
    if (g->stim) (void)hipFree(g->stim);
    g->G = g->Gn = g->Bp = g->stim = nullptr;
    g->Gn32 = nullptr;
}

// Device buffers of one golden trace and its uploaded stimulus.
static hipError_t alloc_golden(riros_golden g, const uint64_t* stimulus, hipStream_t s)
{
    const riros_design d = g->d;
    const uint32_t T = g->T;
    const size_t gbytes = (size_t)T * d->img.N * sizeof(uint64_t);
    const size_t bpbytes = std::max<size_t>((size_t)d->img.bp_rows * ((T + 63) / 64), 1) * sizeof(uint64_t);
    const size_t sbytes = std::max<size_t>((size_t)T * d->img.npi, 1) * sizeof(uint64_t);
    hipError_t e = hipMalloc((void**)&g->G, gbytes);
    if (e == hipSuccess) e = hipMalloc((void**)&g->Gn, gbytes);
    if (e == hipSuccess) e = hipMalloc((void**)&g->Bp, bpbytes);
    if (e == hipSuccess && d->img.max_width <= 32) e = hipMalloc((void**)&g->Gn32, gbytes / 2);
    if (e == hipSuccess) e = hipMalloc((void**)&g->stim, sbytes);
    if (e == hipSuccess && d->img.npi > 0)
        e = hipMemcpyAsync(g->stim, stimulus, (size_t)T * d->img.npi * sizeof(uint64_t), hipMemcpyHostToDevice, s);
    return e;
}

static void free_design_mem(riros_design d)
{
    for (void* p : d->owned) (void)hipFree(p);
    d->owned.clear();
    if (d->ws_slots) (void)hipFree(d->ws_slots);
    if (d->ws_regs) (void)hipFree(d->ws_regs);
    if (d->stamp_dev) (void)hipFree(d->stamp_dev);
    if (d->stage) (void)hipFree(d->stage);
    if (d->d_cov) (void)hipFree(d->d_cov);
    if (d->d_bad) (void)hipFree(d->d_bad);
    if (d->d_nodefeat) (void)hipFree(d->d_nodefeat);
    if (d->ws_words) (void)hipFree(d->ws_words);
    riros::twod_free(d->twod);
    riros::conc_free(d->conc);
}

extern "C" {

const char* riros_last_error(void) { return g_err.c_str(); }

int riros_load_design(const riros_design_desc* desc, riros_design* out)
{
    if (!desc || !out) return set_err(RIROS_EINVAL, "NULL argument");
    riros_design d = new (std::nothrow) riros_design_s();
    if (!d) return set_err(RIROS_ENOMEM, "host allocation failed");
    std::string err;
    int rc = riros::build_image(*desc, d->img, err);
    if (rc != RIROS_OK) {
        delete d;
        return set_err(rc, err);
    }
    hipError_t e = hipGetDevice(&d->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&d->num_cu, hipDeviceAttributeMultiprocessorCount, d->device);
    if (e != hipSuccess) {
        delete d;
        return hip_err(e, "device query");
    }
    const riros::Image& im = d->img;
    std::vector<uint8_t> uwidth(im.N);
    for (uint32_t n = 0; n < im.N; ++n) uwidth[n] = desc->nodes[n].width;
    riros::Desc* p_desc = nullptr;
    uint32_t *p_lvl = nullptr, *p_level = nullptr, *p_fo_off = nullptr, *p_fo = nullptr, *p_fo_lvl = nullptr,
             *p_rfo_off = nullptr, *p_rfo = nullptr, *p_u2i = nullptr;
    uint8_t* p_uw = nullptr;
    riros::NodeRec* p_rec = nullptr;
    riros::LaneRec* p_lrec = nullptr;
    uint32_t* p_bp = nullptr;
    uint64_t* p_fopk = nullptr;
    hipError_t es[14] = {dev_upload(&p_rec, im.rec), dev_upload(&p_lrec, im.lrec), dev_upload(&p_bp, im.bp_off),
        dev_upload(&p_fopk, im.fo_pk),
        dev_upload(&p_desc, im.desc),     dev_upload(&p_lvl, im.lvl_off), dev_upload(&p_level, im.level),
        dev_upload(&p_fo_off, im.fo_off), dev_upload(&p_fo, im.fo),       dev_upload(&p_fo_lvl, im.fo_lvl),
        dev_upload(&p_rfo_off, im.rfo_off), dev_upload(&p_rfo, im.rfo),   dev_upload(&p_u2i, im.u2i),
        dev_upload(&p_uw, uwidth)};
    for (void* p : {(void*)p_rec, (void*)p_lrec, (void*)p_bp, (void*)p_fopk, (void*)p_desc, (void*)p_lvl, (void*)p_level, (void*)p_fo_off, (void*)p_fo, (void*)p_fo_lvl,
                    (void*)p_rfo_off, (void*)p_rfo, (void*)p_u2i, (void*)p_uw})
        if (p) d->owned.push_back(p);
    for (hipError_t x : es)
        if (x != hipSuccess) {
            free_design_mem(d);
            delete d;
            return hip_err(x, "design upload");
        }
    d->dev = riros::DevDesign{p_desc, p_lvl, p_level, p_fo_off, p_fo, p_fo_lvl, p_rfo_off, p_rfo, p_u2i, p_uw,
                              p_rec, p_lrec, p_fopk, p_bp, im.N, im.L, im.R, im.npi, im.bp_rows};
    {
        riros::GoldenParts gp;
        if (riros::build_golden_parts(im, 4u * (uint32_t)std::max(1, d->num_cu), gp)) {
            riros::GNode* p_gn = nullptr;
            uint32_t *p_po = nullptr, *p_gl = nullptr, *p_glo = nullptr;
            hipError_t ge[4] = {dev_upload(&p_gn, gp.node), dev_upload(&p_po, gp.part_off), dev_upload(&p_gl, gp.lvl),
                                dev_upload(&p_glo, gp.lvl_off)};
            for (void* p : {(void*)p_gn, (void*)p_po, (void*)p_gl, (void*)p_glo})
                if (p) d->owned.push_back(p);
            for (hipError_t x : ge)
                if (x != hipSuccess) {
                    free_design_mem(d);
                    delete d;
                    return hip_err(x, "design upload");
                }
            d->gparts = riros::DevGoldenParts{p_gn, p_po, p_gl, p_glo, (uint32_t)gp.part_off.size() - 1, gp.max_nodes};
            e = riros::golden_parts_setup();
            if (e != hipSuccess) {
                free_design_mem(d);
                delete d;
                return hip_err(e, "golden parts setup");
            }
        }
    }
    e = hipMalloc((void**)&d->d_cov, sizeof(riros_coverage));
    if (e == hipSuccess) e = hipMalloc((void**)&d->d_bad, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&d->stamp_dev, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(d->stamp_dev, 0, sizeof(uint64_t));
    if (e != hipSuccess) {
        free_design_mem(d);
        delete d;
        return hip_err(e, "design allocation");
    }
    *out = d;
    return RIROS_OK;
}

void riros_free_design(riros_design d)
{
    if (!d) return;
    DeviceGuard g(d->device);
    (void)hipDeviceSynchronize();
    free_design_mem(d);
    delete d;
}

int riros_design_info(riros_design d, uint32_t* num_nodes, uint32_t* num_levels, uint32_t* num_regs)
{
    if (!d) return set_err(RIROS_EINVAL, "NULL design");
    if (num_nodes) *num_nodes = d->img.N;
    if (num_levels) *num_levels = d->img.L;
    if (num_regs) *num_regs = d->img.R;
    return RIROS_OK;
}

// The part jobs of one design's golden machine (for launches of many designs).
static void append_part_jobs(riros_design d, const uint64_t* stim, uint32_t T, uint64_t* G,
                             std::vector<riros::GPartJob>& jobs, uint32_t& max_nodes)
{
    const riros::DevGoldenParts& gp = d->gparts;
    for (uint32_t p = 0; p < gp.P; ++p)
        jobs.push_back(riros::GPartJob{gp.node, gp.part_off, gp.lvl, gp.lvl_off, stim, G, p, d->img.npi, d->img.N, T});
    max_nodes = std::max(max_nodes, gp.max_nodes);
}

// The golden machine of one design: by parts when it has them.
static hipError_t golden_run(riros_design d, const uint64_t* stim, uint32_t T, uint64_t* G, hipStream_t s)
{
    return d->gparts.P ? riros::launch_golden_parts(d->dev, d->gparts, stim, T, G, s)
                       : riros::launch_golden(d->dev, stim, T, G, s);
}

int riros_golden_sim(riros_design d, const uint64_t* stimulus, uint32_t T, void* stream, riros_golden* out)
{
    if (!d || !out) return set_err(RIROS_EINVAL, "NULL argument");
    if (T == 0) return set_err(RIROS_EINVAL, "T must be positive");
    if (d->img.npi > 0 && !stimulus) return set_err(RIROS_EINVAL, "stimulus is NULL");
    DeviceGuard guard(d->device);
    hipStream_t s = (hipStream_t)stream;
    riros_golden g = new (std::nothrow) riros_golden_s();
    if (!g) return set_err(RIROS_ENOMEM, "host allocation failed");
    g->d = d;
    g->T = T;
    hipError_t e = alloc_golden(g, stimulus, s);
    if (e == hipSuccess) e = golden_run(d, g->stim, T, g->G, s);
    if (e == hipSuccess) e = riros::launch_golden_layouts(d->dev, g->G, T, g->Gn, g->Bp, g->Gn32, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_golden_mem(g);
        delete g;
        return hip_err(e, "golden simulation");
    }
    *out = g;
    return RIROS_OK;
}

int riros_golden_sim_many(uint32_t n, const riros_design* designs, const uint64_t* const* stimulus, const uint32_t* T,
                          void* stream, riros_golden* out)
{
    if (!designs || !stimulus || !T || !out) return set_err(RIROS_EINVAL, "NULL argument");
    if (n == 0) return RIROS_OK;
    for (uint32_t i = 0; i < n; ++i) {
        if (!designs[i]) return set_err(RIROS_EINVAL, "design " + std::to_string(i) + " is NULL");
        if (T[i] == 0) return set_err(RIROS_EINVAL, "design " + std::to_string(i) + ": T must be positive");
        if (designs[i]->img.npi > 0 && !stimulus[i])
            return set_err(RIROS_EINVAL, "design " + std::to_string(i) + ": stimulus is NULL");
        if (designs[i]->device != designs[0]->device) return set_err(RIROS_EINVAL, "designs on different devices");
    }
    DeviceGuard guard(designs[0]->device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<riros_golden> gs(n, nullptr);
    std::vector<riros::DevDesign> td(n);
    // Designs in fewer than two parts run one workgroup each in one launch (so
    // they run at the same time); the parts of the others one workgroup each,
    // in a second launch.
    std::vector<riros::GoldenJob> jobs;
    std::vector<riros::GPartJob> pjobs;
    uint32_t pmax = 0;
    DevBuf<riros::GPartJob> dpjobs;
    DevBuf<riros::DevDesign> dtd;
    DevBuf<riros::GoldenJob> djobs;
    hipError_t e = hipSuccess;
    for (uint32_t i = 0; i < n && e == hipSuccess; ++i) {
        gs[i] = new (std::nothrow) riros_golden_s();
        if (!gs[i]) { e = hipErrorOutOfMemory; break; }
        gs[i]->d = designs[i];
        gs[i]->T = T[i];
        e = alloc_golden(gs[i], stimulus[i], s);
        td[i] = designs[i]->dev;
        if (designs[i]->gparts.P < 2) jobs.push_back(riros::GoldenJob{gs[i]->stim, gs[i]->G, T[i], i});
        else append_part_jobs(designs[i], gs[i]->stim, T[i], gs[i]->G, pjobs, pmax);
    }
    const uint32_t npj = (uint32_t)pjobs.size();
    if (e == hipSuccess && npj) e = dpjobs.alloc(npj);
    if (e == hipSuccess && npj)
        e = hipMemcpyAsync(dpjobs.p, pjobs.data(), npj * sizeof(riros::GPartJob), hipMemcpyHostToDevice, s);
    const uint32_t nj = (uint32_t)jobs.size();
    if (e == hipSuccess && nj) e = dtd.alloc(n);
    if (e == hipSuccess && nj) e = djobs.alloc(nj);
    if (e == hipSuccess && nj)
        e = hipMemcpyAsync(dtd.p, td.data(), n * sizeof(riros::DevDesign), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nj)
        e = hipMemcpyAsync(djobs.p, jobs.data(), nj * sizeof(riros::GoldenJob), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = riros::launch_golden_many(nj, dtd.p, djobs.p, s);
    if (e == hipSuccess) e = riros::launch_golden_parts_many(npj, dpjobs.p, pmax, s);
    for (uint32_t i = 0; i < n && e == hipSuccess; ++i)
        e = riros::launch_golden_layouts(designs[i]->dev, gs[i]->G, T[i], gs[i]->Gn, gs[i]->Bp, gs[i]->Gn32, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        for (riros_golden g : gs)
            if (g) {
                free_golden_mem(g);
                delete g;
            }
        return hip_err(e, "golden simulation of many designs");
    }
    for (uint32_t i = 0; i < n; ++i) out[i] = gs[i];
    return RIROS_OK;
}

void riros_free_golden(riros_golden g)
{
    if (!g) return;
    DeviceGuard guard(g->d->device);
    (void)hipDeviceSynchronize();
    free_golden_mem(g);
    delete g;
}

int riros_golden_read(riros_golden g, uint32_t t0, uint32_t nt, uint64_t* out)
{
    if (!g || !out) return set_err(RIROS_EINVAL, "NULL argument");
    if ((uint64_t)t0 + nt > g->T) return set_err(RIROS_EINVAL, "cycle range outside the trace");
    DeviceGuard guard(g->d->device);
    const uint32_t N = g->d->img.N;
    std::vector<uint64_t> buf((size_t)nt * N);
    HIP_TRY(hipMemcpy(buf.data(), g->G + (size_t)t0 * N, buf.size() * sizeof(uint64_t), hipMemcpyDeviceToHost),
            "golden read");
    const std::vector<uint32_t>& i2u = g->d->img.i2u;
    for (uint32_t t = 0; t < nt; ++t)
        for (uint32_t i = 0; i < N; ++i) out[(size_t)t * N + i2u[i]] = buf[(size_t)t * N + i];
    return RIROS_OK;
}

int riros_last_kernel_ms(float* ms)
{
    if (!ms) return set_err(RIROS_EINVAL, "NULL argument");
    if (!g_ev_valid) return set_err(RIROS_EINVAL, "no fault simulation recorded on this thread");
    HIP_TRY(hipEventSynchronize(g_ev1), "event sync");
    HIP_TRY(hipEventElapsedTime(ms, g_ev0, g_ev1), "event time");
    return RIROS_OK;
}

static int ensure_stage(riros_design d, size_t bytes)
{
    if (d->stage_cap >= bytes) return RIROS_OK;
    if (d->stage) (void)hipFree(d->stage);
    d->stage = nullptr;
    d->stage_cap = 0;
    HIP_TRY(hipMalloc(&d->stage, bytes), "staging allocation");
    d->stage_cap = bytes;
    return RIROS_OK;
}

static int ensure_plain_ws(riros_design d, uint32_t blocks, hipStream_t s)
{
    const size_t nslots = (size_t)blocks * d->img.N;
    const size_t nregs = std::max<size_t>((size_t)blocks * 2 * d->img.R, 1);
    if (d->ws_slots_cap < nslots) {
        HIP_TRY(hipStreamSynchronize(s), "workspace sync");
        if (d->ws_slots) (void)hipFree(d->ws_slots);
        d->ws_slots = nullptr;
        d->ws_slots_cap = 0;
        HIP_TRY(hipMalloc((void**)&d->ws_slots, nslots * sizeof(riros::Slot)), "workspace allocation");
        HIP_TRY(hipMemsetAsync(d->ws_slots, 0, nslots * sizeof(riros::Slot), s), "workspace clear");
        d->ws_slots_cap = nslots;
    }
    if (d->ws_regs_cap < nregs) {
        HIP_TRY(hipStreamSynchronize(s), "workspace sync");
        if (d->ws_regs) (void)hipFree(d->ws_regs);
        d->ws_regs = nullptr;
        d->ws_regs_cap = 0;
        HIP_TRY(hipMalloc((void**)&d->ws_regs, nregs * sizeof(uint64_t)), "workspace allocation");
        d->ws_regs_cap = nregs;
    }
    return RIROS_OK;
}

int riros_fault_sim(riros_design d, riros_golden g, const riros_fault* faults, uint32_t F,
                    const riros_sim_opts* opts, uint32_t* detect, uint64_t* events, riros_coverage* cov)
{
    if (!d || !g || !opts) return set_err(RIROS_EINVAL, "NULL argument");
    if (g->d != d) return set_err(RIROS_EINVAL, "golden trace belongs to another design");
    if (F > 0 && (!faults || !detect)) return set_err(RIROS_EINVAL, "faults or detect is NULL");
    if (opts->mode != RIROS_MODE_PLAIN && opts->mode != RIROS_MODE_TWO_D && opts->mode != RIROS_MODE_CONCURRENT)
        return set_err(RIROS_EINVAL, "unknown mode");
    if (opts->waves_per_cu < 0 || (opts->unified != 0 && opts->unified != 1) || !(opts->monitor_rate >= 0.f) ||
        (opts->light_cap != 0 && opts->light_cap != 4 && opts->light_cap != 8 && opts->light_cap != 16) ||
        !valid_share(opts->struct_share) || !valid_heavy_wg(opts->heavy_wg) || !valid_deal(opts->deal) ||
        !valid_head_lanes(opts->head_lanes) ||
        (opts->xcd_queues != 0 && opts->xcd_queues != 1) || (opts->lockstep != 0 && opts->lockstep != 1))
        return set_err(RIROS_EINVAL, "invalid option (waves_per_cu < 0, unified not 0 or 1, bad monitor_rate, "
                                     "light_cap not 0, 4, 8 or 16, struct_share not 0, 1, 2 or 4, heavy_wg "
                                     "not 0, 64, 128 or 256, deal not 0, 4, 8, 16 or 32, head_lanes not "
                                     "in 0..64, xcd_queues or lockstep not 0 or 1)");
    DeviceGuard guard(d->device);
    hipStream_t s = (hipStream_t)opts->stream;
    const bool on_dev = opts->io_on_device != 0;
    const uint32_t T = g->T;
    const riros::Image& im = d->img;

    if (!g_ev0) {
        HIP_TRY(hipEventCreate(&g_ev0), "event create");
        HIP_TRY(hipEventCreate(&g_ev1), "event create");
    }

    // Faults: validate, and stage host lists on the device.
    const riros_fault* d_faults = faults;
    uint32_t* d_detect = detect;
    uint64_t* d_events = events;
    uint64_t* d_words = opts->words;
    const float* d_prio = opts->priority;
    if (!on_dev) {
        for (uint32_t i = 0; i < F; ++i) {
            const riros_fault& f = faults[i];
            if (f.site >= im.N || f.stuck > RIROS_FAULT_FLIP || f.bit >= d->img.desc[im.u2i[f.site]].width) {
                char buf[128];
                std::snprintf(buf, sizeof buf, "fault %u: site %u bit %u stuck %u invalid", i, f.site, f.bit,
                              f.stuck);
                return set_err(RIROS_EINVAL, buf);
            }
        }
        if (F == 0) {
            if (cov) *cov = riros_coverage{0, 0, 0, 0, 0};
            return RIROS_OK;
        }
        const size_t fb = (size_t)F * sizeof(riros_fault), db = (size_t)F * 4, eb = (size_t)F * 8,
                     pb = opts->priority ? (size_t)F * 4 : 0;
        int rc = ensure_stage(d, fb + db + 2 * eb + pb + 256);
        if (rc) return rc;
        char* base = (char*)d->stage;
        d_faults = (const riros_fault*)base;
        d_detect = (uint32_t*)(base + fb);
        d_events = (uint64_t*)(base + fb + db + (8 - (fb + db) % 8) % 8);
        d_words = d_events + F;
        HIP_TRY(hipMemcpyAsync((void*)d_faults, faults, fb, hipMemcpyHostToDevice, s), "fault upload");
        if (opts->priority) {
            float* dp = (float*)((char*)d_words + eb);
            HIP_TRY(hipMemcpyAsync(dp, opts->priority, pb, hipMemcpyHostToDevice, s), "priority upload");
            d_prio = dp;
        }
    } else {
        if (F == 0) {
            if (cov) HIP_TRY(hipMemsetAsync(cov, 0, sizeof(riros_coverage), s), "coverage clear");
            return RIROS_OK;
        }
        HIP_TRY(hipMemsetAsync(d->d_bad, 0, sizeof(uint32_t), s), "validate clear");
        HIP_TRY(riros::launch_validate_faults(d->dev, faults, F, d->d_bad, s), "validate launch");
        uint32_t bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, d->d_bad, sizeof bad, hipMemcpyDeviceToHost, s), "validate read");
        HIP_TRY(hipStreamSynchronize(s), "validate sync");
        if (bad) return set_err(RIROS_EINVAL, std::to_string(bad) + " invalid faults in device fault list");
        if (!d_words) {
            if (d->ws_words_cap < F) {
                if (d->ws_words) (void)hipFree(d->ws_words);
                d->ws_words = nullptr;
                d->ws_words_cap = 0;
                HIP_TRY(hipMalloc((void**)&d->ws_words, (size_t)F * sizeof(uint64_t)), "words allocation");
                d->ws_words_cap = F;
            }
            d_words = d->ws_words;
        }
    }

    if (opts->mode == RIROS_MODE_PLAIN) {
        if (riros::plain_lds_bytes(d->dev, riros::kWordsNarrow) > 160 * 1024)
            return set_err(RIROS_EINVAL, "design too large for the plain kernel's LDS bitmap");
        int wpc = opts->waves_per_cu > 0 ? opts->waves_per_cu : 16;
        // (this kernel's registers allow about twelve wavefronts a compute
        // unit whatever its LDS, so the wide pass is kept up to that)
        const uint32_t wpp = riros::words_per_pass(d->img.N, d->img.L, d->img.R, (uint32_t)std::min(wpc, 12));
        const size_t lds = riros::plain_lds_bytes(d->dev, wpp);
        const int lds_limit = (int)std::max<size_t>(1, (160 * 1024) / lds);
        wpc = std::min(std::min(wpc, lds_limit), 32);
        uint32_t blocks = (uint32_t)std::min<uint64_t>(F, (uint64_t)d->num_cu * wpc);
        int rc = ensure_plain_ws(d, blocks, s);
        if (rc) return rc;
        const uint64_t per_block = ((uint64_t)F + blocks - 1) / blocks;
        riros::PlainWorkspace ws{d->ws_slots, d->ws_regs, d->stamp_dev};
        HIP_TRY(hipEventRecord(g_ev0, s), "event record");
        HIP_TRY(riros::launch_fault_plain(d->dev, g->view(), d_faults, F, opts->drop ? 1 : 0, blocks, ws, wpp,
                                          d_detect, d_events, d_words, s),
                "plain fault kernel");
        HIP_TRY(hipEventRecord(g_ev1, s), "event record");
        HIP_TRY(riros::launch_advance_stamp(d->stamp_dev, per_block * T + 1, s), "stamp advance");
    } else if (opts->mode == RIROS_MODE_CONCURRENT) {
        std::string err;
        const int rc = riros::run_concurrent(d->dev, d->conc, g->view(), d_faults, F, opts->drop ? 1 : 0,
                                             opts->waves_per_cu, d->num_cu, d_detect, d_events, d_words, g_ev0,
                                             g_ev1, s, err);
        if (rc) return set_err(rc, err);
    } else {
        if (riros::plain_lds_bytes(d->dev, riros::kWordsNarrow) > 160 * 1024)
            return set_err(RIROS_EINVAL, "design too large for the heavy kernel's LDS bitmap");
        // The launches clamp their grids to what is resident at once; the
        // light launch may need no LDS at all, so LDS does not cap this.
        int wpc = opts->waves_per_cu > 0 ? opts->waves_per_cu : 12;
        wpc = std::min(wpc, 32);
        const uint32_t heavy_blocks = (uint32_t)d->num_cu * (uint32_t)wpc;
        int rc = ensure_plain_ws(d, heavy_blocks, s);
        if (rc) return rc;
        riros::PlainWorkspace hws{d->ws_slots, d->ws_regs, d->stamp_dev};
        riros::TwoDParams p;
        p.monitor_rate = opts->monitor_rate;
        p.theta = opts->theta;
        p.light_cap = opts->light_cap;
        p.unified = opts->unified;
        p.share = opts->struct_share;
        p.heavy_wg = opts->heavy_wg > 0 ? opts->heavy_wg : 64;
        p.w32 = im.max_width <= 32 && g->Gn32 != nullptr;   // 32-bit lanes read the 32-bit trace
        p.lockstep = opts->lockstep ? 1 : 0;
        p.deal = (uint32_t)opts->deal;
        p.head_lanes = (uint32_t)opts->head_lanes;
        p.xcd = opts->xcd_queues != 0;
        p.waves_per_cu = wpc;
        p.num_cu = d->num_cu;
        std::string err;
        rc = riros::run_twod(d->dev, d->twod, g->view(), d_faults, d_prio, F, opts->drop ? 1 : 0, p, hws,
                             heavy_blocks, d_detect, d_events, d_words, g_ev0, g_ev1, s, err);
        if (rc) return set_err(rc, err);
    }
    g_ev_valid = true;

    if (!on_dev && opts->mode == RIROS_MODE_TWO_D && d->twod.ctr) {
        std::string err;
        const int rc = riros::twod_check(d->twod, s, err);
        if (rc) return set_err(rc, err);
    }
    riros_coverage* cov_dst = on_dev ? cov : d->d_cov;
    if (cov) HIP_TRY(riros::launch_coverage(d_detect, d_events, d_words, F, T, cov_dst, s), "coverage");
    if (!on_dev) {
        HIP_TRY(hipMemcpyAsync(detect, d_detect, (size_t)F * 4, hipMemcpyDeviceToHost, s), "detect download");
        if (events)
            HIP_TRY(hipMemcpyAsync(events, d_events, (size_t)F * 8, hipMemcpyDeviceToHost, s), "events download");
        if (opts->words)
            HIP_TRY(hipMemcpyAsync(opts->words, d_words, (size_t)F * 8, hipMemcpyDeviceToHost, s),
                    "words download");
        if (cov) HIP_TRY(hipMemcpyAsync(cov, d->d_cov, sizeof(riros_coverage), hipMemcpyDeviceToHost, s),
                         "coverage download");
        HIP_TRY(hipStreamSynchronize(s), "fault simulation sync");
    }
    return RIROS_OK;
}

// ---------------------------------------------------------------------------
// Load predictor
// ---------------------------------------------------------------------------

int riros_features(riros_design d, riros_golden g, const riros_fault* faults, uint32_t F, float* out,
                   int32_t io_on_device, void* stream)
{
    if (!d || !g) return set_err(RIROS_EINVAL, "NULL argument");
    if (g->d != d) return set_err(RIROS_EINVAL, "golden trace belongs to another design");
    if (F > 0 && (!faults || !out)) return set_err(RIROS_EINVAL, "faults or out is NULL");
    DeviceGuard guard(d->device);
    hipStream_t s = (hipStream_t)stream;
    const riros::Image& im = d->img;
    if (!d->d_nodefeat) {
        std::vector<float> nf;
        riros::node_features(im, nf);
        HIP_TRY(hipMalloc((void**)&d->d_nodefeat, (size_t)im.N * sizeof(float4)), "feature allocation");
        HIP_TRY(hipMemcpy(d->d_nodefeat, nf.data(), nf.size() * sizeof(float), hipMemcpyHostToDevice), "feature upload");
    }
    if (F == 0) return RIROS_OK;
    if (io_on_device) {
        HIP_TRY(hipMemsetAsync(d->d_bad, 0, sizeof(uint32_t), s), "validate clear");
        HIP_TRY(riros::launch_validate_faults(d->dev, faults, F, d->d_bad, s), "validate launch");
        uint32_t bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, d->d_bad, sizeof bad, hipMemcpyDeviceToHost, s), "validate read");
        HIP_TRY(hipStreamSynchronize(s), "validate sync");
        if (bad) return set_err(RIROS_EINVAL, std::to_string(bad) + " invalid faults in device fault list");
        HIP_TRY(riros::launch_features(d->dev, g->view(), d->d_nodefeat, faults, F, out, s), "feature kernel");
        return RIROS_OK;
    }
    for (uint32_t i = 0; i < F; ++i) {
        const riros_fault& f = faults[i];
        if (f.site >= im.N || f.stuck > RIROS_FAULT_FLIP || f.bit >= im.desc[im.u2i[f.site]].width)
            return set_err(RIROS_EINVAL, "invalid fault " + std::to_string(i));
    }
    DevBuf<riros_fault> df;
    DevBuf<float> dout;
    HIP_TRY(df.alloc(F), "allocation");
    HIP_TRY(dout.alloc((size_t)F * riros::kMlpFeatures), "allocation");
    HIP_TRY(hipMemcpyAsync(df.p, faults, (size_t)F * sizeof(riros_fault), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(riros::launch_features(d->dev, g->view(), d->d_nodefeat, df.p, F, dout.p, s), "feature kernel");
    HIP_TRY(hipMemcpyAsync(out, dout.p, (size_t)F * riros::kMlpFeatures * sizeof(float), hipMemcpyDeviceToHost, s),
            "download");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return RIROS_OK;
}

int riros_mlp_train(const float* feats, const float* y, uint32_t S, const riros_train_cfg* cfg, float* weights,
                    float* losses, void* stream)
{
    if (!feats || !y || !cfg || !weights) return set_err(RIROS_EINVAL, "NULL argument");
    if (S == 0 || cfg->epochs == 0 || cfg->batch == 0) return set_err(RIROS_EINVAL, "S, epochs and batch must be positive");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t B = std::min(cfg->batch, S);
    const uint32_t steps_per_epoch = (S + B - 1) / B;
    DevBuf<float> dx, dy, dw, dm, dv, dpart, dlp, dloss;
    HIP_TRY(dx.alloc((size_t)S * riros::kMlpFeatures), "allocation");
    HIP_TRY(dy.alloc(S), "allocation");
    HIP_TRY(dw.alloc(riros::kMlpWeights), "allocation");
    HIP_TRY(dm.alloc(riros::kMlpParams), "allocation");
    HIP_TRY(dv.alloc(riros::kMlpParams), "allocation");
    HIP_TRY(dpart.alloc(riros::mlp_partial_floats(B)), "allocation");
    HIP_TRY(dlp.alloc((B + 31) / 32 + 1), "allocation");
    HIP_TRY(dloss.alloc((size_t)cfg->epochs * steps_per_epoch), "allocation");
    HIP_TRY(hipMemcpyAsync(dx.p, feats, (size_t)S * riros::kMlpFeatures * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(hipMemcpyAsync(dy.p, y, (size_t)S * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(hipMemcpyAsync(dw.p, weights, riros::kMlpParams * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(hipMemsetAsync(dm.p, 0, riros::kMlpParams * sizeof(float), s), "clear");
    HIP_TRY(hipMemsetAsync(dv.p, 0, riros::kMlpParams * sizeof(float), s), "clear");
    HIP_TRY(riros::mlp_norm_stats(dx.p, S, dw.p, s), "normalisation");
    const riros::MlpHyper h{cfg->lr, cfg->beta1, cfg->beta2, cfg->eps};
    uint32_t step = 0;
    for (uint32_t e = 0; e < cfg->epochs; ++e)
        for (uint32_t b0 = 0; b0 < S; b0 += B) {
            const uint32_t nb = std::min(B, S - b0);
            HIP_TRY(riros::mlp_step(dw.p, dx.p + (size_t)b0 * riros::kMlpFeatures, dy.p + b0, nb, dpart.p, dlp.p, dm.p,
                                    dv.p, nullptr, dloss.p + step, step + 1, h, s),
                    "training step");
            ++step;
        }
    HIP_TRY(hipMemcpyAsync(weights, dw.p, riros::kMlpWeights * sizeof(float), hipMemcpyDeviceToHost, s), "download");
    if (losses)
        HIP_TRY(hipMemcpyAsync(losses, dloss.p, (size_t)step * sizeof(float), hipMemcpyDeviceToHost, s), "download");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return RIROS_OK;
}

int riros_mlp_predict(const float* weights, const float* feats, uint32_t F, float* out, int32_t io_on_device,
                      void* stream)
{
    if (!weights || (F > 0 && (!feats || !out))) return set_err(RIROS_EINVAL, "NULL argument");
    if (F == 0) return RIROS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (io_on_device) {
        HIP_TRY(riros::mlp_forward(weights, feats, F, out, s), "inference");
        return RIROS_OK;
    }
    DevBuf<float> dw, dx, dout;
    HIP_TRY(dw.alloc(riros::kMlpWeights), "allocation");
    HIP_TRY(dx.alloc((size_t)F * riros::kMlpFeatures), "allocation");
    HIP_TRY(dout.alloc(F), "allocation");
    HIP_TRY(hipMemcpyAsync(dw.p, weights, riros::kMlpWeights * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(hipMemcpyAsync(dx.p, feats, (size_t)F * riros::kMlpFeatures * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(riros::mlp_forward(dw.p, dx.p, F, dout.p, s), "inference");
    HIP_TRY(hipMemcpyAsync(out, dout.p, (size_t)F * sizeof(float), hipMemcpyDeviceToHost, s), "download");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return RIROS_OK;
}

int riros_mlp_grad(const float* weights, const float* feats, const float* y, uint32_t B, float* grad, float* loss,
                   void* stream)
{
    if (!weights || !feats || !y || !grad || !loss) return set_err(RIROS_EINVAL, "NULL argument");
    if (B == 0) return set_err(RIROS_EINVAL, "empty batch");
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> dw, dx, dy, dpart, dlp, dg, dl;
    HIP_TRY(dw.alloc(riros::kMlpWeights), "allocation");
    HIP_TRY(dx.alloc((size_t)B * riros::kMlpFeatures), "allocation");
    HIP_TRY(dy.alloc(B), "allocation");
    HIP_TRY(dpart.alloc(riros::mlp_partial_floats(B)), "allocation");
    HIP_TRY(dlp.alloc((B + 31) / 32 + 1), "allocation");
    HIP_TRY(dg.alloc(riros::kMlpParams), "allocation");
    HIP_TRY(dl.alloc(1), "allocation");
    HIP_TRY(hipMemcpyAsync(dw.p, weights, riros::kMlpWeights * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(hipMemcpyAsync(dx.p, feats, (size_t)B * riros::kMlpFeatures * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    HIP_TRY(hipMemcpyAsync(dy.p, y, (size_t)B * sizeof(float), hipMemcpyHostToDevice, s), "upload");
    const riros::MlpHyper h{0.f, 0.f, 0.f, 0.f};
    HIP_TRY(riros::mlp_step(dw.p, dx.p, dy.p, B, dpart.p, dlp.p, nullptr, nullptr, dg.p, dl.p, 1, h, s), "gradient");
    HIP_TRY(hipMemcpyAsync(grad, dg.p, riros::kMlpParams * sizeof(float), hipMemcpyDeviceToHost, s), "download");
    HIP_TRY(hipMemcpyAsync(loss, dl.p, sizeof(float), hipMemcpyDeviceToHost, s), "download");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return RIROS_OK;
}

// ---------------------------------------------------------------------------
// Batched campaigns
// ---------------------------------------------------------------------------

}  // extern "C"

struct riros_batch_s {
    int device = 0;
    uint32_t n = 0, F = 0;
    std::vector<uint32_t> off;        // host copy of the fault offsets
    riros::BatchPlan plan{};
    riros::TwoDWorkspace tw{};
    std::vector<void*> owned;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last_stream = nullptr;
};

static void free_batch(riros_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (void* p : b->owned) (void)hipFree(p);
    riros::twod_free(b->tw);
}

template <class T>
static hipError_t batch_alloc(riros_batch b, T** p, size_t n)
{
    hipError_t e = hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) b->owned.push_back((void*)*p);
    return e;
}

extern "C" {

int riros_batch_create(uint32_t n, const riros_design* designs, const riros_golden* goldens,
                       const riros_fault* const* faults, const uint32_t* F, const float* const* priority,
                       const riros_sim_opts* opts, riros_batch* out)
{
    if (!designs || !goldens || !faults || !F || !opts || !out) return set_err(RIROS_EINVAL, "NULL argument");
    if (n == 0 || n > 65536) return set_err(RIROS_EINVAL, "n must be in 1..65536");
    if (opts->mode != RIROS_MODE_TWO_D || opts->io_on_device)
        return set_err(RIROS_EINVAL, "campaigns run in RIROS_MODE_TWO_D with host-side inputs");
    if (opts->waves_per_cu < 0 || (opts->unified != 0 && opts->unified != 1) || !(opts->monitor_rate >= 0.f) ||
        (opts->light_cap != 0 && opts->light_cap != 4 && opts->light_cap != 8 && opts->light_cap != 16) ||
        !valid_share(opts->struct_share) || !valid_heavy_wg(opts->heavy_wg) || !valid_deal(opts->deal) ||
        !valid_head_lanes(opts->head_lanes) ||
        (opts->xcd_queues != 0 && opts->xcd_queues != 1) || (opts->lockstep != 0 && opts->lockstep != 1))
        return set_err(RIROS_EINVAL, "invalid option");
    const int dev = designs[0] ? designs[0]->device : 0;
    uint64_t total = 0;
    uint32_t Nmax = 0, Lmax = 0, Rmax = 0, Tmax = 0, Wmax = 0;
    bool all_gn32 = true;
    for (uint32_t i = 0; i < n; ++i) {
        if (!designs[i] || !goldens[i] || goldens[i]->d != designs[i])
            return set_err(RIROS_EINVAL, "design " + std::to_string(i) + ": missing or mismatched golden trace");
        if (designs[i]->device != dev) return set_err(RIROS_EINVAL, "designs on different devices");
        if (F[i] > 0 && !faults[i]) return set_err(RIROS_EINVAL, "faults[" + std::to_string(i) + "] is NULL");
        const riros::Image& im = designs[i]->img;
        for (uint32_t j = 0; j < F[i]; ++j) {
            const riros_fault& f = faults[i][j];
            if (f.site >= im.N || f.stuck > RIROS_FAULT_FLIP || f.bit >= im.desc[im.u2i[f.site]].width)
                return set_err(RIROS_EINVAL, "design " + std::to_string(i) + " fault " + std::to_string(j) + " invalid");
        }
        total += F[i];
        Nmax = std::max(Nmax, im.N);
        Lmax = std::max(Lmax, im.L);
        Rmax = std::max(Rmax, im.R);
        Tmax = std::max(Tmax, goldens[i]->T);
        Wmax = std::max(Wmax, im.max_width);
        all_gn32 = all_gn32 && goldens[i]->Gn32 != nullptr;
    }
    if (total >= 0xFFFFFFFFull) return set_err(RIROS_EINVAL, "too many faults");
    const size_t lds = riros::wave_lds_words(Nmax, Lmax, Rmax, riros::kWordsNarrow) * sizeof(uint32_t);
    if (lds > 160 * 1024) return set_err(RIROS_EINVAL, "largest design too large for the structural path's LDS bitmap");
    DeviceGuard guard(dev);
    riros_batch b = new (std::nothrow) riros_batch_s();
    if (!b) return set_err(RIROS_ENOMEM, "host allocation failed");
    b->device = dev;
    b->n = n;
    b->F = (uint32_t)total;
    auto fail = [&](int code, const std::string& m) {
        free_batch(b);
        delete b;
        return set_err(code, m);
    };
    // Host staging: tables, concatenated faults, design ids, offsets, priorities.
    std::vector<riros::DevDesign> td(n);
    std::vector<riros::GoldenView> tg(n);
    std::vector<riros_fault> fl(b->F);
    std::vector<uint16_t> did(b->F);
    std::vector<float> pr;
    const bool any_prio = priority != nullptr;
    if (any_prio) pr.assign(b->F, 0.f);
    b->off.assign(n + 1, 0);
    for (uint32_t i = 0; i < n; ++i) {
        td[i] = designs[i]->dev;
        tg[i] = goldens[i]->view();
        const uint32_t o = b->off[i];
        if (F[i]) std::memcpy(&fl[o], faults[i], (size_t)F[i] * sizeof(riros_fault));
        for (uint32_t j = 0; j < F[i]; ++j) did[o + j] = (uint16_t)i;
        if (any_prio && priority[i]) std::memcpy(&pr[o], priority[i], (size_t)F[i] * sizeof(float));
        b->off[i + 1] = o + F[i];
    }
    riros::BatchPlan& p = b->plan;
    riros::DevDesign* d_td = nullptr;
    riros::GoldenView* d_tg = nullptr;
    riros_fault* d_fl = nullptr;
    uint16_t* d_did = nullptr;
    uint32_t* d_off = nullptr;
    float* d_pr = nullptr;
    uint32_t* d_det = nullptr;
    uint64_t* d_ev = nullptr;
    uint64_t* d_wk = nullptr;
    riros_coverage* d_cov = nullptr;
    riros::GoldenJob* d_jobs = nullptr;
    riros::Slot* d_slots = nullptr;
    uint64_t* d_regs = nullptr;
    uint64_t* d_stamp = nullptr;
    // Grids are clamped to what is resident at once when the graph is built.
    const int wpc = std::min(opts->waves_per_cu > 0 ? opts->waves_per_cu : 12, 32);
    const uint32_t blocks = (uint32_t)designs[0]->num_cu * (uint32_t)wpc;
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    A(batch_alloc(b, &d_td, n));
    A(batch_alloc(b, &d_tg, n));
    A(batch_alloc(b, &d_fl, b->F));
    A(batch_alloc(b, &d_did, b->F));
    A(batch_alloc(b, &d_off, n + 1));
    if (any_prio) A(batch_alloc(b, &d_pr, b->F));
    A(batch_alloc(b, &d_det, b->F));
    A(batch_alloc(b, &d_ev, b->F));
    A(batch_alloc(b, &d_wk, b->F));
    A(batch_alloc(b, &d_cov, n));
    if (opts->campaign_golden) A(batch_alloc(b, &d_jobs, n));
    A(batch_alloc(b, &d_slots, (size_t)blocks * Nmax));
    A(batch_alloc(b, &d_regs, (size_t)blocks * 2 * std::max(Rmax, 1u)));
    A(batch_alloc(b, &d_stamp, 1));
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? RIROS_ENOMEM : RIROS_EDEVICE, "campaign allocation");
    A(hipMemcpy(d_td, td.data(), n * sizeof(riros::DevDesign), hipMemcpyHostToDevice));
    A(hipMemcpy(d_tg, tg.data(), n * sizeof(riros::GoldenView), hipMemcpyHostToDevice));
    // Golden machines in the graph: designs in fewer than two parts one
    // workgroup each (one launch, all of them at once), the parts of the
    // others one workgroup each (a second launch).
    uint32_t n_jobs = 0, n_pjobs = 0, pmax = 0;
    riros::GPartJob* d_pjobs = nullptr;
    if (d_jobs) {
        std::vector<riros::GoldenJob> jobs;
        std::vector<riros::GPartJob> pjobs;
        for (uint32_t i = 0; i < n; ++i) {
            if (designs[i]->gparts.P < 2)
                jobs.push_back(riros::GoldenJob{goldens[i]->stim, goldens[i]->G, goldens[i]->T, i});
            else
                append_part_jobs(designs[i], goldens[i]->stim, goldens[i]->T, goldens[i]->G, pjobs, pmax);
        }
        n_jobs = (uint32_t)jobs.size();
        n_pjobs = (uint32_t)pjobs.size();
        if (n_jobs) A(hipMemcpy(d_jobs, jobs.data(), n_jobs * sizeof(riros::GoldenJob), hipMemcpyHostToDevice));
        if (n_pjobs) {
            A(batch_alloc(b, &d_pjobs, n_pjobs));
            A(hipMemcpy(d_pjobs, pjobs.data(), n_pjobs * sizeof(riros::GPartJob), hipMemcpyHostToDevice));
        }
    }
    if (b->F) {
        A(hipMemcpy(d_fl, fl.data(), fl.size() * sizeof(riros_fault), hipMemcpyHostToDevice));
        A(hipMemcpy(d_did, did.data(), did.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        if (any_prio) A(hipMemcpy(d_pr, pr.data(), pr.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    A(hipMemcpy(d_off, b->off.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice));
    A(hipMemset(d_slots, 0, (size_t)blocks * Nmax * sizeof(riros::Slot)));
    A(hipMemset(d_stamp, 0, sizeof(uint64_t)));
    A(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    if (e != hipSuccess) return fail(RIROS_EDEVICE, std::string("campaign upload: ") + hipGetErrorString(e));
    p.n = n;
    p.F = b->F;
    p.td = d_td;
    p.tg = d_tg;
    p.did = d_did;
    p.off = d_off;
    p.Nmax = Nmax;
    p.Lmax = Lmax;
    p.Rmax = Rmax;
    p.faults = d_fl;
    p.drop = opts->drop ? 1 : 0;
    p.light_cap = opts->light_cap ? opts->light_cap : 8;
    p.rate_num = opts->monitor_rate > 0.f ? (uint32_t)std::min(4.0e9f, opts->monitor_rate * 4.f + 0.5f) : 0u;
    p.blocks = blocks;
    p.span = (uint64_t)b->F * Tmax + 1;
    p.ws = riros::PlainWorkspace{d_slots, d_regs, d_stamp};
    p.detect = d_det;
    p.events = d_ev;
    p.words = d_wk;
    p.cov = d_cov;
    std::string err;
    int rc = riros::order_batch(b->tw, d_pr, d_fl, b->F, opts->theta, opts->xcd_queues ? 1 : 0, &p.order,
                                b->cap_stream, err);
    if (rc) return fail(rc, err);
    p.heavy = d_pr != nullptr && !(opts->theta > 3.0e38f);
    p.unified = opts->unified;
    p.share = opts->struct_share;
    p.heavy_wg = opts->heavy_wg > 0 ? (uint32_t)opts->heavy_wg : 64u;
    p.w32 = Wmax <= 32 && all_gn32;   // 32-bit lanes read every design's 32-bit trace
    p.lockstep = opts->lockstep ? 1 : 0;
    p.deal = (uint32_t)opts->deal;
    p.head_lanes = (uint32_t)opts->head_lanes;
    p.xcd = opts->xcd_queues != 0;
    p.wpp = riros::words_per_pass(Nmax, Lmax, Rmax, (uint32_t)wpc);
    e = hipStreamSynchronize(b->cap_stream);
    if (e == hipSuccess) e = riros::prepare_twod_batch(p);
    if (e != hipSuccess) return fail(RIROS_EDEVICE, std::string("campaign preparation: ") + hipGetErrorString(e));
    // Capture the run as a graph.
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        if (d_jobs) {
            // The golden machines of all designs (one workgroup for each
            // design without parts, one launch by parts for each of the
            // others), then each trace's other layouts, then the fault
            // simulation.
            le = riros::launch_golden_many(n_jobs, d_td, d_jobs, b->cap_stream);
            if (le == hipSuccess) le = riros::launch_golden_parts_many(n_pjobs, d_pjobs, pmax, b->cap_stream);
            for (uint32_t i = 0; i < n && le == hipSuccess; ++i)
                le = riros::launch_golden_layouts(designs[i]->dev, goldens[i]->G, goldens[i]->T, goldens[i]->Gn,
                                                  goldens[i]->Bp, goldens[i]->Gn32, b->cap_stream);
        }
        if (le == hipSuccess) le = riros::launch_twod_batch(p, b->tw, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(RIROS_EDEVICE, std::string("campaign graph capture: ") + hipGetErrorString(e));
    *out = b;
    return RIROS_OK;
}

int riros_batch_launch(riros_batch b, void* stream)
{
    if (!b) return set_err(RIROS_EINVAL, "NULL campaign");
    DeviceGuard guard(b->device);
    hipStream_t s = (hipStream_t)stream;
    if (!g_ev0) {
        HIP_TRY(hipEventCreate(&g_ev0), "event create");
        HIP_TRY(hipEventCreate(&g_ev1), "event create");
    }
    HIP_TRY(hipEventRecord(g_ev0, s), "event record");
    HIP_TRY(hipGraphLaunch(b->exec, s), "campaign graph launch");
    HIP_TRY(hipEventRecord(g_ev1, s), "event record");
    g_ev_valid = true;
    b->last_stream = s;
    return RIROS_OK;
}

int riros_batch_read(riros_batch b, uint32_t i, uint32_t* detect, uint64_t* events, uint64_t* words,
                     riros_coverage* cov)
{
    if (!b) return set_err(RIROS_EINVAL, "NULL campaign");
    if (i >= b->n) return set_err(RIROS_EINVAL, "design index out of range");
    const uint32_t o = b->off[i], cnt = b->off[i + 1] - b->off[i];
    if (cnt > 0 && !detect) return set_err(RIROS_EINVAL, "detect is NULL");
    DeviceGuard guard(b->device);
    HIP_TRY(hipStreamSynchronize(b->last_stream), "campaign sync");
    if (cnt) {
        HIP_TRY(hipMemcpy(detect, b->plan.detect + o, (size_t)cnt * 4, hipMemcpyDeviceToHost), "detect download");
        if (events)
            HIP_TRY(hipMemcpy(events, b->plan.events + o, (size_t)cnt * 8, hipMemcpyDeviceToHost), "events download");
        if (words)
            HIP_TRY(hipMemcpy(words, b->plan.words + o, (size_t)cnt * 8, hipMemcpyDeviceToHost), "words download");
    }
    if (cov) HIP_TRY(hipMemcpy(cov, b->plan.cov + i, sizeof(riros_coverage), hipMemcpyDeviceToHost), "coverage download");
    return RIROS_OK;
}

void riros_batch_free(riros_batch b)
{
    if (!b) return;
    DeviceGuard guard(b->device);
    (void)hipDeviceSynchronize();
    free_batch(b);
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free plain fault simulation.  Its per-call workspace (each
// wavefront's faulty-value slots and register ping-pong) lives in `scratch`,
// a static device array of RIROS_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends.  In host code `scratch` is a
// stand-in, not a device address: the array's address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever handed to a kernel.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[RIROS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on `dev` (which must be current).
int scratch_on(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_err(RIROS_EDEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_err(e == hipSuccess ? hipErrorInvalidSymbol : e, "scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return RIROS_OK;
}

}  // namespace

extern "C" {

int riros_fault_sim_noalloc(riros_design d, riros_golden g, const riros_fault* faults, uint32_t F,
                            const riros_sim_opts* opts, uint32_t* detect, uint64_t* events, riros_coverage* cov)
{
    if (!d || !g || !opts) return set_err(RIROS_EINVAL, "NULL argument");
    if (g->d != d) return set_err(RIROS_EINVAL, "golden trace belongs to another design");
    if (opts->mode != RIROS_MODE_PLAIN) return set_err(RIROS_EINVAL, "riros_fault_sim_noalloc runs RIROS_MODE_PLAIN only");
    if (!opts->io_on_device)
        return set_err(RIROS_EINVAL, "riros_fault_sim_noalloc takes device-resident inputs and outputs (io_on_device = 1)");
    if (F > 0 && (!faults || !detect)) return set_err(RIROS_EINVAL, "faults or detect is NULL");
    if (opts->waves_per_cu < 0) return set_err(RIROS_EINVAL, "waves_per_cu < 0");
    const riros::Image& im = d->img;
    // One wavefront's workspace: N slots and 2R register words.
    const size_t slot_bytes = (size_t)im.N * sizeof(riros::Slot);
    const size_t reg_bytes = (size_t)2 * std::max(im.R, 1u) * sizeof(uint64_t);
    const size_t per_wave = slot_bytes + reg_bytes;
    if (per_wave > RIROS_NOALLOC_SCRATCH_BYTES) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "design needs %zu bytes of workspace per wavefront; the no-allocation scratch holds %zu",
                      per_wave, (size_t)RIROS_NOALLOC_SCRATCH_BYTES);
        return set_err(RIROS_EINVAL, buf);
    }
    if (riros::plain_lds_bytes(d->dev, riros::kWordsNarrow) > 160 * 1024)
        return set_err(RIROS_EINVAL, "design too large for the plain kernel's LDS bitmap");
    DeviceGuard guard(d->device);
    hipStream_t s = (hipStream_t)opts->stream;
    const uint32_t T = g->T;
    unsigned char* base = nullptr;
    int rc = scratch_on(d->device, &base);
    if (rc) return rc;
    if (F == 0) {
        if (cov) HIP_TRY(riros::launch_coverage(nullptr, nullptr, nullptr, 0, T, cov, s), "coverage");
        return RIROS_OK;
    }
    // Faults: validated on the device (the count of bad ones comes back to
    // the host once); the counter is cleared by a kernel.
    HIP_TRY(riros::launch_fill_u32(d->d_bad, 1, 0u, s), "validate clear");
    HIP_TRY(riros::launch_validate_faults(d->dev, faults, F, d->d_bad, s), "validate launch");
    uint32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, d->d_bad, sizeof bad, hipMemcpyDeviceToHost, s), "validate read");
    HIP_TRY(hipStreamSynchronize(s), "validate sync");
    if (bad) return set_err(RIROS_EINVAL, std::to_string(bad) + " invalid faults in device fault list");
    // Grid: as riros_fault_sim's plain mode, cut to the wavefronts whose
    // workspace fits the scratch array.
    int wpc = opts->waves_per_cu > 0 ? opts->waves_per_cu : 16;
    const uint32_t wpp = riros::words_per_pass(im.N, im.L, im.R, (uint32_t)std::min(wpc, 12));
    const size_t lds = riros::plain_lds_bytes(d->dev, wpp);
    const int lds_limit = (int)std::max<size_t>(1, (160 * 1024) / lds);
    wpc = std::min(std::min(wpc, lds_limit), 32);
    const uint64_t fit = (uint64_t)(RIROS_NOALLOC_SCRATCH_BYTES - 256) / per_wave;
    const uint32_t blocks =
        (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(std::min<uint64_t>(F, (uint64_t)d->num_cu * wpc), fit));
    riros::Slot* slots = (riros::Slot*)base;
    const size_t reg_off = ((size_t)blocks * slot_bytes + 255) & ~(size_t)255;
    uint64_t* regs = (uint64_t*)(base + reg_off);
    // Slots left by an earlier call (of any design) must not carry a valid
    // stamp: clear the ones this call uses.
    HIP_TRY(riros::launch_fill_u32((uint32_t*)slots, (size_t)blocks * slot_bytes / 4, 0u, s), "scratch clear");
    const uint64_t per_block = ((uint64_t)F + blocks - 1) / blocks;
    riros::PlainWorkspace ws{slots, regs, d->stamp_dev};
    HIP_TRY(riros::launch_fault_plain(d->dev, g->view(), faults, F, opts->drop ? 1 : 0, blocks, ws, wpp, detect,
                                      events, opts->words, s),
            "plain fault kernel");
    HIP_TRY(riros::launch_advance_stamp(d->stamp_dev, per_block * T + 1, s), "stamp advance");
    if (cov) HIP_TRY(riros::launch_coverage(detect, events, opts->words, F, T, cov, s), "coverage");
    return RIROS_OK;
}

}  // extern "C"
