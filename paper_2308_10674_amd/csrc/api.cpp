// C ABI of libptyc: context, ingest, schedule and sweep orchestration.
// Declarations and the contract of every call are in include/ptyc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ptyc.h"
#include "kernels.h"
#include "schedule.h"

using namespace ptyc;

// Work memory of ptyc_sweep_noalloc (the spectrum exchange, the partial
// maxima of the windows, the error partials and sums, the device copy of a
// sweep's order): a file-scope device array, so that entry point allocates
// nothing.  Every GPU the library runs on holds its own copy until the
// process ends.  Host code never hands the array's name to a kernel (on the
// host it only names a stand-in); its device address on each device is
// taken once with hipGetSymbolAddress (noalloc_setup, from ptyc_init) and
// that pointer is used instead.
constexpr size_t kNoallocBytes = PTYC_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

thread_local std::string g_init_error;

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// the device address of `scratch` on `device` (current), taken once
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[device] = p;
    return hipSuccess;
}

void* noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

// the default way a multi-context call runs (the stepped launches with the
// eight-slot inverse tile for scans whose batches hold at most 16
// positions; the fastest on the sixteen-scan workload, see kMultiVariants)
constexpr int kMultiDefault = 6;

struct ptyc_ctx {
    ptyc_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool poisoned = false;
    std::string err;
    int form = kFormBatch;          // launch form of a sweep
    int capacity = 0;               // co-resident workgroups of the persistent kernel
    int capacity_multi = 0;         // co-resident workgroups of the multi-scan persistent kernel (0: not yet asked)
    Shape sb{}, sp{}, sm{};         // work split of the per-batch (default tile), persistent and mixed-size launches
    int tile = 0;                   // tile variant of the per-batch kernels (batch and graph forms)
    Shape st{};                     // work split of that variant
    int col_blocks_max = 0;         // over every form and variant (error partials per position)

    // device state
    DevBuf obj, probe, tw;
    DevBuf sqrt_i, pos, sum_i;       // per position, capacity cap
    int64_t cap = 0, n_loaded = 0;
    DevBuf scratch, winmax;          // per batch slot, capacity slots
    int64_t slots = 0;
    DevBuf pmax_part;                // two halves of max_probe_blocks floats (see pmax_cur)
    int pmax_cur = 0;                // the half holding the current probe's partial maxima
    DevBuf order;                    // OrderEntry [order_cap]
    DevBuf offs;                     // int64 batch offsets of the persistent form
    DevBuf err_part, err_dev;
    DevBuf bad;                      // int flag for ingest validation
    DevBuf sync;                     // [0] barrier counter, [1] barrier fault flag
    DevBuf multi;                    // batch descriptors of a multi-context call
    DevBuf mbar;                     // arrival counters of the multi-scan persistent kernel (first context of a call)
    int multi_variant = kMultiDefault; // how a multi-context call led by this context launches (kMultiVariants)
    unsigned spin_limit = kSpinLimitDefault; // bound of a persistent kernel's barrier wait (PTYC_SPIN_LIMIT at init)
    hipGraphExec_t mgexec = nullptr; // multi-scan persistent launch captured as a graph (graph form)
    const void* mg_tab = nullptr;    // the descriptor table, count, grid and barrier counters the captured graph was built for
    int mg_count = 0, mg_grid = 0;
    const void* mg_bars = nullptr;
    int mg_nbars = 0;
    DevBuf mask;                     // uint8 [n][n] measured detector pixels (stored layout), if set
    ptyc_ingest ingest{};            // how raw frames become stored amplitudes
    DevBuf staging;                  // host intensities staged on the device
    DevBuf gpart;                    // amplitude-loss adjoint: partial sums of dL/dP

    // host state
    std::vector<int32_t> h_pos;      // 2 per position
    Colouring* colouring = nullptr;
    int64_t sweeps_done = 0;
    int64_t* pinned_order = nullptr; // pinned upload buffer (order entries, then offsets)
    size_t pinned_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    // pinned upload buffers of the amplitude loss, used in turn: the host
    // prepares a minibatch while the uploads of the previous ones are still
    // queued (it waits only for the upload made kLossRing calls earlier)
    struct PinSlot {
        void* p = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    };
    static constexpr int kLossRing = 4;
    PinSlot lpin[kLossRing];
    int lring = 0;

    size_t dev_bytes = 0, dev_limit = 0;

    // launch form "graph": one instantiated sweep graph, rebuilt when the
    // batch count, the largest batch or a buffer address changes; each sweep
    // copies its order and offsets into gorder / goffs first
    hipGraphExec_t gexec = nullptr;
    BatchArgs gkey{};
    int64_t g_nb = -1, g_maxb = -1;
    int g_tile = -1;
    DevBuf gorder, goffs;
    DevBuf tune_save;                // object and probe saved while ptyc_tune times the variants

    // optional per-kernel timing with events on the context's stream
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;      // created on demand, reused
    size_t ev_used = 0;
    struct Mark { int kind; size_t e0, e1; int64_t units; };
    std::vector<Mark> marks;               // pending intervals
    double prof_ms[PTYC_KERNEL_KINDS] = {};
    int64_t prof_launches[PTYC_KERNEL_KINDS] = {};
    int64_t prof_units[PTYC_KERNEL_KINDS] = {};
};

namespace {

int fail(ptyc_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(ptyc_ctx* c, hipError_t e, const char* what) {
    c->poisoned = true;
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return PTYC_ERR_HIP;
}

#define HIPCHK(c, expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
    } while (0)

// PTYC_SPIN_LIMIT: polls a software-barrier wait of the persistent kernels
// may take before it raises the fault flag (default kSpinLimitDefault; a
// small value forces the failure path in tests)
unsigned env_spin_limit() {
    const char* s = std::getenv("PTYC_SPIN_LIMIT");
    if (!s || !*s) return kSpinLimitDefault;
    return (unsigned)std::strtoul(s, nullptr, 10);
}

size_t env_limit() {
    const char* s = std::getenv("PTYC_MAX_DEVICE_BYTES");
    if (!s || !*s) return 0;
    return (size_t)std::strtoull(s, nullptr, 10);
}

// (re)allocate a device buffer to at least `bytes`, keeping `keep` bytes of content
int ensure(ptyc_ctx* c, DevBuf& b, size_t bytes, size_t keep = 0) {
    if (b.bytes >= bytes) return PTYC_OK;
    size_t want = std::max(bytes, b.bytes + b.bytes / 2);
    if (c->dev_limit && c->dev_bytes - b.bytes + want > c->dev_limit) {
        want = bytes;
        if (c->dev_bytes - b.bytes + want > c->dev_limit)
            return fail(c, PTYC_ERR_OOM, "device memory cap (PTYC_MAX_DEVICE_BYTES) exceeded");
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, PTYC_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    if (b.p) {
        if (keep) {
            e = hipMemcpyAsync(p, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync(grow)");
        }
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize(grow)");
        (void)hipFree(b.p);
        c->dev_bytes -= b.bytes;
    }
    b.p = p;
    b.bytes = want;
    c->dev_bytes += want;
    return PTYC_OK;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

bool valid_kind(int k) { return k == PTYC_MEM_HOST || k == PTYC_MEM_DEVICE; }

hipMemcpyKind to_dev(int k) { return k == PTYC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice; }
hipMemcpyKind from_dev(int k) { return k == PTYC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice; }

int validate_config(const ptyc_config* cfg, std::string* why) {
    if (!cfg) { *why = "cfg is NULL"; return PTYC_ERR_ARG; }
    if (!supported_n(cfg->n)) { *why = "n must be a power of two in [16, 256]"; return PTYC_ERR_ARG; }
    if (cfg->h < cfg->n || cfg->w < cfg->n) { *why = "object must be at least n x n"; return PTYC_ERR_ARG; }
    if (cfg->h > 65536 || cfg->w > 65536) { *why = "object sides must be <= 65536"; return PTYC_ERR_ARG; }
    if (cfg->mode != PTYC_MODE_STRICT && cfg->mode != PTYC_MODE_COLOURED) { *why = "unknown mode"; return PTYC_ERR_ARG; }
    if (cfg->max_batch < 0) { *why = "max_batch must be >= 0"; return PTYC_ERR_ARG; }
    if (!std::isfinite(cfg->alpha) || !std::isfinite(cfg->beta)) { *why = "alpha and beta must be finite"; return PTYC_ERR_ARG; }
    if (cfg->flags & ~(PTYC_I_IS_SQRT | PTYC_I_CENTERED)) { *why = "unknown flag bits"; return PTYC_ERR_ARG; }
    if (cfg->reserved != 0) { *why = "reserved must be 0"; return PTYC_ERR_ARG; }
    return PTYC_OK;
}

int usable(ptyc_ctx* c) {
    if (!c) return PTYC_ERR_ARG;
    if (c->poisoned) return PTYC_ERR_STATE;
    return PTYC_OK;
}

int32_t max_batch_of(const ptyc_ctx* c) { return c->cfg.max_batch > 0 ? c->cfg.max_batch : 1024; }

// the schedule the library uses for sweep number `sweep`
void default_schedule(const ptyc_ctx* c, int64_t sweep, std::vector<int64_t>& order,
                      std::vector<int64_t>& off) {
    order.clear();
    off.clear();
    off.push_back(0);
    if (c->cfg.mode == PTYC_MODE_STRICT) {
        order = shuffled(c->n_loaded, c->cfg.seed, (uint64_t)sweep);
        for (int64_t i = 1; i <= c->n_loaded; ++i) off.push_back(i);
        return;
    }
    const auto& mem = c->colouring->members();
    std::vector<int64_t> perm = shuffled((int64_t)mem.size(), c->cfg.seed, (uint64_t)sweep);
    order.reserve((size_t)c->n_loaded);
    for (int64_t b : perm) {
        const auto& m = mem[(size_t)b];
        order.insert(order.end(), m.begin(), m.end());
        off.push_back((int64_t)order.size());
    }
}

const Shape& shape_of(const ptyc_ctx* c) { return c->form == kFormPersistent ? c->sp : c->st; }
int max_row_blocks(const ptyc_ctx* c) { return std::max(c->sb.row_blocks, c->sp.row_blocks); }
int max_col_blocks(const ptyc_ctx* c) { return c->col_blocks_max; }
int max_probe_blocks(const ptyc_ctx* c) { return std::max(c->sb.probe_blocks, c->sp.probe_blocks); }

float* pmax_half(const ptyc_ctx* c, int k) { return (float*)c->pmax_part.p + (size_t)k * max_probe_blocks(c); }

BatchArgs base_args(ptyc_ctx* c) {
    BatchArgs a{};
    a.obj = (cf*)c->obj.p;
    a.h = c->cfg.h;
    a.w = c->cfg.w;
    a.probe = (cf*)c->probe.p;
    a.tw = (const cf*)c->tw.p;
    a.sqrt_i = (const float*)c->sqrt_i.p;
    a.pos = (const int2*)c->pos.p;
    a.order = (const OrderEntry*)c->order.p;
    a.scratch = (cf*)c->scratch.p;
    a.winmax = (float*)c->winmax.p;
    a.pmax_in = pmax_half(c, c->pmax_cur);
    a.pmax_out = pmax_half(c, c->pmax_cur ^ 1);
    a.err_part = (double*)c->err_part.p;
    a.alpha = c->cfg.alpha;
    a.beta = c->cfg.beta;
    a.n = c->cfg.n;
    a.mask = (const unsigned char*)c->mask.p;
    return a;
}

IngestSpec ingest_spec(const ptyc_ctx* c) {
    IngestSpec sp{};
    sp.frame_h = c->ingest.frame_h;
    sp.frame_w = c->ingest.frame_w;
    sp.crop_y = c->ingest.crop_y;
    sp.crop_x = c->ingest.crop_x;
    sp.orient = c->ingest.orient;
    sp.centred = (c->ingest.flags & PTYC_I_CENTERED) != 0;
    sp.is_sqrt = (c->ingest.flags & PTYC_I_IS_SQRT) != 0;
    sp.scale = c->ingest.scale;
    sp.mask = (const unsigned char*)c->mask.p;
    return sp;
}

// stored-layout pixel (a, b) of crop pixel (r, c), as the ingest kernel maps it
void ingest_map(const ptyc_ingest& g, int n, int r, int cc, int* a, int* b) {
    int y = r, x = cc;
    if (g.orient & 1) std::swap(y, x);
    if (g.orient & 2) y = n - 1 - y;
    if (g.orient & 4) x = n - 1 - x;
    if (g.flags & PTYC_I_CENTERED) {
        y = (y + n / 2) % n;
        x = (x + n / 2) % n;
    }
    *a = y;
    *b = x;
}

int copy_square_in(ptyc_ctx* c, DevBuf& dst, const void* src, size_t bytes, int kind) {
    HIPCHK(c, hipMemcpyAsync(dst.p, src, bytes, to_dev(kind), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PTYC_OK;
}

int refresh_probe_max(ptyc_ctx* c) {
    BatchArgs a = base_args(c);
    a.bsize = 0;
    HIPCHK(c, launch_probe_reduce(c->cfg.n, a, c->form, c->stream));
    c->pmax_cur ^= 1;
    return PTYC_OK;
}

// next n events of the profiling pool (created as needed)
int take_events(ptyc_ctx* c, size_t n, size_t* first) {
    while (c->ev_pool.size() < c->ev_used + n) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    *first = c->ev_used;
    c->ev_used += n;
    return PTYC_OK;
}

// fold the pending intervals into the totals (synchronises the stream)
int collect_profile(ptyc_ctx* c) {
    if (c->marks.empty()) return PTYC_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (const auto& m : c->marks) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[m.e0], c->ev_pool[m.e1]));
        c->prof_ms[m.kind] += ms;
        c->prof_launches[m.kind] += 1;
        c->prof_units[m.kind] += m.units;
    }
    c->marks.clear();
    c->ev_used = 0;
    return PTYC_OK;
}

// after a synchronisation: did a persistent sweep give up on a barrier?
int check_fault(ptyc_ctx* c) {
    if (!c->sync.p) return PTYC_OK;
    unsigned v[2] = {0, 0};
    HIPCHK(c, hipMemcpy(v, c->sync.p, sizeof(v), hipMemcpyDeviceToHost));
    if (v[1]) {
        c->poisoned = true;
        c->err = "persistent sweep kernel: a grid barrier wait exceeded its bound (results invalid)";
        return PTYC_ERR_HIP;
    }
    return PTYC_OK;
}

}  // namespace

extern "C" {

int ptyc_version(void) { return 100; }

const char* ptyc_init_error(void) { return g_init_error.c_str(); }

int ptyc_init(ptyc_ctx** out, const ptyc_config* cfg, const void* probe0, const void* object0,
              int mem_kind, void* hip_stream) {
    g_init_error.clear();
    std::string why;
    if (!out) { g_init_error = "out is NULL"; return PTYC_ERR_ARG; }
    *out = nullptr;
    int rc = validate_config(cfg, &why);
    if (rc != PTYC_OK) { g_init_error = why; return rc; }
    if (!probe0 || !object0) { g_init_error = "probe0 and object0 must not be NULL"; return PTYC_ERR_ARG; }
    if (!valid_kind(mem_kind)) { g_init_error = "unknown mem_kind"; return PTYC_ERR_ARG; }

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        g_init_error = std::string("no HIP device: ") + hipGetErrorString(e);
        return PTYC_ERR_HIP;
    }
    ptyc_ctx* c = new ptyc_ctx();
    c->cfg = *cfg;
    c->stream = (hipStream_t)hip_stream;
    c->sb = shape_for(cfg->n, kFormBatch);
    c->st = c->sb;
    c->sp = shape_for(cfg->n, kFormPersistent);
    c->sm = shape_for(cfg->n, kFormMixed);
    c->col_blocks_max = std::max(c->sp.col_blocks, c->sm.col_blocks);
    for (int v = 0; v < tile_variants(cfg->n); ++v)
        c->col_blocks_max = std::max(c->col_blocks_max, shape_for(cfg->n, kFormBatch, v).col_blocks);
    if (mixed_n(cfg->n)) c->col_blocks_max = std::max(c->col_blocks_max, multi_col_blocks(cfg->n));
    c->dev_limit = env_limit();
    c->spin_limit = env_spin_limit();
    c->colouring = new Colouring(cfg->n, max_batch_of(c));
    c->ingest.frame_h = c->ingest.frame_w = cfg->n;
    c->ingest.scale = 1.0f;
    c->ingest.flags = cfg->flags;
    (void)hipGetDevice(&c->device);
    if ((e = noalloc_setup(c->device)) != hipSuccess) {
        hip_fail(c, e, "hipGetSymbolAddress(scratch)");
        g_init_error = c->err;
        ptyc_destroy(c);
        return PTYC_ERR_HIP;
    }

    const int n = cfg->n;
    const size_t obj_bytes = (size_t)cfg->h * cfg->w * sizeof(cf);
    const size_t pr_bytes = (size_t)n * n * sizeof(cf);
    auto bail = [&](int code) {
        g_init_error = c->err;
        ptyc_destroy(c);
        return code;
    };
    if ((rc = ensure(c, c->obj, obj_bytes)) != PTYC_OK) return bail(rc);
    if ((rc = ensure(c, c->probe, pr_bytes)) != PTYC_OK) return bail(rc);
    if ((rc = ensure(c, c->tw, n * sizeof(cf))) != PTYC_OK) return bail(rc);
    if ((rc = ensure(c, c->pmax_part, 2 * (size_t)max_probe_blocks(c) * sizeof(float))) != PTYC_OK) return bail(rc);
    if ((rc = ensure(c, c->bad, sizeof(int))) != PTYC_OK) return bail(rc);
    c->capacity = persistent_capacity(n);
    // [0] the persistent sweep's top barrier counter, [1] the barrier fault
    // flag, then its group counters
    const size_t sync_bytes = (size_t)bar_words(std::max(c->capacity, 1)) * sizeof(unsigned);
    if ((rc = ensure(c, c->sync, sync_bytes)) != PTYC_OK) return bail(rc);
    if ((e = hipMemsetAsync(c->sync.p, 0, sync_bytes, c->stream)) != hipSuccess) {
        hip_fail(c, e, "hipMemsetAsync(sync)");
        return bail(PTYC_ERR_HIP);
    }
    // twiddles exp(-2 pi i m / n) in double precision, rounded once to float
    std::vector<cf> tw((size_t)n);
    for (int m = 0; m < n; ++m) {
        const double ang = -2.0 * M_PI * (double)m / (double)n;
        tw[(size_t)m] = cf{(float)std::cos(ang), (float)std::sin(ang)};
    }
    if ((rc = copy_square_in(c, c->tw, tw.data(), n * sizeof(cf), PTYC_MEM_HOST)) != PTYC_OK) return bail(rc);
    if ((rc = copy_square_in(c, c->obj, object0, obj_bytes, mem_kind)) != PTYC_OK) return bail(rc);
    if ((rc = copy_square_in(c, c->probe, probe0, pr_bytes, mem_kind)) != PTYC_OK) return bail(rc);
    if ((e = hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming)) != hipSuccess) {
        hip_fail(c, e, "hipEventCreate");
        return bail(PTYC_ERR_HIP);
    }
    if ((rc = refresh_probe_max(c)) != PTYC_OK) return bail(rc);
    *out = c;
    return PTYC_OK;
}

void ptyc_destroy(ptyc_ctx* c) {
    if (!c) return;
    if (!c->poisoned) (void)hipStreamSynchronize(c->stream);
    DevBuf* bufs[] = {&c->obj, &c->probe, &c->tw, &c->sqrt_i, &c->pos, &c->sum_i, &c->scratch,
                      &c->winmax, &c->pmax_part, &c->order, &c->offs, &c->err_part,
                      &c->err_dev, &c->bad, &c->sync, &c->multi, &c->mask, &c->staging,
                      &c->gorder, &c->goffs, &c->tune_save, &c->mbar, &c->gpart};
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->mgexec) (void)hipGraphExecDestroy(c->mgexec);
    for (DevBuf* b : bufs) release(*b);
    if (c->pinned_order) (void)hipHostFree(c->pinned_order);
    if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    for (auto& ps : c->lpin) {
        if (ps.p) (void)hipHostFree(ps.p);
        if (ps.done) (void)hipEventDestroy(ps.done);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c->colouring;
    delete c;
}

const char* ptyc_last_error(const ptyc_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int64_t ptyc_num_positions(const ptyc_ctx* c) { return c ? c->n_loaded : -1; }

int64_t ptyc_sweep_count(const ptyc_ctx* c) { return c ? c->sweeps_done : -1; }

int ptyc_synchronize(ptyc_ctx* c) {
    int rc = usable(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_fault(c);
}

int ptyc_set_form(ptyc_ctx* c, int form) {
    int rc = usable(c);
    if (rc) return rc;
    if (form == 0) form = kFormBatch;
    if (form != kFormBatch && form != kFormPersistent && form != kFormGraph)
        return fail(c, PTYC_ERR_ARG, "unknown launch form");
    if (form == kFormPersistent && c->capacity <= 0)
        return fail(c, PTYC_ERR_ARG, "the persistent form cannot be launched on this device");
    c->form = form;
    return refresh_probe_max(c);
}

int ptyc_get_form(const ptyc_ctx* c) { return c ? c->form : -1; }

int ptyc_tile_count(const ptyc_ctx* c) { return c ? tile_variants(c->cfg.n) : -1; }

int ptyc_set_tile(ptyc_ctx* c, int tile) {
    int rc = usable(c);
    if (rc) return rc;
    if (tile < 0 || tile >= tile_variants(c->cfg.n)) return fail(c, PTYC_ERR_ARG, "tile variant out of range");
    c->tile = tile;
    c->st = shape_for(c->cfg.n, kFormBatch, tile);
    return PTYC_OK;
}

int ptyc_get_tile(const ptyc_ctx* c) { return c ? c->tile : -1; }

constexpr double kTuneMargin = 0.02;   // a variant must be 2 % faster to replace the current one

int ptyc_tune(ptyc_ctx* c, int32_t reps, int32_t* tile_out, double* ms_out) {
    int rc = usable(c);
    if (rc) return rc;
    if (reps < 1 || reps > 100) return fail(c, PTYC_ERR_ARG, "reps must be in 1..100");
    const int nv = tile_variants(c->cfg.n);
    if (ms_out)
        for (int v = 0; v < PTYC_TILE_MAX; ++v) ms_out[v] = 0.0;
    if (c->n_loaded == 0 || nv <= 1) {
        if (tile_out) *tile_out = c->tile;
        return PTYC_OK;
    }
    // the state a sweep changes: object, probe (and its maxima), sweep counter
    const size_t ob = (size_t)c->cfg.h * c->cfg.w * sizeof(cf), pb = (size_t)c->cfg.n * c->cfg.n * sizeof(cf);
    if ((rc = ensure(c, c->tune_save, ob + pb)) != PTYC_OK) return rc;
    char* save = (char*)c->tune_save.p;
    HIPCHK(c, hipMemcpyAsync(save, c->obj.p, ob, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(save + ob, c->probe.p, pb, hipMemcpyDeviceToDevice, c->stream));
    const int64_t done0 = c->sweeps_done;
    const int form0 = c->form, tile0 = c->tile;
    const bool prof0 = c->prof;
    c->prof = false;
    c->form = kFormBatch;
    auto restore = [&]() -> int {
        HIPCHK(c, hipMemcpyAsync(c->obj.p, save, ob, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->probe.p, save + ob, pb, hipMemcpyDeviceToDevice, c->stream));
        c->sweeps_done = done0;
        return refresh_probe_max(c);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = tile0;
    double best_ms = 0.0;
    std::vector<double> times((size_t)nv, 0.0);
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) rc = hip_fail(c, he, "hipEventCreate");
    for (int v = 0; v < nv && rc == PTYC_OK; ++v) {
        c->tile = v;
        c->st = shape_for(c->cfg.n, kFormBatch, v);
        double vbest = 0.0;
        for (int r = 0; r < reps && rc == PTYC_OK; ++r) {
            if ((rc = restore()) != PTYC_OK) break;
            if ((he = hipEventRecord(e0, c->stream)) != hipSuccess) { rc = hip_fail(c, he, "hipEventRecord"); break; }
            if ((rc = ptyc_sweep(c, 1, nullptr, 0, nullptr, 0, nullptr)) != PTYC_OK) break;
            if ((he = hipEventRecord(e1, c->stream)) != hipSuccess) { rc = hip_fail(c, he, "hipEventRecord"); break; }
            if ((he = hipEventSynchronize(e1)) != hipSuccess) { rc = hip_fail(c, he, "hipEventSynchronize"); break; }
            float ms = 0.f;
            if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_fail(c, he, "hipEventElapsedTime"); break; }
            if (r == 0 || ms < vbest) vbest = ms;
        }
        if (rc != PTYC_OK) break;
        if (ms_out && v < PTYC_TILE_MAX) ms_out[v] = vbest;
        times[(size_t)v] = vbest;
    }
    if (rc == PTYC_OK) {
        // switch only for a clear gain: the variants are often within the
        // noise of one another, and a choice that flips from call to call
        // helps nobody
        best = tile0;
        best_ms = times[(size_t)tile0];
        for (int v = 0; v < nv; ++v)
            if (times[(size_t)v] < best_ms * (1.0 - kTuneMargin)) {
                best = v;
                best_ms = times[(size_t)v];
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->prof = prof0;
    if (c->poisoned) return rc;
    const int keep = rc == PTYC_OK ? best : tile0;
    c->tile = keep;
    c->st = shape_for(c->cfg.n, kFormBatch, keep);
    const int rc2 = restore();            // back to the saved state (batch layout)
    c->form = form0;
    const int rc3 = rc2 == PTYC_OK ? refresh_probe_max(c) : rc2;   // maxima in the caller's form
    if (rc == PTYC_OK) rc = rc3;
    if (rc == PTYC_OK) HIPCHK(c, hipStreamSynchronize(c->stream));
    if (tile_out) *tile_out = c->tile;
    return rc;
}

int ptyc_profile(ptyc_ctx* c, int enable) {
    int rc = usable(c);
    if (rc) return rc;
    if ((rc = collect_profile(c)) != PTYC_OK) return rc;
    c->prof = enable != 0;
    for (int k = 0; k < PTYC_KERNEL_KINDS; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_launches[k] = 0;
        c->prof_units[k] = 0;
    }
    return PTYC_OK;
}

int ptyc_profile_read(ptyc_ctx* c, int kind, double* total_ms, int64_t* launches, int64_t* positions) {
    int rc = usable(c);
    if (rc) return rc;
    if (kind < 0 || kind >= PTYC_KERNEL_KINDS || !total_ms || !launches || !positions)
        return fail(c, PTYC_ERR_ARG, "bad kernel kind or NULL output");
    if ((rc = collect_profile(c)) != PTYC_OK) return rc;
    *total_ms = c->prof_ms[kind];
    *launches = c->prof_launches[kind];
    *positions = c->prof_units[kind];
    return PTYC_OK;
}

int ptyc_add_positions(ptyc_ctx* c, int64_t count, const int32_t* pos_yx, const float* inten,
                       int mem_kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (count < 0) return fail(c, PTYC_ERR_ARG, "count must be >= 0");
    if (count == 0) return PTYC_OK;
    if (!pos_yx || !inten) return fail(c, PTYC_ERR_ARG, "pos_yx and intensities must not be NULL");
    if (!valid_kind(mem_kind)) return fail(c, PTYC_ERR_ARG, "unknown mem_kind");
    const int n = c->cfg.n;
    const size_t nn = (size_t)n * n;

    // positions to the host for the bounds check and the schedule
    std::vector<int32_t> p((size_t)(2 * count));
    if (mem_kind == PTYC_MEM_HOST) {
        std::memcpy(p.data(), pos_yx, p.size() * sizeof(int32_t));
    } else {
        HIPCHK(c, hipMemcpyAsync(p.data(), pos_yx, p.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    for (int64_t i = 0; i < count; ++i) {
        const int32_t y = p[(size_t)(2 * i)], x = p[(size_t)(2 * i + 1)];
        if (y < 0 || x < 0 || y > c->cfg.h - n || x > c->cfg.w - n)
            return fail(c, PTYC_ERR_BOUNDS, "position " + std::to_string(i) + " (" + std::to_string(y) + ", " +
                                                std::to_string(x) + ") puts its window outside the object");
    }
    const int64_t first = c->n_loaded, total = first + count;
    if (total > c->cap) {
        int64_t ncap = std::max<int64_t>(total, std::max<int64_t>(64, c->cap * 2));
        if ((rc = ensure(c, c->sqrt_i, (size_t)ncap * nn * sizeof(float), (size_t)first * nn * sizeof(float))) != PTYC_OK) return rc;
        if ((rc = ensure(c, c->pos, (size_t)ncap * sizeof(int2), (size_t)first * sizeof(int2))) != PTYC_OK) return rc;
        if ((rc = ensure(c, c->sum_i, (size_t)ncap * sizeof(double), (size_t)first * sizeof(double))) != PTYC_OK) return rc;
        c->cap = ncap;
    }
    HIPCHK(c, hipMemsetAsync(c->bad.p, 0, sizeof(int), c->stream));
    const IngestSpec sp = ingest_spec(c);
    const size_t fsz = (size_t)sp.frame_h * sp.frame_w;   // floats per raw frame
    float* dst = (float*)c->sqrt_i.p + (size_t)first * nn;
    double* sdst = (double*)c->sum_i.p + first;
    if (mem_kind == PTYC_MEM_DEVICE) {
        HIPCHK(c, launch_ingest(n, inten, dst, sdst, count, sp, (int*)c->bad.p, c->stream));
    } else {
        // stage through a bounded device buffer
        const int64_t chunk = std::max<int64_t>(1, (int64_t)((size_t)(64u << 20) / (fsz * sizeof(float))));
        const int64_t cn = std::min(chunk, count);
        if ((rc = ensure(c, c->staging, (size_t)cn * fsz * sizeof(float))) != PTYC_OK) return rc;
        for (int64_t a = 0; a < count; a += cn) {
            const int64_t m = std::min(cn, count - a);
            HIPCHK(c, hipMemcpyAsync(c->staging.p, inten + (size_t)a * fsz, (size_t)m * fsz * sizeof(float),
                                     hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, launch_ingest(n, (const float*)c->staging.p, dst + (size_t)a * nn, sdst + a, m, sp,
                                    (int*)c->bad.p, c->stream));
        }
    }
    std::vector<int2> pd((size_t)count);
    for (int64_t i = 0; i < count; ++i) pd[(size_t)i] = make_int2(p[(size_t)(2 * i)], p[(size_t)(2 * i + 1)]);
    HIPCHK(c, hipMemcpyAsync((int2*)c->pos.p + first, pd.data(), (size_t)count * sizeof(int2),
                             hipMemcpyHostToDevice, c->stream));
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->bad.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) return fail(c, PTYC_ERR_ARG, "intensities must be finite and >= 0");
    c->h_pos.insert(c->h_pos.end(), p.begin(), p.end());
    c->colouring->extend(c->h_pos.data(), first, count);
    c->n_loaded = total;
    return PTYC_OK;
}

int ptyc_set_ingest(ptyc_ctx* c, const ptyc_ingest* g) {
    int rc = usable(c);
    if (rc) return rc;
    if (!g) return fail(c, PTYC_ERR_ARG, "spec is NULL");
    if (c->n_loaded > 0 || c->mask.p) return fail(c, PTYC_ERR_ARG, "set the ingest spec before the mask and any data");
    const int n = c->cfg.n;
    if (g->frame_h < n || g->frame_w < n || g->crop_y < 0 || g->crop_x < 0 || g->crop_y > g->frame_h - n ||
        g->crop_x > g->frame_w - n)
        return fail(c, PTYC_ERR_ARG, "the n x n crop must lie inside the frame");
    if (g->orient < 0 || g->orient > 7) return fail(c, PTYC_ERR_ARG, "orient must be in 0..7");
    if (!(g->scale > 0.f) || !std::isfinite(g->scale)) return fail(c, PTYC_ERR_ARG, "scale must be finite and > 0");
    if (g->flags & ~(PTYC_I_IS_SQRT | PTYC_I_CENTERED)) return fail(c, PTYC_ERR_ARG, "unknown flag bits");
    if (g->reserved != 0) return fail(c, PTYC_ERR_ARG, "reserved must be 0");
    c->ingest = *g;
    return PTYC_OK;
}

int ptyc_set_mask(ptyc_ctx* c, const uint8_t* mask, int kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (!mask || !valid_kind(kind)) return fail(c, PTYC_ERR_ARG, "bad mask buffer or mem_kind");
    if (c->n_loaded > 0) return fail(c, PTYC_ERR_ARG, "set the mask before adding data");
    const ptyc_ingest& g = c->ingest;
    const size_t fsz = (size_t)g.frame_h * g.frame_w;
    std::vector<uint8_t> raw(fsz);
    if (kind == PTYC_MEM_HOST) {
        std::memcpy(raw.data(), mask, fsz);
    } else {
        HIPCHK(c, hipMemcpyAsync(raw.data(), mask, fsz, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    const int n = c->cfg.n;
    std::vector<uint8_t> m((size_t)n * n, 0);
    for (int r = 0; r < n; ++r)
        for (int cc = 0; cc < n; ++cc) {
            int a, b;
            ingest_map(g, n, r, cc, &a, &b);
            m[(size_t)a * n + b] = raw[(size_t)(g.crop_y + r) * g.frame_w + g.crop_x + cc] ? 1 : 0;
        }
    if ((rc = ensure(c, c->mask, m.size())) != PTYC_OK) return rc;
    HIPCHK(c, hipMemcpyAsync(c->mask.p, m.data(), m.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PTYC_OK;
}

int ptyc_get_patterns(ptyc_ctx* c, int64_t first, int64_t count, float* out, int kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (first < 0 || count < 0 || first + count > c->n_loaded) return fail(c, PTYC_ERR_ARG, "range outside the loaded positions");
    if (count == 0) return PTYC_OK;
    if (!out || !valid_kind(kind)) return fail(c, PTYC_ERR_ARG, "bad output buffer or mem_kind");
    const size_t nn = (size_t)c->cfg.n * c->cfg.n;
    const float* src = (const float*)c->sqrt_i.p + (size_t)first * nn;
    // the stored layout (column blocks) back to row-major order: directly
    // into a device destination, through the staging buffer for the host
    if (kind == PTYC_MEM_DEVICE) {
        HIPCHK(c, launch_amp_rowmajor(c->cfg.n, src, out, count, c->stream));
    } else {
        const int64_t chunk = std::max<int64_t>(1, (int64_t)((size_t)(64u << 20) / (nn * sizeof(float))));
        const int64_t cn = std::min(chunk, count);
        int rc2;
        if ((rc2 = ensure(c, c->staging, (size_t)cn * nn * sizeof(float))) != PTYC_OK) return rc2;
        for (int64_t k = 0; k < count; k += cn) {
            const int64_t m = std::min(cn, count - k);
            HIPCHK(c, launch_amp_rowmajor(c->cfg.n, src + (size_t)k * nn, (float*)c->staging.p, m, c->stream));
            HIPCHK(c, hipMemcpyAsync(out + (size_t)k * nn, c->staging.p, (size_t)m * nn * sizeof(float),
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PTYC_OK;
}

int ptyc_get_schedule(ptyc_ctx* c, int64_t* order, int64_t* off, int64_t* n_batches) {
    int rc = usable(c);
    if (rc) return rc;
    if (!n_batches) return fail(c, PTYC_ERR_ARG, "n_batches must not be NULL");
    std::vector<int64_t> o, f;
    default_schedule(c, c->sweeps_done, o, f);
    *n_batches = (int64_t)f.size() - 1;
    if (order) std::memcpy(order, o.data(), o.size() * sizeof(int64_t));
    if (off) std::memcpy(off, f.data(), f.size() * sizeof(int64_t));
    return PTYC_OK;
}

}  // extern "C"

namespace {

// Schedules of the sweeps of one call, before anything reaches the device.
struct Plan {
    std::vector<std::vector<int64_t>> orders, offs;
    int64_t olen = 0, nb = 0, max_b = 1;
};

// Validate the arguments of a sweep call and build its schedules.  Leaves
// p.olen == 0 when there is nothing to run.
int plan_sweeps(ptyc_ctx* c, int32_t n_sweeps, const int64_t* order, int64_t order_len, const int64_t* off,
                int64_t n_batches, Plan& p) {
    std::string why;
    const bool strict = c->cfg.mode == PTYC_MODE_STRICT;
    if (order) {
        if (order_len < 0) return fail(c, PTYC_ERR_ARG, "order_len must be >= 0");
        if (strict && off) return fail(c, PTYC_ERR_ARG, "strict mode takes no batch_offsets");
        if (!strict && !off) return fail(c, PTYC_ERR_ARG, "coloured mode needs batch_offsets with an explicit order");
        if (!strict) {
            if (n_batches < 0) return fail(c, PTYC_ERR_ARG, "n_batches must be >= 0");
            if (!check_batches(c->n_loaded, c->h_pos.data(), c->cfg.n, order, order_len, off, n_batches, &why))
                return fail(c, PTYC_ERR_ARG, why);
        } else {
            for (int64_t i = 0; i < order_len; ++i)
                if (order[i] < 0 || order[i] >= c->n_loaded)
                    return fail(c, PTYC_ERR_ARG, "order index " + std::to_string(order[i]) + " is not a loaded position");
        }
    }
    p = Plan{};
    if (c->n_loaded == 0 || (order && order_len == 0)) return PTYC_OK;
    p.orders.resize((size_t)n_sweeps);
    p.offs.resize((size_t)n_sweeps);
    for (int s = 0; s < n_sweeps; ++s) {
        if (order) {
            p.orders[(size_t)s].assign(order, order + order_len);
            if (strict) {
                p.offs[(size_t)s].resize((size_t)order_len + 1);
                for (int64_t i = 0; i <= order_len; ++i) p.offs[(size_t)s][(size_t)i] = i;
            } else {
                p.offs[(size_t)s].assign(off, off + n_batches + 1);
            }
        } else {
            default_schedule(c, c->sweeps_done + s, p.orders[(size_t)s], p.offs[(size_t)s]);
        }
    }
    p.olen = (int64_t)p.orders[0].size();
    p.nb = (int64_t)p.offs[0].size() - 1;
    for (int s = 1; s < n_sweeps; ++s)
        if ((int64_t)p.offs[(size_t)s].size() - 1 != p.nb) return fail(c, PTYC_ERR_ARG, "internal: batch count varies");
    for (int s = 0; s < n_sweeps; ++s)
        for (size_t b = 0; b + 1 < p.offs[(size_t)s].size(); ++b)
            p.max_b = std::max(p.max_b, p.offs[(size_t)s][b + 1] - p.offs[(size_t)s][b]);
    return PTYC_OK;
}

// The device form of an order: each position index with its window corner.
void to_entries(const ptyc_ctx* c, const int64_t* idx, int64_t n, OrderEntry* out) {
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j = idx[i];
        out[i] = OrderEntry{c->h_pos[(size_t)(2 * j)], c->h_pos[(size_t)(2 * j + 1)], j};
    }
}

// Size the work buffers for a plan, upload its orders and offsets, refresh
// the probe maxima in the layout of `form`.
int stage_plan(ptyc_ctx* c, const Plan& p, int32_t n_sweeps, int form) {
    int rc;
    const size_t nn = (size_t)c->cfg.n * c->cfg.n;
    if (p.max_b > c->slots) {
        if ((rc = ensure(c, c->scratch, (size_t)p.max_b * nn * sizeof(cf))) != PTYC_OK) return rc;
        if ((rc = ensure(c, c->winmax, (size_t)p.max_b * max_row_blocks(c) * sizeof(float))) != PTYC_OK) return rc;
        c->slots = p.max_b;
    }
    const size_t obytes = (size_t)n_sweeps * p.olen * sizeof(OrderEntry);
    const size_t fbytes = (size_t)n_sweeps * (p.nb + 1) * sizeof(int64_t);
    if (c->upload_pending) {
        HIPCHK(c, hipEventSynchronize(c->upload_done));
        c->upload_pending = false;
    }
    if ((rc = ensure(c, c->order, obytes)) != PTYC_OK) return rc;
    if ((rc = ensure(c, c->offs, fbytes)) != PTYC_OK) return rc;
    if ((rc = ensure(c, c->err_part, (size_t)p.olen * max_col_blocks(c) * sizeof(double))) != PTYC_OK) return rc;
    if ((rc = ensure(c, c->err_dev, (size_t)n_sweeps * sizeof(double))) != PTYC_OK) return rc;
    if (c->pinned_bytes < obytes + fbytes) {
        if (c->pinned_order) (void)hipHostFree(c->pinned_order);
        c->pinned_order = nullptr;
        c->pinned_bytes = 0;
        hipError_t e = hipHostMalloc((void**)&c->pinned_order, obytes + fbytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, PTYC_ERR_OOM, "pinned host allocation failed");
        }
        c->pinned_bytes = obytes + fbytes;
    }
    OrderEntry* pin_ent = (OrderEntry*)c->pinned_order;
    int64_t* pin_off = (int64_t*)(pin_ent + (size_t)n_sweeps * p.olen);
    for (int s = 0; s < n_sweeps; ++s) {
        to_entries(c, p.orders[(size_t)s].data(), p.olen, pin_ent + (size_t)s * p.olen);
        std::memcpy(pin_off + (size_t)s * (p.nb + 1), p.offs[(size_t)s].data(), (size_t)(p.nb + 1) * sizeof(int64_t));
    }
    HIPCHK(c, hipMemcpyAsync(c->order.p, c->pinned_order, obytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->offs.p, pin_off, fbytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipEventRecord(c->upload_done, c->stream));
    c->upload_pending = true;
    BatchArgs a = base_args(c);
    a.bsize = 0;
    HIPCHK(c, launch_probe_reduce(c->cfg.n, a, form, c->stream));
    c->pmax_cur ^= 1;
    return PTYC_OK;
}

// the error-metric reduction of sweep s of a plan whose column stage wrote
// gc partials per position
int launch_sweep_error(ptyc_ctx* c, const Plan& p, int s, int gc) {
    const OrderEntry* ord = (const OrderEntry*)c->order.p + (size_t)s * p.olen;
    HIPCHK(c, launch_err_reduce((const double*)c->err_part.p, p.olen * gc, ord, p.olen, (const double*)c->sum_i.p,
                                (double*)c->err_dev.p + s, c->stream));
    return PTYC_OK;
}

// do two graph keys name the same buffers and constants?
bool same_key(const BatchArgs& x, const BatchArgs& y) {
    return x.obj == y.obj && x.h == y.h && x.w == y.w && x.probe == y.probe && x.tw == y.tw &&
           x.sqrt_i == y.sqrt_i && x.pos == y.pos && x.order == y.order && x.scratch == y.scratch &&
           x.winmax == y.winmax &&
           x.pmax_in == y.pmax_in && x.pmax_out == y.pmax_out && x.err_part == y.err_part &&
           x.alpha == y.alpha && x.beta == y.beta && x.mask == y.mask && x.boffs == y.boffs;
}

// sweep s of a plan in the graph form: (re)build the graph if needed, copy
// the sweep's order and offsets into the graph's fixed buffers, replay
int graph_sweep(ptyc_ctx* c, const Plan& p, int s) {
    int rc;
    if ((rc = ensure(c, c->gorder, (size_t)p.olen * sizeof(OrderEntry))) != PTYC_OK) return rc;
    if ((rc = ensure(c, c->goffs, (size_t)(p.nb + 1) * sizeof(int64_t))) != PTYC_OK) return rc;
    // the graph's first node reads the maxima from half 0
    if (c->pmax_cur != 0 && (rc = refresh_probe_max(c)) != PTYC_OK) return rc;
    BatchArgs a = base_args(c);
    a.order = (const OrderEntry*)c->gorder.p;
    a.boffs = (const int64_t*)c->goffs.p;
    if (!c->gexec || c->g_nb != p.nb || c->g_maxb < p.max_b || c->g_tile != c->tile || !same_key(a, c->gkey)) {
        if (c->gexec) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            HIPCHK(c, hipGraphExecDestroy(c->gexec));
            c->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPCHK(c, build_sweep_graph(c->cfg.n, c->tile, a, (int)p.nb, (int)p.max_b, &g));
        hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->gexec = nullptr;
            return hip_fail(c, e, "hipGraphInstantiate");
        }
        c->gkey = a;
        c->g_nb = p.nb;
        c->g_maxb = p.max_b;
        c->g_tile = c->tile;
    }
    HIPCHK(c, hipMemcpyAsync(c->gorder.p, (const OrderEntry*)c->order.p + (size_t)s * p.olen,
                             (size_t)p.olen * sizeof(OrderEntry), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->goffs.p, (const int64_t*)c->offs.p + (size_t)s * (p.nb + 1),
                             (size_t)(p.nb + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream));
    size_t e0 = 0;
    if (c->prof) {
        if ((rc = take_events(c, 2, &e0)) != PTYC_OK) return rc;
        HIPCHK(c, hipEventRecord(c->ev_pool[e0], c->stream));
    }
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    c->pmax_cur = (int)(p.nb & 1);
    if (c->prof) {
        HIPCHK(c, hipEventRecord(c->ev_pool[e0 + 1], c->stream));
        c->marks.push_back({PTYC_KERNEL_GRAPH, e0, e0 + 1, p.olen});
    }
    return PTYC_OK;
}

// How a multi-context call runs.  persistent: one persistent kernel for all
// scans (pattern sizes 64, 128, 256), each scan on its own group of
// workgroups with its own barriers; inv64 / inv128: the inverse-stage tile
// at 64 and 128 px; share: workgroups are given to scans in proportion to
// (positions x N^2 log2 N)^share, capped at what a scan's largest stage can
// use.  Otherwise every unfinished scan advances one batch per step, three
// launches per step for all scans together, and a scan whose largest batch
// holds at most `small` positions uses the eight-slot inverse tile.
struct MultiVariant {
    bool persistent;
    int inv64, inv128;
    double share;
    int small;
};
constexpr MultiVariant kMultiVariants[] = {
    {true, 0, 0, 1.0, 0},   {true, 1, 1, 1.0, 0},   {true, 1, 1, 0.5, 0}, {true, 0, 0, 0.5, 0},
    {false, 0, 0, 1.0, 0},  {false, 0, 0, 1.0, 8},  {false, 0, 0, 1.0, 16},
};
constexpr int kMultiVariantCount = (int)(sizeof(kMultiVariants) / sizeof(kMultiVariants[0]));

// Workgroups per scan: at least one each, the rest in proportion to the
// weights, none beyond its cap, whatever a capped scan cannot use going to
// the others (largest remainders first).  Returns the total given.
int share_groups(const std::vector<double>& wt, const std::vector<int>& cap, int total, std::vector<int>& g) {
    const size_t k = wt.size();
    g.assign(k, 1);
    int left = total - (int)k;
    while (left > 0) {
        double sw = 0.0;
        for (size_t i = 0; i < k; ++i)
            if (g[i] < cap[i]) sw += wt[i];
        if (sw <= 0.0) break;
        std::vector<std::pair<double, size_t>> frac;
        int given = 0;
        for (size_t i = 0; i < k; ++i) {
            if (g[i] >= cap[i]) continue;
            const double want = left * wt[i] / sw;
            int add = std::min((int)want, cap[i] - g[i]);
            g[i] += add;
            given += add;
            if (g[i] < cap[i]) frac.push_back({want - std::floor(want), i});
        }
        std::sort(frac.begin(), frac.end(), [](auto& x, auto& y) { return x.first > y.first || (x.first == y.first && x.second < y.second); });
        for (auto& f : frac) {
            if (given >= left) break;
            if (g[f.second] < cap[f.second]) {
                ++g[f.second];
                ++given;
            }
        }
        if (given == 0) break;
        left -= given;
    }
    int sum = 0;
    for (int x : g) sum += x;
    return sum;
}

// the barrier counters of the scans of a multi-scan launch lie a multiple
// of kBarStride counters (4 KiB) apart: workgroups of different scans then
// poll different memory lines
constexpr size_t kBarStride = 1024;

// The persistent multi-scan launch.  Plans are staged (orders and offsets
// of all sweeps on each context's device buffers, probe maxima refreshed).
int multi_persistent(ptyc_ctx* const* ctxs, int n_ctx, int n_sweeps, double* err_out, const std::vector<Plan>& plans,
                     const MultiVariant& mv) {
    ptyc_ctx* c0 = ctxs[0];
    std::vector<ScanArgs> sc;
    std::vector<int> who, cap;
    std::vector<double> wt;
    for (int i = 0; i < n_ctx; ++i) {
        const Plan& p = plans[(size_t)i];
        if (p.olen == 0) continue;
        ptyc_ctx* c = ctxs[i];
        const int n = c->cfg.n;
        ScanArgs x{};
        x.a = base_args(c);
        x.a.order = (const OrderEntry*)c->order.p;
        x.offs = (const int64_t*)c->offs.p;
        x.olen = p.olen;
        x.nb = (int)p.nb;
        x.n_sweeps = n_sweeps;
        x.inv_tile = n == 64 ? mv.inv64 : n == 128 ? mv.inv128 : 0;
        x.err = err_out ? (double*)c->err_dev.p : nullptr;
        x.sum_i = (const double*)c->sum_i.p;
        x.spin_limit = c0->spin_limit;
        sc.push_back(x);
        who.push_back(i);
        cap.push_back(multi_need(n, (int)p.max_b, x.inv_tile));
        wt.push_back(std::pow((double)p.olen * n * n * std::log2((double)n), mv.share));
    }
    if (c0->capacity_multi <= 0) c0->capacity_multi = multi_capacity();
    if (sc.empty() || (int)sc.size() > c0->capacity_multi) return 1;   // nothing to run / not enough workgroups
    std::vector<int> g;
    const int grid = share_groups(wt, cap, c0->capacity_multi, g);
    int g0 = 0;
    int rc;
    size_t stride = kBarStride;   // counters per scan: bar_words of its workgroups, in whole 4 KiB steps
    for (size_t k = 0; k < sc.size(); ++k)
        stride = std::max(stride, ((size_t)bar_words(g[k]) + kBarStride - 1) / kBarStride * kBarStride);
    const int n_bars = (int)(sc.size() * stride);
    if ((rc = ensure(c0, c0->mbar, (size_t)n_bars * sizeof(unsigned))) != PTYC_OK) return rc;
    for (size_t k = 0; k < sc.size(); ++k) {
        sc[k].g0 = g0;
        sc[k].gn = g[k];
        sc[k].bar = (unsigned*)c0->mbar.p + k * stride;
        g0 += g[k];
    }
    // the descriptor table may still be read by an earlier call's kernels
    HIPCHK(c0, hipStreamSynchronize(c0->stream));
    if ((rc = ensure(c0, c0->multi, sc.size() * sizeof(ScanArgs))) != PTYC_OK) return rc;
    HIPCHK(c0, hipMemcpyAsync(c0->multi.p, sc.data(), sc.size() * sizeof(ScanArgs), hipMemcpyHostToDevice,
                              c0->stream));
    HIPCHK(c0, hipStreamSynchronize(c0->stream));
    const ScanArgs* dev = (const ScanArgs*)c0->multi.p;
    int* fault = (int*)((unsigned*)c0->sync.p + 1);
    if (c0->form == kFormGraph) {
        // the launch built as a graph once and replayed while the table, the
        // scan count and the grid stay the same (the table's contents change
        // from call to call; the kernels read them when they run)
        if (!c0->mgexec || c0->mg_tab != (const void*)dev || c0->mg_count != (int)sc.size() || c0->mg_grid != grid ||
            c0->mg_bars != c0->mbar.p || c0->mg_nbars != n_bars) {
            if (c0->mgexec) {
                HIPCHK(c0, hipGraphExecDestroy(c0->mgexec));
                c0->mgexec = nullptr;
            }
            hipGraph_t gr = nullptr;
            HIPCHK(c0, build_multi_graph(dev, (int)sc.size(), grid, (unsigned*)c0->mbar.p, n_bars, fault, &gr));
            const hipError_t ie = hipGraphInstantiate(&c0->mgexec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (ie != hipSuccess) {
                c0->mgexec = nullptr;
                return hip_fail(c0, ie, "hipGraphInstantiate");
            }
            c0->mg_tab = dev;
            c0->mg_count = (int)sc.size();
            c0->mg_grid = grid;
            c0->mg_bars = c0->mbar.p;
            c0->mg_nbars = n_bars;
        }
        HIPCHK(c0, hipGraphLaunch(c0->mgexec, c0->stream));
    } else {
        HIPCHK(c0, launch_multi_persist(dev, (int)sc.size(), grid, (unsigned*)c0->mbar.p, n_bars, fault, true,
                                        c0->stream));
    }
    // each kernel swapped its scan's maxima halves after every non-empty batch
    for (size_t k = 0; k < sc.size(); ++k) {
        ptyc_ctx* c = ctxs[who[k]];
        const Plan& p = plans[(size_t)who[k]];
        int flips = 0;
        for (int s = 0; s < n_sweeps; ++s)
            for (size_t b = 0; b + 1 < p.offs[(size_t)s].size(); ++b) flips += p.offs[(size_t)s][b + 1] > p.offs[(size_t)s][b];
        c->pmax_cur ^= flips & 1;
    }
    for (int i = 0; i < n_ctx; ++i) ctxs[i]->sweeps_done += n_sweeps;
    if (err_out) {
        for (int i = 0; i < n_ctx; ++i) {
            if (plans[(size_t)i].olen == 0) {
                for (int s = 0; s < n_sweeps; ++s) err_out[(size_t)i * n_sweeps + s] = 0.0;
                continue;
            }
            HIPCHK(c0, hipMemcpyAsync(err_out + (size_t)i * n_sweeps, ctxs[i]->err_dev.p,
                                      (size_t)n_sweeps * sizeof(double), hipMemcpyDeviceToHost, c0->stream));
        }
        HIPCHK(c0, hipStreamSynchronize(c0->stream));
        return check_fault(c0);
    }
    return PTYC_OK;
}

}  // namespace

extern "C" {

int ptyc_sweep(ptyc_ctx* c, int32_t n_sweeps, const int64_t* order, int64_t order_len,
               const int64_t* off, int64_t n_batches, double* err_out) {
    int rc = usable(c);
    if (rc) return rc;
    if (n_sweeps < 0) return fail(c, PTYC_ERR_ARG, "n_sweeps must be >= 0");
    if (n_sweeps == 0) return PTYC_OK;
    Plan p;
    if ((rc = plan_sweeps(c, n_sweeps, order, order_len, off, n_batches, p)) != PTYC_OK) return rc;
    if (p.olen == 0) {
        if (err_out)
            for (int s = 0; s < n_sweeps; ++s) err_out[s] = 0.0;
        c->sweeps_done += n_sweeps;
        return PTYC_OK;
    }
    if ((rc = stage_plan(c, p, n_sweeps, c->form)) != PTYC_OK) return rc;
    const int64_t olen = p.olen, nb = p.nb;
    for (int s = 0; s < n_sweeps; ++s) {
        BatchArgs a = base_args(c);
        a.order = (const OrderEntry*)c->order.p + (size_t)s * olen;
        if (c->form == kFormPersistent && c->cfg.mode == PTYC_MODE_STRICT && c->cfg.n <= kStrictMaxN) {
            // sequential ePIE: one workgroup walks the whole order
            size_t e0 = 0;
            if (c->prof) {
                if ((rc = take_events(c, 2, &e0)) != PTYC_OK) return rc;
                HIPCHK(c, hipEventRecord(c->ev_pool[e0], c->stream));
            }
            a.off = 0;
            HIPCHK(c, launch_strict(c->cfg.n, a, (int)olen, c->stream));
            if (c->prof) {
                HIPCHK(c, hipEventRecord(c->ev_pool[e0 + 1], c->stream));
                c->marks.push_back({PTYC_KERNEL_STRICT, e0, e0 + 1, olen});
            }
            if ((rc = refresh_probe_max(c)) != PTYC_OK) return rc;
            if (err_out && (rc = launch_sweep_error(c, p, s, 1)) != PTYC_OK) return rc;
            continue;
        } else if (c->form == kFormPersistent) {
            ScanArgs sc{};
            sc.a = a;
            sc.offs = (const int64_t*)c->offs.p + (size_t)s * (nb + 1);
            sc.olen = olen;
            sc.nb = (int)nb;
            sc.n_sweeps = 1;
            sc.bar = (unsigned*)c->sync.p;
            sc.spin_limit = c->spin_limit;
            sc.sum_i = (const double*)c->sum_i.p;
            size_t e0 = 0;
            if (c->prof) {
                if ((rc = take_events(c, 2, &e0)) != PTYC_OK) return rc;
                HIPCHK(c, hipEventRecord(c->ev_pool[e0], c->stream));
            }
            HIPCHK(c, launch_sweep(c->cfg.n, sc, (int)p.max_b, c->capacity, (int*)((unsigned*)c->sync.p + 1),
                                   c->stream));
            // the kernel swaps the maxima halves after every non-empty batch
            const auto& f = p.offs[(size_t)s];
            for (size_t b = 0; b + 1 < f.size(); ++b) c->pmax_cur ^= (f[b + 1] > f[b]) ? 1 : 0;
            if (c->prof) {
                HIPCHK(c, hipEventRecord(c->ev_pool[e0 + 1], c->stream));
                c->marks.push_back({PTYC_KERNEL_SWEEP, e0, e0 + 1, olen});
            }
        } else if (c->form == kFormGraph) {
            if ((rc = graph_sweep(c, p, s)) != PTYC_OK) return rc;
        } else {
            const auto& f = p.offs[(size_t)s];
            for (size_t b = 0; b + 1 < f.size(); ++b) {
                a.off = f[b];
                a.bsize = (int)(f[b + 1] - f[b]);
                if (a.bsize == 0) continue;
                a.pmax_in = pmax_half(c, c->pmax_cur);
                a.pmax_out = pmax_half(c, c->pmax_cur ^ 1);
                c->pmax_cur ^= 1;
                if (c->prof) {
                    size_t e0 = 0;
                    if ((rc = take_events(c, 6, &e0)) != PTYC_OK) return rc;
                    hipEvent_t ev[6];
                    for (int k = 0; k < 6; ++k) ev[k] = c->ev_pool[e0 + k];
                    HIPCHK(c, launch_batch(c->cfg.n, c->tile, a, c->stream, ev));
                    c->marks.push_back({PTYC_KERNEL_ROWS_FWD, e0, e0 + 1, a.bsize});
                    c->marks.push_back({PTYC_KERNEL_COLS, e0 + 2, e0 + 3, a.bsize});
                    c->marks.push_back({PTYC_KERNEL_ROWS_INV, e0 + 4, e0 + 5, a.bsize});
                } else {
                    HIPCHK(c, launch_batch(c->cfg.n, c->tile, a, c->stream));
                }
            }
        }
        if (err_out && (rc = launch_sweep_error(c, p, s, shape_of(c).col_blocks)) != PTYC_OK) return rc;
    }
    c->sweeps_done += n_sweeps;
    if (err_out) {
        HIPCHK(c, hipMemcpyAsync(err_out, c->err_dev.p, (size_t)n_sweeps * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return check_fault(c);
    }
    return PTYC_OK;
}

int ptyc_sweep_noalloc(ptyc_ctx* c, int32_t n_sweeps, const int64_t* order, int64_t order_len,
                       const int64_t* off, int64_t n_batches, double* err_out) {
    int rc = usable(c);
    if (rc) return rc;
    if (n_sweeps < 0) return fail(c, PTYC_ERR_ARG, "n_sweeps must be >= 0");
    if (n_sweeps == 0) return PTYC_OK;
    // one error sum per sweep must fit beside the rest (checked before the
    // schedules of all sweeps are built on the host)
    if ((size_t)n_sweeps * sizeof(double) > kNoallocBytes / 4)
        return fail(c, PTYC_ERR_ARG, "ptyc_sweep_noalloc: too many sweeps in one call for its work memory");
    Plan p;
    if ((rc = plan_sweeps(c, n_sweeps, order, order_len, off, n_batches, p)) != PTYC_OK) return rc;
    unsigned char* base = (unsigned char*)noalloc_ptr(c->device);
    if (!base) return fail(c, PTYC_ERR_STATE, "no work memory address for this device");
    if (p.olen == 0) {
        if (err_out)
            for (int s = 0; s < n_sweeps; ++s) err_out[s] = 0.0;
        c->sweeps_done += n_sweeps;
        return PTYC_OK;
    }
    // layout of the work memory: one sweep's order entries, the spectrum
    // exchange of the largest batch, its partial maxima of |S_j O|^2, the
    // error partials of one sweep and one error sum per sweep
    const size_t nn = (size_t)c->cfg.n * c->cfg.n;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_ent = 0;
    const size_t o_exch = o_ent + up((size_t)p.olen * sizeof(OrderEntry));
    const size_t o_wmax = o_exch + up((size_t)p.max_b * nn * sizeof(cf));
    const size_t o_epart = o_wmax + up((size_t)p.max_b * c->st.row_blocks * sizeof(float));
    const size_t o_esum = o_epart + up((size_t)p.olen * c->st.col_blocks * sizeof(double));
    const size_t total = o_esum + up((size_t)n_sweeps * sizeof(double));
    if (total > kNoallocBytes)
        return fail(c, PTYC_ERR_ARG, "ptyc_sweep_noalloc needs " + std::to_string(total) +
                                         " bytes of work memory; its limit is " + std::to_string(kNoallocBytes));
    // an earlier pinned upload of ptyc_sweep may still be in flight
    if (c->upload_pending) {
        HIPCHK(c, hipEventSynchronize(c->upload_done));
        c->upload_pending = false;
    }
    OrderEntry* d_ent = (OrderEntry*)(base + o_ent);
    double* d_epart = (double*)(base + o_epart);
    double* d_esum = (double*)(base + o_esum);
    if ((rc = refresh_probe_max(c)) != PTYC_OK) return rc;
    std::vector<OrderEntry> ents((size_t)p.olen);
    for (int s = 0; s < n_sweeps; ++s) {
        to_entries(c, p.orders[(size_t)s].data(), p.olen, ents.data());
        // pageable source: the copy has read `ents` when the call returns,
        // and it runs after the previous sweep's kernels on the stream
        HIPCHK(c, hipMemcpyAsync(d_ent, ents.data(), (size_t)p.olen * sizeof(OrderEntry), hipMemcpyHostToDevice,
                                 c->stream));
        BatchArgs a = base_args(c);
        a.order = d_ent;
        a.scratch = (cf*)(base + o_exch);
        a.winmax = (float*)(base + o_wmax);
        a.err_part = d_epart;
        const auto& f = p.offs[(size_t)s];
        for (size_t b = 0; b + 1 < f.size(); ++b) {
            a.off = f[b];
            a.bsize = (int)(f[b + 1] - f[b]);
            if (a.bsize == 0) continue;
            a.pmax_in = pmax_half(c, c->pmax_cur);
            a.pmax_out = pmax_half(c, c->pmax_cur ^ 1);
            c->pmax_cur ^= 1;
            HIPCHK(c, launch_batch(c->cfg.n, c->tile, a, c->stream));
        }
        if (err_out)
            HIPCHK(c, launch_err_reduce(d_epart, p.olen * c->st.col_blocks, d_ent, p.olen,
                                        (const double*)c->sum_i.p, d_esum + s, c->stream));
    }
    c->sweeps_done += n_sweeps;
    if (err_out)
        HIPCHK(c, hipMemcpyAsync(err_out, d_esum, (size_t)n_sweeps * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PTYC_OK;
}

int ptyc_sweep_multi(ptyc_ctx* const* ctxs, int32_t n_ctx, int32_t n_sweeps, double* err_out) {
    if (!ctxs || n_ctx <= 0 || n_ctx > PTYC_MULTI_MAX || n_sweeps < 0) return PTYC_ERR_ARG;
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i]) return PTYC_ERR_ARG;
        int rc = usable(ctxs[i]);
        if (rc) return rc;
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) return fail(ctxs[i], PTYC_ERR_ARG, "a context appears twice");
        if (ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->device != ctxs[0]->device)
            return fail(ctxs[i], PTYC_ERR_ARG, "all contexts must share one device and stream");
    }
    if (n_sweeps == 0) return PTYC_OK;
    int rc;
    std::vector<Plan> plans((size_t)n_ctx);
    for (int i = 0; i < n_ctx; ++i)
        if ((rc = plan_sweeps(ctxs[i], n_sweeps, nullptr, 0, nullptr, 0, plans[(size_t)i])) != PTYC_OK) return rc;
    for (int i = 0; i < n_ctx; ++i)
        if (plans[(size_t)i].olen > 0 && (rc = stage_plan(ctxs[i], plans[(size_t)i], n_sweeps, kFormBatch)) != PTYC_OK)
            return rc;
    const MultiVariant& mv = kMultiVariants[ctxs[0]->multi_variant];
    bool persistent = mv.persistent;
    for (int i = 0; i < n_ctx; ++i) persistent = persistent && mixed_n(ctxs[i]->cfg.n);
    if (persistent) {
        rc = multi_persistent(ctxs, n_ctx, n_sweeps, err_out, plans, mv);
        if (rc <= 0) return rc;   // else: fewer workgroups than scans, or nothing to run; the stepped launches below
    }
    // one step advances every unfinished context by one batch.  The pattern
    // sizes 64, 128 and 256 share three launches per step (mixed-size
    // kernels); 16 and 32 get three launches per size.  (Running the sizes
    // on streams of their own instead was measured slower: each kernel
    // boundary's cache maintenance then lands in the middle of the other
    // streams' kernels.)
    int64_t steps = 0;
    for (int i = 0; i < n_ctx; ++i) steps = std::max(steps, (int64_t)n_sweeps * plans[(size_t)i].nb);
    constexpr int kGroups[] = {0, 16, 32};        // 0: the mixed-size group
    std::vector<BatchArgs> tab;
    struct Launch {
        int n;                                    // 0: mixed sizes
        size_t first;
        int count;
        std::vector<std::pair<int, int>> ends;    // (context, sweep) whose sweep ends with this launch
    };
    std::vector<Launch> work;                     // in step order
    for (int64_t k = 0; k < steps; ++k) {
        for (int grp : kGroups) {
            Launch L{grp, tab.size(), 0, {}};
            for (int i = 0; i < n_ctx; ++i) {
                ptyc_ctx* c = ctxs[i];
                const Plan& p = plans[(size_t)i];
                const bool in = grp == 0 ? mixed_n(c->cfg.n) : c->cfg.n == grp;
                if (!in || p.olen == 0 || k >= (int64_t)n_sweeps * p.nb) continue;
                const int s = (int)(k / p.nb);
                const int64_t b = k % p.nb;
                BatchArgs a = base_args(c);
                a.itile = p.max_b <= mv.small ? 1 : 0;
                c->pmax_cur ^= 1;   // this entry's inverse stage writes the other half
                a.order = (const OrderEntry*)c->order.p + (size_t)s * p.olen;
                a.off = p.offs[(size_t)s][(size_t)b];
                a.bsize = (int)(p.offs[(size_t)s][(size_t)b + 1] - a.off);
                tab.push_back(a);
                ++L.count;
                if (b == p.nb - 1) L.ends.push_back({i, s});
            }
            if (L.count) work.push_back(std::move(L));
        }
    }
    ptyc_ctx* c0 = ctxs[0];
    // the descriptor table may still be read by an earlier call's kernels
    HIPCHK(c0, hipStreamSynchronize(c0->stream));
    if ((rc = ensure(c0, c0->multi, tab.size() * sizeof(BatchArgs))) != PTYC_OK) return rc;
    if (!tab.empty()) {
        HIPCHK(c0, hipMemcpyAsync(c0->multi.p, tab.data(), tab.size() * sizeof(BatchArgs), hipMemcpyHostToDevice,
                                  c0->stream));
        HIPCHK(c0, hipStreamSynchronize(c0->stream));
    }
    for (const Launch& L : work) {
        const BatchArgs* dev = (const BatchArgs*)c0->multi.p + L.first;
        if (L.n == 0)
            HIPCHK(c0, launch_batch_mixed(dev, tab.data() + L.first, L.count, c0->stream));
        else
            HIPCHK(c0, launch_batch_multi(L.n, dev, tab.data() + L.first, L.count, c0->stream));
        if (err_out)
            for (auto [i, s] : L.ends) {
                ptyc_ctx* c = ctxs[i];
                const int gc = L.n == 0 ? c->sm.col_blocks : c->sb.col_blocks;
                if ((rc = launch_sweep_error(c, plans[(size_t)i], s, gc)) != PTYC_OK) return rc;
            }
    }
    for (int i = 0; i < n_ctx; ++i) ctxs[i]->sweeps_done += n_sweeps;
    if (err_out) {
        for (int i = 0; i < n_ctx; ++i) {
            if (plans[(size_t)i].olen == 0) {
                for (int s = 0; s < n_sweeps; ++s) err_out[(size_t)i * n_sweeps + s] = 0.0;
                continue;
            }
            HIPCHK(c0, hipMemcpyAsync(err_out + (size_t)i * n_sweeps, ctxs[i]->err_dev.p,
                                      (size_t)n_sweeps * sizeof(double), hipMemcpyDeviceToHost, c0->stream));
        }
        HIPCHK(c0, hipStreamSynchronize(c0->stream));
    }
    return PTYC_OK;
}

int ptyc_multi_variant_count(void) { return kMultiVariantCount; }

int ptyc_set_multi_variant(ptyc_ctx* c, int v) {
    int rc = usable(c);
    if (rc) return rc;
    if (v < 0 || v >= kMultiVariantCount) return fail(c, PTYC_ERR_ARG, "multi-context variant out of range");
    c->multi_variant = v;
    return PTYC_OK;
}

int ptyc_get_multi_variant(const ptyc_ctx* c) { return c ? c->multi_variant : -1; }

int ptyc_tune_multi(ptyc_ctx* const* ctxs, int32_t n_ctx, int32_t reps, int32_t* variant_out, double* ms_out) {
    if (!ctxs || n_ctx <= 0 || n_ctx > PTYC_MULTI_MAX) return PTYC_ERR_ARG;
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i]) return PTYC_ERR_ARG;
        int rc = usable(ctxs[i]);
        if (rc) return rc;
    }
    ptyc_ctx* c0 = ctxs[0];
    if (reps < 1 || reps > 100) return fail(c0, PTYC_ERR_ARG, "reps must be in 1..100");
    if (ms_out)
        for (int v = 0; v < PTYC_MULTI_VARIANTS; ++v) ms_out[v] = 0.0;
    int rc;
    // the state a sweep changes: object, probe (and its maxima), sweep counter
    std::vector<int64_t> done0((size_t)n_ctx);
    for (int i = 0; i < n_ctx; ++i) {
        ptyc_ctx* c = ctxs[i];
        const size_t ob = (size_t)c->cfg.h * c->cfg.w * sizeof(cf), pb = (size_t)c->cfg.n * c->cfg.n * sizeof(cf);
        if ((rc = ensure(c, c->tune_save, ob + pb)) != PTYC_OK) return rc;
        HIPCHK(c, hipMemcpyAsync(c->tune_save.p, c->obj.p, ob, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync((char*)c->tune_save.p + ob, c->probe.p, pb, hipMemcpyDeviceToDevice, c->stream));
        done0[(size_t)i] = c->sweeps_done;
    }
    auto restore = [&]() -> int {
        for (int i = 0; i < n_ctx; ++i) {
            ptyc_ctx* c = ctxs[i];
            const size_t ob = (size_t)c->cfg.h * c->cfg.w * sizeof(cf), pb = (size_t)c->cfg.n * c->cfg.n * sizeof(cf);
            HIPCHK(c, hipMemcpyAsync(c->obj.p, c->tune_save.p, ob, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->probe.p, (char*)c->tune_save.p + ob, pb, hipMemcpyDeviceToDevice, c->stream));
            c->sweeps_done = done0[(size_t)i];
            int r = refresh_probe_max(c);
            if (r != PTYC_OK) return r;
        }
        return PTYC_OK;
    };
    const int v0 = c0->multi_variant;
    std::vector<double> times((size_t)kMultiVariantCount, 0.0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    rc = he == hipSuccess ? PTYC_OK : hip_fail(c0, he, "hipEventCreate");
    for (int v = 0; v < kMultiVariantCount && rc == PTYC_OK; ++v) {
        c0->multi_variant = v;
        for (int r = 0; r < reps && rc == PTYC_OK; ++r) {
            if ((rc = restore()) != PTYC_OK) break;
            if ((he = hipEventRecord(e0, c0->stream)) != hipSuccess) { rc = hip_fail(c0, he, "hipEventRecord"); break; }
            if ((rc = ptyc_sweep_multi(ctxs, n_ctx, 1, nullptr)) != PTYC_OK) break;
            if ((he = hipEventRecord(e1, c0->stream)) != hipSuccess) { rc = hip_fail(c0, he, "hipEventRecord"); break; }
            if ((he = hipEventSynchronize(e1)) != hipSuccess) { rc = hip_fail(c0, he, "hipEventSynchronize"); break; }
            float ms = 0.f;
            if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_fail(c0, he, "hipEventElapsedTime"); break; }
            if (r == 0 || ms < times[(size_t)v]) times[(size_t)v] = ms;
        }
        if (rc == PTYC_OK && ms_out && v < PTYC_MULTI_VARIANTS) ms_out[v] = times[(size_t)v];
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    int best = v0;
    if (rc == PTYC_OK) {
        for (int v = 0; v < kMultiVariantCount; ++v)
            if (times[(size_t)v] < times[(size_t)best] * (1.0 - kTuneMargin)) best = v;
    }
    for (int i = 0; i < n_ctx; ++i)
        if (ctxs[i]->poisoned) return rc != PTYC_OK ? rc : PTYC_ERR_HIP;
    c0->multi_variant = best;
    const int rc2 = restore();
    if (rc == PTYC_OK) rc = rc2;
    if (rc == PTYC_OK) HIPCHK(c0, hipStreamSynchronize(c0->stream));
    if (variant_out) *variant_out = c0->multi_variant;
    return rc;
}

int ptyc_get_object(ptyc_ctx* c, void* out, int kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (!out || !valid_kind(kind)) return fail(c, PTYC_ERR_ARG, "bad output buffer or mem_kind");
    HIPCHK(c, hipMemcpyAsync(out, c->obj.p, (size_t)c->cfg.h * c->cfg.w * sizeof(cf), from_dev(kind), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_fault(c);
}

int ptyc_get_probe(ptyc_ctx* c, void* out, int kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (!out || !valid_kind(kind)) return fail(c, PTYC_ERR_ARG, "bad output buffer or mem_kind");
    HIPCHK(c, hipMemcpyAsync(out, c->probe.p, (size_t)c->cfg.n * c->cfg.n * sizeof(cf), from_dev(kind), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_fault(c);
}

int ptyc_set_object(ptyc_ctx* c, const void* in, int kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (!in || !valid_kind(kind)) return fail(c, PTYC_ERR_ARG, "bad input buffer or mem_kind");
    return copy_square_in(c, c->obj, in, (size_t)c->cfg.h * c->cfg.w * sizeof(cf), kind);
}

int ptyc_set_probe(ptyc_ctx* c, const void* in, int kind) {
    int rc = usable(c);
    if (rc) return rc;
    if (!in || !valid_kind(kind)) return fail(c, PTYC_ERR_ARG, "bad input buffer or mem_kind");
    if ((rc = copy_square_in(c, c->probe, in, (size_t)c->cfg.n * c->cfg.n * sizeof(cf), kind)) != PTYC_OK) return rc;
    return refresh_probe_max(c);
}

int ptyc_average(ptyc_ctx* const* ctxs, int32_t n_ctx) {
    if (!ctxs || n_ctx <= 0 || n_ctx > PTYC_MULTI_MAX) return PTYC_ERR_ARG;
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i]) return PTYC_ERR_ARG;
        int rc = usable(ctxs[i]);
        if (rc) return rc;
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) return fail(ctxs[i], PTYC_ERR_ARG, "a context appears twice");
        const ptyc_config& a = ctxs[0]->cfg;
        const ptyc_config& b = ctxs[i]->cfg;
        if (a.n != b.n || a.h != b.h || a.w != b.w)
            return fail(ctxs[i], PTYC_ERR_ARG, "all contexts must share pattern and object size");
        if (ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->device != ctxs[0]->device)
            return fail(ctxs[i], PTYC_ERR_ARG, "all contexts must share one device and stream");
    }
    ptyc_ctx* c0 = ctxs[0];
    std::vector<void*> o((size_t)n_ctx), p((size_t)n_ctx);
    for (int i = 0; i < n_ctx; ++i) {
        o[(size_t)i] = ctxs[i]->obj.p;
        p[(size_t)i] = ctxs[i]->probe.p;
    }
    HIPCHK(c0, launch_mean(o.data(), n_ctx, (int64_t)c0->cfg.h * c0->cfg.w, c0->stream));
    HIPCHK(c0, launch_mean(p.data(), n_ctx, (int64_t)c0->cfg.n * c0->cfg.n, c0->stream));
    for (int i = 0; i < n_ctx; ++i) {
        int rc = refresh_probe_max(ctxs[i]);
        if (rc) return rc;
    }
    return PTYC_OK;
}

}  // extern "C"

namespace {

// The amplitude loss (and its gradient) of a minibatch, enqueued on the
// context's stream: the forward stages over the whole minibatch in one
// launch pair (they write nothing but the exchange and the loss partials);
// for the gradient, one adjoint row launch over the whole minibatch leaves
// every position's contributions to dL/dO and dL/dP in work buffers, which
// two sums in minibatch order reduce (dL/dP over slots, dL/dO by object
// tiles, each tile over the positions whose windows cover it), so the
// result does not depend on timing.  The loss sum lands in loss_dev.
int amp_loss_enqueue(ptyc_ctx* c, const void* obj, const void* probe, const int64_t* idx, int64_t count,
                     float grad_scale, void* grad_obj, void* grad_probe, double* loss_dev) {
    if (!obj || !probe) return fail(c, PTYC_ERR_ARG, "obj and probe must not be NULL");
    if ((grad_obj == nullptr) != (grad_probe == nullptr))
        return fail(c, PTYC_ERR_ARG, "grad_obj and grad_probe must both be given or both be NULL");
    if (count < 0 || (count > 0 && !idx)) return fail(c, PTYC_ERR_ARG, "bad index list");
    // slot and tile-list indices are 32-bit on the device
    if (count > (int64_t)1 << 24) return fail(c, PTYC_ERR_ARG, "minibatch larger than 2^24 positions");
    if (!std::isfinite(grad_scale)) return fail(c, PTYC_ERR_ARG, "grad_scale must be finite");
    for (int64_t i = 0; i < count; ++i)
        if (idx[i] < 0 || idx[i] >= c->n_loaded)
            return fail(c, PTYC_ERR_ARG, "index " + std::to_string(idx[i]) + " is not a loaded position");
    int rc;
    const bool grad = grad_obj != nullptr;
    const int n = c->cfg.n;
    const int64_t h = c->cfg.h, w = c->cfg.w;
    const size_t nn = (size_t)n * n;
    if (grad && count == 0) HIPCHK(c, launch_fill_zero(grad_probe, (int64_t)nn, c->stream));
    // dL/dO by object tiles: for every tile of the object, the slots whose
    // windows cover it in ascending order (compressed rows: tile_off, tile_slot)
    const int tiles_y = (int)((h + kGradTR - 1) / kGradTR), tiles_x = (int)((w + kGradTC - 1) / kGradTC);
    const size_t n_tiles = (size_t)tiles_y * tiles_x;
    std::vector<int32_t> tile_off, tile_slot;
    if (grad) {
        auto span = [&](int64_t i, int& ty0, int& ty1, int& tx0, int& tx1) {
            const int32_t row = c->h_pos[(size_t)(2 * idx[i])], col = c->h_pos[(size_t)(2 * idx[i] + 1)];
            ty0 = row / kGradTR;
            ty1 = (row + n - 1) / kGradTR;
            tx0 = col / kGradTC;
            tx1 = (col + n - 1) / kGradTC;
        };
        tile_off.assign(n_tiles + 1, 0);
        for (int64_t i = 0; i < count; ++i) {
            int ty0, ty1, tx0, tx1;
            span(i, ty0, ty1, tx0, tx1);
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) ++tile_off[(size_t)ty * tiles_x + tx + 1];
        }
        for (size_t t = 0; t < n_tiles; ++t) tile_off[t + 1] += tile_off[t];
        std::vector<int32_t> fill(tile_off.begin(), tile_off.end() - 1);
        tile_slot.resize((size_t)tile_off.back());
        for (int64_t i = 0; i < count; ++i) {
            int ty0, ty1, tx0, tx1;
            span(i, ty0, ty1, tx0, tx1);
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) tile_slot[(size_t)fill[(size_t)ty * tiles_x + tx]++] = (int32_t)i;
        }
    }
    const int64_t slots = std::max<int64_t>(count, 1);
    if (slots > c->slots) {
        if ((rc = ensure(c, c->scratch, (size_t)slots * nn * sizeof(cf))) != PTYC_OK) return rc;
        if ((rc = ensure(c, c->winmax, (size_t)slots * max_row_blocks(c) * sizeof(float))) != PTYC_OK) return rc;
        c->slots = slots;
    }
    const int64_t parts = (count + kAdjGroup - 1) / kAdjGroup;   // partial sums of dL/dP
    if (grad && count > 0 && (rc = ensure(c, c->gpart, (size_t)parts * nn * sizeof(cf))) != PTYC_OK) return rc;
    // one upload: the order entries, then the tile lists
    const size_t obytes = (size_t)count * sizeof(OrderEntry);
    const size_t tbytes = (tile_off.size() + tile_slot.size()) * sizeof(int32_t);
    const size_t ubytes = obytes + tbytes;
    if ((rc = ensure(c, c->order, std::max<size_t>(ubytes, sizeof(OrderEntry)))) != PTYC_OK) return rc;
    if ((rc = ensure(c, c->err_part, (size_t)slots * c->sb.col_blocks * sizeof(double))) != PTYC_OK) return rc;
    const int32_t* d_tile_off = (const int32_t*)((const char*)c->order.p + obytes);
    const int32_t* d_tile_slot = d_tile_off + tile_off.size();
    if (ubytes > 0) {
        // this call's pinned buffer may still feed the copy made kLossRing calls ago
        ptyc_ctx::PinSlot& ps = c->lpin[c->lring];
        c->lring = (c->lring + 1) % ptyc_ctx::kLossRing;
        if (ps.pending) {
            HIPCHK(c, hipEventSynchronize(ps.done));
            ps.pending = false;
        }
        if (!ps.done) HIPCHK(c, hipEventCreateWithFlags(&ps.done, hipEventDisableTiming));
        if (ps.bytes < ubytes) {
            if (ps.p) (void)hipHostFree(ps.p);
            ps.p = nullptr;
            ps.bytes = 0;
            hipError_t e = hipHostMalloc(&ps.p, ubytes, hipHostMallocDefault);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(c, PTYC_ERR_OOM, "pinned host allocation failed");
            }
            ps.bytes = ubytes;
        }
        to_entries(c, idx, count, (OrderEntry*)ps.p);
        int32_t* pt = (int32_t*)((char*)ps.p + obytes);
        std::copy(tile_off.begin(), tile_off.end(), pt);
        std::copy(tile_slot.begin(), tile_slot.end(), pt + tile_off.size());
        HIPCHK(c, hipMemcpyAsync(c->order.p, ps.p, ubytes, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipEventRecord(ps.done, c->stream));
        ps.pending = true;
    }
    BatchArgs a = base_args(c);
    a.obj = (cf*)obj;
    a.probe = (cf*)probe;
    a.gscale = grad_scale;
    a.off = 0;
    a.bsize = (int)count;
    HIPCHK(c, launch_loss_fwd(n, a, grad, c->stream));
    if (!grad) {
        HIPCHK(c, launch_sum_reduce((const double*)c->err_part.p, count * c->sb.col_blocks, loss_dev, c->stream));
        return PTYC_OK;
    }
    if (count > 0) HIPCHK(c, launch_adjoint_rows(n, a, c->gpart.p, c->stream));
    // dL/dO, dL/dP and the loss sum in one launch
    GradFinish f{};
    f.co = (const cf*)c->scratch.p;
    f.order = (const OrderEntry*)c->order.p;
    f.n = n;
    f.h = h;
    f.w = w;
    f.tile_off = d_tile_off;
    f.tile_slot = d_tile_slot;
    f.gobj = (cf*)grad_obj;
    f.part = (const cf*)c->gpart.p;
    f.nn = count > 0 ? (int64_t)nn : 0;   // an empty minibatch: dL/dP was cleared above
    f.parts = (int)parts;
    f.gprobe = (cf*)grad_probe;
    f.loss_part = (const double*)c->err_part.p;
    f.n_loss_part = count * c->sb.col_blocks;
    f.loss = loss_dev;
    HIPCHK(c, launch_grad_finish(f, c->stream));
    return PTYC_OK;
}

}  // namespace

extern "C" {

int ptyc_amp_loss(ptyc_ctx* c, const void* obj, const void* probe, const int64_t* idx, int64_t count,
                  float grad_scale, void* grad_obj, void* grad_probe, double* loss_out) {
    int rc = usable(c);
    if (rc) return rc;
    if (!loss_out) return fail(c, PTYC_ERR_ARG, "loss_out must not be NULL");
    if ((rc = ensure(c, c->err_dev, sizeof(double))) != PTYC_OK) return rc;
    if ((rc = amp_loss_enqueue(c, obj, probe, idx, count, grad_scale, grad_obj, grad_probe,
                               (double*)c->err_dev.p)) != PTYC_OK)
        return rc;
    HIPCHK(c, hipMemcpyAsync(loss_out, c->err_dev.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PTYC_OK;
}

int ptyc_amp_loss_async(ptyc_ctx* c, const void* obj, const void* probe, const int64_t* idx, int64_t count,
                        void* grad_obj, void* grad_probe, double* loss_dev) {
    int rc = usable(c);
    if (rc) return rc;
    if (!loss_dev) return fail(c, PTYC_ERR_ARG, "loss_dev must not be NULL");
    return amp_loss_enqueue(c, obj, probe, idx, count, 1.0f, grad_obj, grad_probe, loss_dev);
}

int ptyc_scale_c64(ptyc_ctx* c, void* data, int64_t count, const double* scale_dev) {
    int rc = usable(c);
    if (rc) return rc;
    if (count < 0 || (count > 0 && (!data || !scale_dev))) return fail(c, PTYC_ERR_ARG, "bad buffer or count");
    HIPCHK(c, launch_scale(data, count, scale_dev, c->stream));
    return PTYC_OK;
}

int ptyc_colour(int64_t count, const int32_t* pos_yx, int32_t n, int32_t max_batch, int32_t* colour_out,
                int32_t* n_colours) {
    if (count < 0 || n <= 0 || max_batch < 0 || (count > 0 && (!pos_yx || !colour_out)) || !n_colours)
        return PTYC_ERR_ARG;
    for (int64_t i = 0; i < 2 * count; ++i)
        if (pos_yx[i] < 0) return PTYC_ERR_BOUNDS;
    Colouring col(n, max_batch > 0 ? max_batch : 1024);
    col.extend(pos_yx, 0, count);
    for (int64_t i = 0; i < count; ++i) colour_out[i] = col.colour()[(size_t)i];
    *n_colours = (int32_t)col.members().size();
    return PTYC_OK;
}

int ptyc_check_batches(int64_t count, const int32_t* pos_yx, int32_t n, const int64_t* order, int64_t order_len,
                       const int64_t* off, int64_t n_batches) {
    if (count < 0 || n <= 0 || order_len < 0 || n_batches < 0 || !off || (order_len > 0 && !order) ||
        (count > 0 && !pos_yx))
        return PTYC_ERR_ARG;
    std::string why;
    return check_batches(count, pos_yx, n, order, order_len, off, n_batches, &why) ? PTYC_OK : PTYC_ERR_ARG;
}

}  // extern "C"
