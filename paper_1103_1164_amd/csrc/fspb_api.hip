// fspb_api.hip -- host side of libfspb: the C ABI of include/fspb.h.
//
// Responsibilities: argument validation (pure host, before any HIP call),
// device buffers owned by the geometry handle, packing of the commissioned
// tables into the layouts the kernels read, and kernel launches.  All of the
// method's per-voxel and per-beamlet arithmetic runs in the kernels.
#include "fspb.h"
#include "gamma.h"
#include "kernels.h"
#include "mlp.h"

#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <deque>
#include <functional>
#include <cmath>
#include <map>
#include <new>
#include <mutex>
#include <string>
#include <vector>

using namespace fspb;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(FSPB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// Device memory comes from a per-device caching pool: blocks freed by
// fspb_destroy are kept (by size class) and handed to the next geometry, so a
// stream of plans does not pay hipMalloc/hipFree on every create.  Sizes are
// rounded up to classes at most 1/8 above the request.  A destroyed handle's
// blocks rejoin the pool when an event recorded after its last queued work
// has completed (pending releases are bounded; see fspb_destroy).
struct Deferred {
    int device;
    std::vector<hipEvent_t> evs;                    // one per stream the handle used
    std::vector<std::pair<void*, size_t>> blocks;   // (pointer, class)
};
struct Pool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void*>> free_blocks;  // (device, class) -> blocks
    size_t cached = 0;
    std::deque<Deferred> deferred;   // oldest first
};

Pool& pool() {
    static Pool* p = new Pool();  // never destroyed: blocks may be returned during exit
    return *p;
}

size_t size_class(size_t bytes) {
    if (bytes <= 4096) return 4096;
    size_t top = (size_t)1 << (63 - __builtin_clzll(bytes));
    size_t q = std::max<size_t>(top / 8, 4096);
    return (bytes + q - 1) / q * q;
}

// Moves the blocks of completed releases into the free lists; while more than
// `limit` releases are pending, waits for the oldest.  Caller holds pool().mu.
void reap_locked(size_t limit) {
    auto& d = pool().deferred;
    while (!d.empty()) {
        Deferred& x = d.front();
        bool done = true;
        for (hipEvent_t ev : x.evs)
            if (hipEventQuery(ev) == hipErrorNotReady) done = false;
        if (!done) {
            if (d.size() <= limit) break;
            for (hipEvent_t ev : x.evs) (void)hipEventSynchronize(ev);
        }
        (void)hipGetLastError();
        for (auto& b : x.blocks) {
            pool().free_blocks[{x.device, b.second}].push_back(b.first);
            pool().cached += b.second;
        }
        for (hipEvent_t ev : x.evs) (void)hipEventDestroy(ev);
        d.pop_front();
    }
}

// Test hook: FSPB_TEST_FAIL_ALLOC=n makes the n-th device allocation after the
// variable was set (or changed) fail, to exercise the out-of-memory paths.
int g_alloc_count = 0;
std::string g_alloc_env;

int pool_alloc(int dev, void** p, size_t bytes, size_t* cls_out) {
    *p = nullptr;
    const char* inj = getenv("FSPB_TEST_FAIL_ALLOC");
    {
        std::lock_guard<std::mutex> lk(pool().mu);
        std::string cur = inj ? inj : "";
        if (cur != g_alloc_env) {
            g_alloc_env = cur;
            g_alloc_count = 0;
        }
        ++g_alloc_count;
        if (inj && atoi(inj) == g_alloc_count)
            return fail(FSPB_E_NOMEM, "device allocation of %zu bytes failed (injected)", bytes);
    }
    const size_t cls = size_class(bytes);
    *cls_out = cls;
    {
        std::lock_guard<std::mutex> lk(pool().mu);
        reap_locked((size_t)-1);
        auto it = pool().free_blocks.find({dev, cls});
        if (it != pool().free_blocks.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            pool().cached -= cls;
            return FSPB_OK;
        }
    }
    hipError_t e = hipMalloc(p, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give the cached blocks back to the runtime and try once more
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> lk(pool().mu);
            for (auto& kv : pool().free_blocks)
                if (kv.first.first == dev) {
                    drop.insert(drop.end(), kv.second.begin(), kv.second.end());
                    kv.second.clear();
                }
        }
        for (void* q : drop) (void)hipFree(q);
        e = hipMalloc(p, cls);
        if (e != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return fail(FSPB_E_NOMEM, "hipMalloc of %zu bytes failed: %s", cls, hipGetErrorString(e));
        }
    }
    return FSPB_OK;
}

void pool_free(int dev, void* p, size_t cls) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(pool().mu);
    pool().free_blocks[{dev, cls}].push_back(p);
    pool().cached += cls;
}

bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }

int check_table(const fspb_table1d& t, const char* name) {
    if (t.n < 1 || !t.v) return fail(FSPB_E_ARG, "table %s: needs n >= 1 and values", name);
    if (!isfinite(t.start) || (t.n > 1 && !finite_pos(t.step)))
        return fail(FSPB_E_ARG, "table %s: start must be finite and step > 0", name);
    return FSPB_OK;
}

}  // namespace

// Packed commissioned tables (water, A and density tables in the layouts the
// kernels read), shared by every geometry built from bitwise-identical tables
// on a device.  Sets stay while a geometry uses them; unused ones are kept
// (up to kMaxIdleTableSets per process) for the next plan, and
// fspb_release_cached_memory frees them.
struct TableSet {
    int device = 0;
    std::vector<uint32_t> key;   // every table parameter and value, bitwise
    float4* dtab = nullptr;
    float4* atab = nullptr;
    float* denstab = nullptr;
    DensTabs dens{};
    float w2c = 1.0f;            // b2 = w2c b1 at every sample when w2_one
    int w2_one = 0;
    int refs = 0;
    unsigned long long last_use = 0;
};

namespace {
constexpr int kMaxIdleTableSets = 8;
std::mutex g_tables_mu;
unsigned long long g_tables_clock = 0;
std::vector<TableSet*>& table_sets() {
    static auto* v = new std::vector<TableSet*>();   // never destroyed
    return *v;
}
void free_table_set(TableSet* t) {
    (void)hipFree(t->dtab);
    (void)hipFree(t->atab);
    (void)hipFree(t->denstab);
    delete t;
}
}  // namespace

struct fspb_geometry {
    int device = 0;
    PlanConst P{};
    DensTabs dens{};
    int n_beams = 0, n_beamlets = 0, k_stride = 0;
    int dc_created = 0, dc_enabled = 0;
    int smooth_r[3] = {0, 0, 0};
    float sample_step = 0.0f;
    size_t device_bytes = 0;
    // device buffers
    float* rhohat = nullptr;
    float4* fac = nullptr;
    BeamDesc* beams = nullptr;
    BeamIn* beam_in = nullptr;
    Frame64* frames = nullptr;
    BeamletDesc* desc = nullptr;
    TraceInfo* tinfo = nullptr;
    float4* dtab = nullptr;
    float4* atab = nullptr;
    float* denstab = nullptr;
    float2* tT = nullptr;
    float4* tTW = nullptr;    // DC only: depth + first weight-drift table (16-byte entries)
    float2* tW2 = nullptr;    // DC only: second weight-drift table (8-byte entries, same index)
    float4* sid = nullptr;    // exact (Siddon) depth tables, when the plan asks for them
    int siddon = 0, sid_stride = 0;
    float* w3 = nullptr;
    int* counts = nullptr;
    int* order = nullptr;      // bricks in decreasing order of estimated work
    int* cost = nullptr;       // estimated work per brick (candidate beamlets)
    float* adj_part = nullptr; // the adjoint's per-(slab, beamlet) partial sums
    unsigned* surr_live = nullptr;   // the surrogate's listed rows (allocated on first use)
    unsigned* surr_count = nullptr;
    float4* surr_quad = nullptr;     // the CT's 2x2 neighbourhoods, per call
    int adj_slab = 0;          // the adjoint's slab thickness (0: adjoint_slab(P))
    int* adj_queue = nullptr;  // the adjoint's per-XCD unit counters
    // per-beam schedule (allocated on first use): sorted items, XCD runs,
    // their scratch, and the per-beam partial doses [n_beams][stride]
    SplitSched split{};
    float* planes = nullptr;
    float* tmp0 = nullptr;     // smoothing intermediates (alias the depth tables when they fit)
    float* tmp1 = nullptr;
    float* rho = nullptr;      // the handle's copy of the CT it was created from
    // creation work is asynchronous: `ready` is recorded on `ready_stream`
    // after it; first use on another stream (or from the host) waits for it
    hipEvent_t ready = nullptr;
    hipStream_t ready_stream = nullptr;
    bool pending = false;
    // the streams of the handle's queued work (release waits for each); more
    // than kMaxHandleStreams, or work captured into a graph, make
    // fspb_destroy wait for the whole device
    std::vector<hipStream_t> streams;
    bool many_streams = false;
    TileCfg tile;
    std::vector<int> h_cost;   // host copy of cost (fetched when a batch needs it)
    bool h_cost_valid = false;
    TraceGrid tg{};
    TraceParams tp{};
    int n_cu = 0;              // the device's compute units
    unsigned long long* partial = nullptr;
    unsigned long long* total = nullptr;
    // host copies
    std::vector<BeamletDesc> h_desc;
    std::vector<Frame64> h_frames;
    std::vector<TraceInfo> h_info;
    int k_max = 0, n_hit = 0, n_amb = 0;
    bool host_ready = false;               // host copies are fetched on first use
    std::vector<std::pair<void*, size_t>> blocks;   // pool blocks owned by the handle

    int alloc(void** p, size_t bytes) {
        size_t cls = 0;
        int rc = pool_alloc(device, p, bytes, &cls);
        if (rc == FSPB_OK) {
            blocks.push_back({*p, cls});
            device_bytes += cls;
        }
        return rc;
    }

    DoseArgs args() const {
        DoseArgs a;
        a.P = P;
        a.P.dc = dc_enabled;
        a.beams = beams;
        a.bl = desc;
        a.fac = fac;
        a.dtab = dtab;
        a.atab = atab;
        a.tT = tT;
        a.tTW = tTW;
        a.tW2 = tW2;
        a.sid = sid;
        return a;
    }

    TableSet* tabs = nullptr;      // shared commissioned tables (not owned)

    void release() {
        if (ready) (void)hipEventDestroy(ready);
        ready = nullptr;
        pending = false;
        for (auto& b : blocks) pool_free(device, b.first, b.second);
        blocks.clear();
        if (tabs) {
            std::lock_guard<std::mutex> lk(g_tables_mu);
            --tabs->refs;
            tabs = nullptr;
        }
    }

    int fetch_host() const;
};

namespace {

int validate(const fspb_ct* ct, int n_beams, const fspb_beam* beams, const fspb_tables* t,
             const fspb_options* o) {
    if (!ct || !beams || !t) return fail(FSPB_E_ARG, "ct, beams and tables must be non-NULL");
    if (ct->nx < 1 || ct->ny < 1 || ct->nz < 1)
        return fail(FSPB_E_ARG, "grid size %dx%dx%d must be positive", ct->nx, ct->ny, ct->nz);
    if (!finite_pos(ct->dx) || !finite_pos(ct->dy) || !finite_pos(ct->dz))
        return fail(FSPB_E_ARG, "voxel sizes must be positive");
    if (!isfinite(ct->ox) || !isfinite(ct->oy) || !isfinite(ct->oz))
        return fail(FSPB_E_ARG, "grid origin must be finite");
    if (!ct->density) return fail(FSPB_E_ARG, "ct->density is NULL");
    long long nv = (long long)ct->nx * ct->ny * ct->nz;
    if (nv > (1LL << 31) - 1) return fail(FSPB_E_ARG, "grid of %lld voxels exceeds 2^31-1", nv);
    if (n_beams < 1) return fail(FSPB_E_ARG, "n_beams must be >= 1");
    long long nbl = 0;
    for (int b = 0; b < n_beams; ++b) {
        const fspb_beam& B = beams[b];
        if (B.nbx < 1 || B.nby < 1) return fail(FSPB_E_ARG, "beam %d: empty beamlet grid", b);
        if (!finite_pos(B.wx) || !finite_pos(B.wy) || !finite_pos(B.sad))
            return fail(FSPB_E_ARG, "beam %d: beamlet widths and SAD must be positive", b);
        if (!isfinite(B.gantry) || !isfinite(B.couch) || !isfinite(B.cx) || !isfinite(B.cy) ||
            !isfinite(B.iso[0]) || !isfinite(B.iso[1]) || !isfinite(B.iso[2]))
            return fail(FSPB_E_ARG, "beam %d: angles, offsets and isocentre must be finite", b);
        nbl += (long long)B.nbx * B.nby;
    }
    if (nbl > (1 << 24)) return fail(FSPB_E_ARG, "too many beamlets (%lld)", nbl);
    const fspb_table1d* all[] = {&t->A, &t->u1x, &t->u1y, &t->u2x, &t->u2y, &t->w1, &t->w2,
                                 &t->fu1, &t->fu2, &t->fw1, &t->fw2, &t->b1, &t->b2};
    const char* names[] = {"A", "u1x", "u1y", "u2x", "u2y", "w1", "w2",
                           "fu1", "fu2", "fw1", "fw2", "b1", "b2"};
    for (int q = 0; q < 13; ++q) {
        int rc = check_table(*all[q], names[q]);
        if (rc) return rc;
    }
    if (t->n_theta < 1 || (t->n_theta > 1 && !finite_pos(t->theta_step)))
        return fail(FSPB_E_ARG, "A table: n_theta >= 1 and theta_step > 0 required");
    const fspb_table1d* dts[] = {&t->u1y, &t->u2x, &t->u2y, &t->w1, &t->w2};
    for (const fspb_table1d* d : dts)
        if (d->start != t->u1x.start || d->n != t->u1x.n || (d->n > 1 && d->step != t->u1x.step))
            return fail(FSPB_E_ARG, "the water tables u1x..w2 must share one depth grid");
    if (o) {
        if (o->flags & ~FSPB_FLAG_SIDDON) return fail(FSPB_E_ARG, "options.flags: unknown bits");
        if (o->dc_enabled != 0 && o->dc_enabled != 1)
            return fail(FSPB_E_ARG, "options.dc_enabled must be 0 or 1");
        if (o->roi_radius < 0 || o->smooth_sigma < 0 || o->sample_step < 0 ||
            !isfinite(o->roi_radius) || !isfinite(o->smooth_sigma) || !isfinite(o->sample_step) ||
            !isfinite(o->rho_surface) || !isfinite(o->rho_min) || !isfinite(o->rho_max))
            return fail(FSPB_E_ARG, "options must be finite and non-negative");
        if ((o->rho_min != 0 || o->rho_max != 0) && !(o->rho_min < o->rho_max))
            return fail(FSPB_E_ARG, "options: rho_min must be below rho_max");
        if (o->schedule != 0 && o->schedule != 1)
            return fail(FSPB_E_ARG, "options.schedule must be 0 or 1");
        if (o->schedule == 1 && (o->flags & FSPB_FLAG_SIDDON))
            return fail(FSPB_E_ARG, "options.schedule 1 is not available with exact depth tables");
        if (o->tile_waves != 0) {
            if (o->tile_shape < 0 || o->tile_shape >= kNumShapes)
                return fail(FSPB_E_ARG, "options.tile_shape %d out of range", o->tile_shape);
            if (o->tile_waves != 1 && o->tile_waves != 2 && o->tile_waves != 4 &&
                o->tile_waves != kLdsWaves)
                return fail(FSPB_E_ARG, "options.tile_waves must be 0, 1, 2, 4 or 8");
        }
    }
    // every voxel must lie in front of every source (positive depth along the
    // central axis), so that the isocentre-plane projection is defined
    double lo[3] = {ct->ox - 0.5 * ct->dx, ct->oy - 0.5 * ct->dy, ct->oz - 0.5 * ct->dz};
    double hi[3] = {ct->ox + (ct->nx - 0.5) * ct->dx, ct->oy + (ct->ny - 0.5) * ct->dy,
                    ct->oz + (ct->nz - 0.5) * ct->dz};
    for (int b = 0; b < n_beams; ++b) {
        const fspb_beam& B = beams[b];
        double phi = B.gantry, psi = B.couch;
        double c0[3] = {-sin(phi), cos(phi), 0.0};
        double cax[3] = {cos(psi) * c0[0] + sin(psi) * c0[2], c0[1], -sin(psi) * c0[0] + cos(psi) * c0[2]};
        double src[3];
        for (int q = 0; q < 3; ++q) src[q] = B.iso[q] - (double)B.sad * cax[q];
        for (int c = 0; c < 8; ++c) {
            double p[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
            double z = (p[0] - src[0]) * cax[0] + (p[1] - src[1]) * cax[1] + (p[2] - src[2]) * cax[2];
            if (!(z > 1e-3))
                return fail(FSPB_E_ARG, "beam %d: the grid must lie entirely in front of the source", b);
        }
    }
    return FSPB_OK;
}

int check_device(int* dev) {
    // the architecture of each device is looked up once (the property query
    // is slow compared with creating a plan)
    constexpr int kMaxDevices = 64;
    static std::atomic<int> arch_ok[kMaxDevices];   // 0 unknown, 1 gfx950, -1 other
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return fail(FSPB_E_UNSUPPORTED, "no HIP device available");
    }
    HIP_TRY(hipGetDevice(dev));
    const int v = (*dev >= 0 && *dev < kMaxDevices) ? arch_ok[*dev].load() : 0;
    if (v == 1) return FSPB_OK;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, *dev));
    const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (*dev >= 0 && *dev < kMaxDevices) arch_ok[*dev].store(ok ? 1 : -1);
    if (!ok)
        return fail(FSPB_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", *dev,
                    prop.gcnArchName);
    return FSPB_OK;
}

}  // namespace

// Waits (on the host) for the handle's creation work.
static int settle_host(fspb_geometry* g) {
    if (!g->pending) return FSPB_OK;
    if (hipEventQuery(g->ready) != hipSuccess) HIP_TRY(hipEventSynchronize(g->ready));
    g->pending = false;
    return FSPB_OK;
}

constexpr size_t kMaxHandleStreams = 4;

static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return st != hipStreamCaptureStatusNone;
}

// Notes a stream the handle's work goes to; returns whether s is capturing.
static bool note_stream(fspb_geometry* g, hipStream_t s) {
    const bool cap = capturing(s);
    if (cap) g->many_streams = true;
    if (std::find(g->streams.begin(), g->streams.end(), s) == g->streams.end()) {
        if (g->streams.size() < kMaxHandleStreams) g->streams.push_back(s);
        else g->many_streams = true;
    }
    return cap;
}

// Orders work on stream s after the handle's creation work: on the creation
// stream that order holds already; another stream waits for the ready event
// on the device (or, while capturing a graph, on the host).
static int settle(fspb_geometry* g, hipStream_t s) {
    const bool cap = note_stream(g, s);
    if (!g->pending || s == g->ready_stream) return FSPB_OK;
    if (hipEventQuery(g->ready) == hipSuccess) {
        g->pending = false;
        return FSPB_OK;
    }
    (void)hipGetLastError();
    if (cap) return settle_host(g);
    HIP_TRY(hipStreamWaitEvent(s, g->ready, 0));
    return FSPB_OK;
}

int fspb_geometry::fetch_host() const {
    fspb_geometry* G = const_cast<fspb_geometry*>(this);
    if (G->host_ready) return FSPB_OK;
    if (int rc = settle_host(G)) return rc;
    const int nbl = n_beamlets;
    G->h_desc.resize(nbl);
    G->h_frames.resize(nbl);
    G->h_info.resize(nbl);
    HIP_TRY(hipMemcpy(G->h_desc.data(), desc, sizeof(BeamletDesc) * nbl, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(G->h_frames.data(), frames, sizeof(Frame64) * nbl, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(G->h_info.data(), tinfo, sizeof(TraceInfo) * nbl, hipMemcpyDeviceToHost));
    G->n_hit = G->k_max = G->n_amb = 0;
    for (int i = 0; i < nbl; ++i) {
        if (G->h_desc[i].hit) ++G->n_hit;
        G->k_max = std::max(G->k_max, G->h_desc[i].K);
        if (G->h_info[i].k_entry >= 0 && G->h_info[i].margin <= 1e-9) ++G->n_amb;
    }
    G->host_ready = true;
    return FSPB_OK;
}

extern "C" {

const char* fspb_error_string(int code) {
    switch (code) {
        case FSPB_OK: return "success";
        case FSPB_E_ARG: return "invalid argument";
        case FSPB_E_HIP: return "HIP runtime error";
        case FSPB_E_NOMEM: return "out of memory";
        case FSPB_E_STATE: return "invalid state for this handle";
        case FSPB_E_UNSUPPORTED: return "unsupported device";
        default: return "unknown error";
    }
}

const char* fspb_last_error(void) { return g_last_error.c_str(); }

// Brick schedule for the handle's tile shape: estimated work per brick
// (candidate beamlets), longest first, built on the device (asynchronous).
static int build_order(fspb_geometry* G, hipStream_t s) {
    const long nb = brick_count(G->P, G->tile.shape);
    launch_brick_cost(G->args(), G->tile, G->cost, s);
    launch_order_bricks(G->cost, nb, G->order, s);
    HIP_TRY(hipGetLastError());
    G->h_cost_valid = false;
    if (G->tile.per_beam) {
        // buffers for the largest item count of any shape, allocated once
        if (!G->planes) {
            long max_items = 0;
            for (int sh = 0; sh < kNumShapes; ++sh)
                max_items = std::max(max_items, brick_count(G->P, sh) * G->P.n_beams);
            const long nv = (long)G->P.nx * G->P.ny * G->P.nz;
            const long stride = (nv + 63) / 64 * 64;
            int rc;
            if ((rc = G->alloc((void**)&G->split.order, sizeof(int) * max_items)) != FSPB_OK ||
                (rc = G->alloc((void**)&G->split.cost, sizeof(int) * max_items)) != FSPB_OK ||
                (rc = G->alloc((void**)&G->split.key, sizeof(int) * max_items)) != FSPB_OK ||
                (rc = G->alloc((void**)&G->split.chunk, sizeof(int) * (8 * kSplitSegments + 1))) != FSPB_OK ||
                (rc = G->alloc((void**)&G->split.hist_n, sizeof(int) * 64 * kSplitKeys)) != FSPB_OK ||
                (rc = G->alloc((void**)&G->split.hist_w, sizeof(unsigned int) * 64 * kSplitKeys)) != FSPB_OK ||
                (rc = G->alloc((void**)&G->planes, sizeof(float) * stride * G->P.n_beams)) != FSPB_OK)
                return rc;
        }
        launch_split_schedule(G->args(), G->tile, G->split, s);
        HIP_TRY(hipGetLastError());
    }
    return FSPB_OK;
}

// Host copy of the brick costs for the batch scheduler (synchronises s).
static int fetch_cost(fspb_geometry* G, hipStream_t s) {
    if (G->h_cost_valid) return FSPB_OK;
    const long nb = brick_count(G->P, G->tile.shape);
    G->h_cost.assign(nb, 0);
    HIP_TRY(hipMemcpyAsync(G->h_cost.data(), G->cost, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    G->h_cost_valid = true;
    return FSPB_OK;
}

// Packs the commissioned tables into the kernels' layouts (once per
// distinct set and device):
//   dtab[j], dtab[n + j], dtab[2n + j] (n samples): (u1x, u1y, u2x, u2y) log2 e
//                   at depth sample j, their slopes to sample j+1, and
//                   (w1, w2, w1', w2') -- three planes, 16-byte stride
//   atab[r n_A + j]: (a, b, c, e) / 4 with a = A[r][j], b = A[r+1][j] - a,
//                   c = A[r][j+1] - a, e = A[r+1][j+1] - A[r+1][j] - c, for
//                   theta rows r < a_cols and depth samples j < n_A; the 1/4
//                   is the product of the two factors 1/2 of Eq. 4's profiles
//   denstab: the six density tables back to back (offsets in dens)
// The key of a table set: every parameter and value, bitwise, in a fixed
// order.  A lookup compares the cached keys with the tables in place; the
// key is only built for a new set.
static void table_key_walk(const fspb_tables* t,
                           const std::function<bool(const void*, size_t)>& part) {
    auto put_tab = [&](const fspb_table1d& tb, size_t count) {
        const uint32_t n = (uint32_t)tb.n;
        return part(&n, 4) && part(&tb.start, 4) && part(&tb.step, 4) &&
               part(tb.v, sizeof(float) * count);
    };
    const uint32_t nth = (uint32_t)t->n_theta;
    if (!part(&nth, 4) || !part(&t->theta_step, 4)) return;
    if (!put_tab(t->A, (size_t)t->n_theta * t->A.n)) return;
    const fspb_table1d* all[12] = {&t->u1x, &t->u1y, &t->u2x, &t->u2y, &t->w1, &t->w2,
                                   &t->fu1, &t->fu2, &t->fw1, &t->fw2, &t->b1, &t->b2};
    for (const fspb_table1d* tb : all)
        if (!put_tab(*tb, (size_t)tb->n)) return;
}

static bool table_key_equals(const std::vector<uint32_t>& key, const fspb_tables* t) {
    size_t pos = 0;
    bool eq = true;
    table_key_walk(t, [&](const void* p, size_t bytes) {
        const size_t words = bytes / 4;
        eq = pos + words <= key.size() && memcmp(key.data() + pos, p, bytes) == 0;
        pos += words;
        return eq;
    });
    return eq && pos == key.size();
}

// True when b2 = c b1 at every sample of one density grid (Section 2.1 uses
// a single b for both weight components: c = 1).  c is the ratio at the
// largest |b1|, and every sample must then satisfy c b1 == b2 exactly in
// FP32; b1 = b2 = 0 gives c = 1.
static bool drift_proportional(const fspb_table1d& b1, const fspb_table1d& b2, float* c) {
    if (b1.n != b2.n || b1.start != b2.start || (b1.n > 1 && b1.step != b2.step)) return false;
    int k0 = -1;
    for (int k = 0; k < b1.n; ++k)
        if (b1.v[k] != 0.0f && (k0 < 0 || std::fabs(b1.v[k]) > std::fabs(b1.v[k0]))) k0 = k;
    const float cc = k0 >= 0 ? b2.v[k0] / b1.v[k0] : 1.0f;
    if (!std::isfinite(cc)) return false;
    for (int k = 0; k < b1.n; ++k)
        if (!(cc * b1.v[k] == b2.v[k])) return false;
    *c = cc;
    return true;
}

static int acquire_tables(int dev, const fspb_tables* t, int a_cols, TableSet** out) {
    std::lock_guard<std::mutex> lk(g_tables_mu);
    auto& sets = table_sets();
    for (TableSet* ts : sets)
        if (ts->device == dev && table_key_equals(ts->key, t)) {
            ++ts->refs;
            ts->last_use = ++g_tables_clock;
            *out = ts;
            return FSPB_OK;
        }
    std::vector<uint32_t> key;
    table_key_walk(t, [&](const void* p, size_t bytes) {
        const size_t k0 = key.size();
        key.resize(k0 + bytes / 4);
        memcpy(key.data() + k0, p, bytes);
        return true;
    });

    const int dn = t->u1x.n;
    std::vector<float4> dtab(3 * (size_t)dn);
    const fspb_table1d* U[4] = {&t->u1x, &t->u1y, &t->u2x, &t->u2y};
    auto at = [](const fspb_table1d& tb, int i) { return (double)tb.v[std::min(i, tb.n - 1)]; };
    for (int j = 0; j < dn; ++j) {
        float u[4], du[4];
        for (int q = 0; q < 4; ++q) {
            u[q] = (float)(at(*U[q], j) * 1.4426950408889634);
            du[q] = (float)((at(*U[q], j + 1) - at(*U[q], j)) * 1.4426950408889634);
        }
        dtab[j] = make_float4(u[0], u[1], u[2], u[3]);
        dtab[dn + j] = make_float4(du[0], du[1], du[2], du[3]);
        dtab[2 * dn + j] = make_float4(t->w1.v[j], t->w2.v[j], (float)(at(t->w1, j + 1) - at(t->w1, j)),
                                      (float)(at(t->w2, j + 1) - at(t->w2, j)));
    }
    const int an = t->A.n, nth = t->n_theta, ac = a_cols;
    std::vector<float4> atab((size_t)an * ac);
    auto A = [&](int r, int j) {
        return (double)t->A.v[(size_t)std::min(r, nth - 1) * an + std::min(j, an - 1)];
    };
    // each entry is formed in FP64 and rounded to FP32 once
    for (int r = 0; r < ac; ++r)
        for (int j = 0; j < an; ++j)
            atab[(size_t)r * an + j] = make_float4(
                (float)(0.25 * A(r, j)), (float)(0.25 * (A(r + 1, j) - A(r, j))),
                (float)(0.25 * (A(r, j + 1) - A(r, j))),
                (float)(0.25 * ((A(r + 1, j + 1) - A(r + 1, j)) - (A(r, j + 1) - A(r, j)))));
    TableSet* ts = new (std::nothrow) TableSet();
    if (!ts) return fail(FSPB_E_NOMEM, "host allocation failed");
    ts->device = dev;
    const fspb_table1d* D[6] = {&t->fu1, &t->fu2, &t->fw1, &t->fw2, &t->b1, &t->b2};
    DTab* DT[6] = {&ts->dens.fu1, &ts->dens.fu2, &ts->dens.fw1, &ts->dens.fw2, &ts->dens.b1,
                   &ts->dens.b2};
    std::vector<float> dens;
    for (int q = 0; q < 6; ++q) {
        DT[q]->start = D[q]->start;
        DT[q]->step = D[q]->n > 1 ? D[q]->step : 1.0f;
        DT[q]->inv_step = D[q]->n > 1 ? (float)(1.0 / D[q]->step) : 0.0f;
        DT[q]->n = D[q]->n;
        DT[q]->off = (int)dens.size();
        dens.insert(dens.end(), D[q]->v, D[q]->v + D[q]->n);
    }
    ts->w2_one = drift_proportional(t->b1, t->b2, &ts->w2c) ? 1 : 0;
    hipError_t e = hipMalloc((void**)&ts->dtab, sizeof(float4) * dtab.size());
    if (e == hipSuccess) e = hipMalloc((void**)&ts->atab, sizeof(float4) * atab.size());
    if (e == hipSuccess) e = hipMalloc((void**)&ts->denstab, sizeof(float) * dens.size());
    if (e == hipSuccess)
        e = hipMemcpy(ts->dtab, dtab.data(), sizeof(float4) * dtab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ts->atab, atab.data(), sizeof(float4) * atab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ts->denstab, dens.data(), sizeof(float) * dens.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_table_set(ts);
        return fail(e == hipErrorOutOfMemory ? FSPB_E_NOMEM : FSPB_E_HIP,
                    "uploading the commissioned tables failed: %s", hipGetErrorString(e));
    }
    ts->key = std::move(key);
    ts->refs = 1;
    ts->last_use = ++g_tables_clock;
    // keep at most kMaxIdleTableSets unused sets: drop the least recently used
    int idle = 0;
    for (TableSet* x : sets) idle += x->refs == 0;
    while (idle > kMaxIdleTableSets) {
        auto it = std::min_element(sets.begin(), sets.end(), [](TableSet* a, TableSet* b) {
            if ((a->refs == 0) != (b->refs == 0)) return a->refs == 0;
            return a->last_use < b->last_use;
        });
        free_table_set(*it);
        sets.erase(it);
        --idle;
    }
    sets.push_back(ts);
    *out = ts;
    return FSPB_OK;
}

static int create_impl(const fspb_ct* ct, int n_beams, const fspb_beam* beams,
                       const fspb_tables* t, const fspb_options* opts, hipStream_t s,
                       fspb_geometry* G) {
    fspb_options o;
    if (opts) {
        o = *opts;
    } else {
        memset(&o, 0, sizeof o);
        o.dc_enabled = 1;
    }
    if (o.roi_radius == 0) o.roi_radius = 5.0f;
    if (o.rho_surface == 0) o.rho_surface = 0.5f;
    if (o.smooth_sigma == 0) o.smooth_sigma = 0.5f;
    if (o.rho_min == 0 && o.rho_max == 0) {
        o.rho_min = 0.1f;
        o.rho_max = 2.0f;
    }
    const double dmin = std::min(std::min((double)ct->dx, (double)ct->dy), (double)ct->dz);
    double step = o.sample_step > 0 ? (double)o.sample_step : 0.5 * dmin;
    G->sample_step = (float)step;

    const int nx = ct->nx, ny = ct->ny, nz = ct->nz;
    const long nv = (long)nx * ny * nz;
    G->n_beams = n_beams;
    G->dc_created = G->dc_enabled = o.dc_enabled;
    G->siddon = (o.flags & FSPB_FLAG_SIDDON) ? 1 : 0;
    G->tile.per_beam = o.schedule;
    if (o.tile_waves != 0) {
        G->tile.shape = o.tile_shape;
        G->tile.waves_per_block = o.tile_waves;
    }
    int nbl = 0;
    for (int b = 0; b < n_beams; ++b) nbl += beams[b].nbx * beams[b].nby;
    G->n_beamlets = nbl;

    // plan reference point: grid centre
    double P0[3] = {ct->ox + 0.5 * (nx - 1) * ct->dx, ct->oy + 0.5 * (ny - 1) * ct->dy,
                    ct->oz + 0.5 * (nz - 1) * ct->dz};
    double L[3] = {nx * (double)ct->dx, ny * (double)ct->dy, nz * (double)ct->dz};
    double diag = sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    G->k_stride = (int)floor(diag / step) + 3;
    // the pair kernels address the depth tables (32-byte records) with
    // 32-bit byte offsets
    if ((long long)G->k_stride * nbl > (1LL << 27) - 1)
        return fail(FSPB_E_ARG, "depth tables of %d x %d samples exceed 2^27-1", nbl, G->k_stride);

    PlanConst& P = G->P;
    P.nx = nx;
    P.ny = ny;
    P.nz = nz;
    P.n_beams = n_beams;
    P.dx = ct->dx;
    P.dy = ct->dy;
    P.dz = ct->dz;
    P.R2 = o.roi_radius * o.roi_radius;
    P.qx0 = (float)(ct->ox - P0[0]);
    P.qy0 = (float)(ct->oy - P0[1]);
    P.qz0 = (float)(ct->oz - P0[2]);
    P.inv_d = (float)(1.0 / step);
    P.dt_inv = t->u1x.n > 1 ? (float)(1.0 / t->u1x.step) : 0.0f;
    P.dt_off = t->u1x.n > 1 ? (float)(-(double)t->u1x.start / t->u1x.step) : 0.0f;
    P.dt_n = t->u1x.n;
    P.at_inv = t->A.n > 1 ? (float)(1.0 / t->A.step) : 0.0f;
    P.at_off = t->A.n > 1 ? (float)(-(double)t->A.start / t->A.step) : 0.0f;
    P.at_n = t->A.n;
    P.a_cols = std::max(t->n_theta - 1, 1);
    P.dc = o.dc_enabled;
    long max_bricks = 0;
    for (int sh = 0; sh < kNumShapes; ++sh) max_bricks = std::max(max_bricks, brick_count(P, sh));

    // ---- commissioned tables: packed and uploaded once per distinct set -------
    int rc;
    if ((rc = acquire_tables(G->device, t, P.a_cols, &G->tabs)) != FSPB_OK) return rc;
    P.w2c = G->tabs->w2c;
    P.w2_one = G->tabs->w2_one;
    G->dtab = G->tabs->dtab;
    G->atab = G->tabs->atab;
    G->denstab = G->tabs->denstab;
    G->dens = G->tabs->dens;
    G->dens.rho_min = o.rho_min;
    G->dens.rho_max = o.rho_max;

    // beams: FP64 inputs of the setup kernel and FP32 culling descriptors
    std::vector<BeamIn> bin(n_beams);
    std::vector<BeamDesc> bd(n_beams);
    int first = 0;
    for (int b = 0; b < n_beams; ++b) {
        const fspb_beam& B = beams[b];
        BeamIn& I = bin[b];
        I.gantry = B.gantry;
        I.couch = B.couch;
        for (int q = 0; q < 3; ++q) I.iso[q] = B.iso[q];
        I.sad = B.sad;
        I.wx = B.wx;
        I.wy = B.wy;
        I.cx = B.cx;
        I.cy = B.cy;
        I.nbx = B.nbx;
        I.nby = B.nby;
        I.first = first;
        double phi = B.gantry, psi = B.couch, cp = cos(psi), sp = sin(psi);
        double c0[3] = {-sin(phi), cos(phi), 0.0}, e0[3] = {cos(phi), sin(phi), 0.0};
        double cax[3] = {cp * c0[0] + sp * c0[2], c0[1], -sp * c0[0] + cp * c0[2]};
        double ex[3] = {cp * e0[0] + sp * e0[2], e0[1], -sp * e0[0] + cp * e0[2]};
        double ey[3] = {sp, 0.0, cp};
        BeamDesc& Q = bd[b];
        for (int q = 0; q < 3; ++q) {
            Q.src[q] = (float)(B.iso[q] - (double)B.sad * cax[q] - P0[q]);
            Q.cax[q] = (float)cax[q];
            Q.ex[q] = (float)ex[q];
            Q.ey[q] = (float)ey[q];
        }
        Q.sad = B.sad;
        Q.a0 = (float)(-0.5 * (B.nbx - 1) * B.wx + B.cx);
        Q.b0 = (float)(-0.5 * (B.nby - 1) * B.wy + B.cy);
        Q.wx = B.wx;
        Q.wy = B.wy;
        Q.nbx = B.nbx;
        Q.nby = B.nby;
        Q.first = first;
        double am = 0.5 * (B.nbx - 1) * B.wx + fabs((double)B.cx);
        double bm = 0.5 * (B.nby - 1) * B.wy + fabs((double)B.cy);
        Q.pad_scale = (float)(o.roi_radius * sqrt((double)B.sad * B.sad + am * am + bm * bm));
        // depth range of the grid box along the central axis (per-beam schedule)
        {
            const double h[3] = {0.5 * nx * ct->dx, 0.5 * ny * ct->dy, 0.5 * nz * ct->dz};
            double zlo = 1e300, zhi = -1e300;
            for (int c = 0; c < 8; ++c) {
                double z = 0.0;
                for (int q = 0; q < 3; ++q)
                    z += (((c >> q) & 1) ? h[q] : -h[q]) * cax[q] - (double)Q.src[q] * cax[q];
                zlo = std::min(zlo, z);
                zhi = std::max(zhi, z);
            }
            Q.nbins = std::max(1, kSplitKeys / n_beams);
            Q.zlo = (float)zlo;
            Q.zinv = (float)(Q.nbins / std::max(zhi - zlo, 1e-3));
        }
        first += B.nbx * B.nby;
    }

    // smoothing weights (normalised 1-D Gaussians per axis)
    const double del[3] = {ct->dx, ct->dy, ct->dz};
    std::vector<float> w3;
    for (int a = 0; a < 3; ++a) {
        double sg = o.smooth_sigma;
        int r = sg > 0 ? (int)ceil(3.0 * sg / del[a] - 1e-6) : 0;
        if (r > 64) return fail(FSPB_E_ARG, "smoothing radius %d voxels is too large", r);
        G->smooth_r[a] = r;
        std::vector<double> g(2 * r + 1);
        double sum = 0;
        for (int q = -r; q <= r; ++q) {
            double x = q * del[a];
            g[q + r] = sg > 0 ? exp(-x * x / (2.0 * sg * sg)) : 1.0;
            sum += g[q + r];
        }
        for (double v : g) w3.push_back((float)(v / sum));
    }

    // ---- device buffers ----------------------------------------------------
#define ALLOC(ptr, bytes)                                                   \
    if ((rc = G->alloc((void**)&(ptr), (bytes))) != FSPB_OK) return rc;
    // the small per-plan inputs (beam descriptors, setup inputs, smoothing
    // weights) travel in one block and one copy
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t off_bin = align(sizeof(BeamDesc) * n_beams);
    const size_t off_w3 = off_bin + align(sizeof(BeamIn) * n_beams);
    const size_t small_bytes = off_w3 + sizeof(float) * w3.size();
    std::vector<unsigned char> small(small_bytes, 0);
    memcpy(small.data(), bd.data(), sizeof(BeamDesc) * n_beams);
    memcpy(small.data() + off_bin, bin.data(), sizeof(BeamIn) * n_beams);
    memcpy(small.data() + off_w3, w3.data(), sizeof(float) * w3.size());
    unsigned char* dsmall = nullptr;
    ALLOC(dsmall, small_bytes);
    G->beams = reinterpret_cast<BeamDesc*>(dsmall);
    G->beam_in = reinterpret_cast<BeamIn*>(dsmall + off_bin);
    G->w3 = reinterpret_cast<float*>(dsmall + off_w3);
    ALLOC(G->frames, sizeof(Frame64) * nbl);
    ALLOC(G->desc, sizeof(BeamletDesc) * nbl);
    ALLOC(G->tinfo, sizeof(TraceInfo) * nbl);
    ALLOC(G->tT, sizeof(float2) * (size_t)nbl * G->k_stride);
    ALLOC(G->order, sizeof(int) * max_bricks);
    ALLOC(G->cost, sizeof(int) * max_bricks);
    ALLOC(G->adj_part, sizeof(float) * (size_t)kAdjMaxSlabs * nbl);
    ALLOC(G->adj_queue, sizeof(int) * 8 * kAdjQueueInts);
    if (o.dc_enabled) {
        // one block: the 16-byte plane, then the 8-byte plane
        ALLOC(G->tTW, (sizeof(float4) + sizeof(float2)) * (size_t)nbl * G->k_stride);
        G->tW2 = reinterpret_cast<float2*>(G->tTW + (size_t)nbl * G->k_stride);
        ALLOC(G->rhohat, sizeof(float) * nv);
        ALLOC(G->fac, sizeof(float4) * nv);
    }
    HIP_TRY(hipMemcpyAsync(dsmall, small.data(), small_bytes, hipMemcpyHostToDevice, s));
    // the handle reads its own copy of the CT (taken by the first smoothing
    // pass, or by a copy without density correction): create returns once
    // the copy is taken, while kernels 1-4 may still run
    ALLOC(G->rho, sizeof(float) * nv);
    HIP_TRY(hipEventCreateWithFlags(&G->ready, hipEventDisableTiming));
    if (!o.dc_enabled) {
        HIP_TRY(hipMemcpyAsync(G->rho, ct->density, sizeof(float) * nv, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipEventRecord(G->ready, s));
    }

    // ---- kernels 1-4 ---------------------------------------------------------
    if (o.dc_enabled) {
        // the two intermediate passes use the (not yet written) depth-table
        // buffer as scratch when it is large enough, else two pool blocks
        const size_t tt_bytes = sizeof(float2) * (size_t)nbl * G->k_stride;
        if (tt_bytes >= 2 * sizeof(float) * (size_t)nv) {
            G->tmp0 = reinterpret_cast<float*>(G->tT);
            G->tmp1 = G->tmp0 + nv;
        } else {
            ALLOC(G->tmp0, sizeof(float) * nv);
            ALLOC(G->tmp1, sizeof(float) * nv);
        }
        launch_smooth(ct->density, G->rho, G->ready, G->tmp0, G->tmp1, G->rhohat, G->fac, nx, ny,
                      nz, G->w3, G->smooth_r, G->denstab, G->dens, s);
        HIP_TRY(hipGetLastError());
    }
#undef ALLOC
    double lo[3] = {ct->ox - 0.5 * ct->dx, ct->oy - 0.5 * ct->dy, ct->oz - 0.5 * ct->dz};
    double hi[3] = {ct->ox + (nx - 0.5) * ct->dx, ct->oy + (ny - 0.5) * ct->dy,
                    ct->oz + (nz - 0.5) * ct->dz};
    launch_setup(G->beam_in, n_beams, nbl, lo, hi, step, G->frames, s);
    HIP_TRY(hipGetLastError());
    TraceGrid& tg = G->tg;
    tg.o[0] = ct->ox;
    tg.o[1] = ct->oy;
    tg.o[2] = ct->oz;
    tg.inv[0] = 1.0 / (double)ct->dx;
    tg.inv[1] = 1.0 / (double)ct->dy;
    tg.inv[2] = 1.0 / (double)ct->dz;
    tg.n[0] = nx;
    tg.n[1] = ny;
    tg.n[2] = nz;
    tg.del[0] = ct->dx;
    tg.del[1] = ct->dy;
    tg.del[2] = ct->dz;
    TraceParams& tp = G->tp;
    tp.step = step;
    tp.rho_surface = o.rho_surface;
    tp.theta_step = t->n_theta > 1 ? (double)t->theta_step : 1.0;
    for (int q = 0; q < 3; ++q) tp.p0[q] = P0[q];
    tp.n_theta = t->n_theta;
    tp.n_A = t->A.n;
    tp.k_stride = G->k_stride;
    launch_trace(G->frames, nbl, G->rho, tg, tp, G->denstab, G->dens, G->tT, G->tTW, G->tW2,
                 G->desc, G->tinfo, s);
    HIP_TRY(hipGetLastError());
    if (G->siddon) {
        // exact tables replace the uniform samples (records, entrance, K)
        G->sid_stride = nx + ny + nz + 2;
        if ((long long)G->sid_stride * nbl > (1LL << 27) - 1)
            return fail(FSPB_E_ARG, "exact depth tables of %d x %d records are too large", nbl,
                        G->sid_stride);
        if ((rc = G->alloc((void**)&G->sid, 2 * sizeof(float4) * (size_t)nbl * G->sid_stride)) != FSPB_OK)
            return rc;
        launch_siddon(G->frames, nbl, G->rho, tg, tp, G->sid_stride, G->denstab, G->dens,
                      G->sid, G->desc, G->tinfo, s);
        HIP_TRY(hipGetLastError());
    }

    if ((rc = build_order(G, s)) != FSPB_OK) return rc;
    HIP_TRY(hipEventSynchronize(G->ready));   // the copy of ct->density is taken
    HIP_TRY(hipEventRecord(G->ready, s));     // end of the creation work
    G->ready_stream = s;
    G->pending = true;
    note_stream(G, s);
    return FSPB_OK;
}

int fspb_create_geometry(const fspb_ct* ct, int n_beams, const fspb_beam* beams,
                         const fspb_tables* tables, const fspb_options* opts, void* stream,
                         fspb_geometry** out) {
    if (!out) return fail(FSPB_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate(ct, n_beams, beams, tables, opts);
    if (rc) return rc;
    int dev = 0;
    rc = check_device(&dev);
    if (rc) return rc;
    fspb_geometry* G = new (std::nothrow) fspb_geometry();
    if (!G) return fail(FSPB_E_NOMEM, "host allocation failed");
    G->device = dev;
    if (hipDeviceGetAttribute(&G->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete G;
        return fail(FSPB_E_HIP, "hipDeviceGetAttribute failed");
    }
    rc = create_impl(ct, n_beams, beams, tables, opts, (hipStream_t)stream, G);
    if (rc) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        G->release();
        delete G;
        return rc;
    }
    *out = G;
    g_last_error.clear();
    return FSPB_OK;
}

// The forward of a handle, with its depth tables' kind.
static void enqueue_forward(fspb_geometry* g, const float* fluence, float* dose, hipStream_t s) {
    if (g->siddon)
        launch_forward_siddon(g->args(), g->dc_enabled != 0, g->tile, g->order, fluence, dose, s);
    else if (g->tile.per_beam)
        launch_forward_split(g->args(), g->dc_enabled != 0, g->tile, g->split, fluence, g->planes,
                             dose, s);
    else
        launch_forward(g->args(), g->dc_enabled != 0, g->tile, g->order, fluence, dose, s);
}

int fspb_forward(fspb_geometry* g, const float* fluence, float* dose, void* stream) {
    if (!g || !fluence || !dose) return fail(FSPB_E_ARG, "forward: NULL argument");
    int rc = settle(g, (hipStream_t)stream);
    if (rc) return rc;
    enqueue_forward(g, fluence, dose, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

static int adj_slab_of(const fspb_geometry* g) {
    return g->adj_slab > 0 ? g->adj_slab : adjoint_slab(g->P);
}

int fspb_set_adjoint_slab(fspb_geometry* g, int planes) {
    if (!g) return fail(FSPB_E_ARG, "set_adjoint_slab: NULL handle");
    if (planes != 0 && (planes < adjoint_min_slab(g->P) || planes > g->P.nz))
        return fail(FSPB_E_ARG, "set_adjoint_slab: %d planes outside [%d, %d] (or 0)", planes,
                    adjoint_min_slab(g->P), g->P.nz);
    g->adj_slab = planes;
    return FSPB_OK;
}

int fspb_get_adjoint_slab(const fspb_geometry* g, int* planes) {
    if (!g || !planes) return fail(FSPB_E_ARG, "get_adjoint_slab: NULL argument");
    *planes = adj_slab_of(g);
    return FSPB_OK;
}

int fspb_adjoint(fspb_geometry* g, const float* voxel_weight, float* grad, void* stream) {
    if (!g || !voxel_weight || !grad) return fail(FSPB_E_ARG, "adjoint: NULL argument");
    if (g->siddon) return fail(FSPB_E_STATE, "adjoint: not available with exact depth tables");
    int rc = settle(g, (hipStream_t)stream);
    if (rc) return rc;
    launch_adjoint(g->args(), g->dc_enabled != 0, g->n_beamlets, voxel_weight, grad, g->adj_part,
                   g->adj_queue, adj_slab_of(g), g->n_cu, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_beamlet_pair_counts(fspb_geometry* g, int* counts, void* stream) {
    if (!g || !counts) return fail(FSPB_E_ARG, "beamlet_pair_counts: NULL argument");
    int rc = settle(g, (hipStream_t)stream);
    if (rc) return rc;
    launch_adjoint_count(g->args(), g->n_beamlets, counts, g->adj_part, g->adj_queue,
                         adj_slab_of(g), g->n_cu, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

constexpr int kCountParts = 256;   // first-stage partial sums of a pair count

int fspb_count_pairs(fspb_geometry* g, const float* fluence, int* counts,
                     unsigned long long* total, void* stream) {
    if (!g || !total) return fail(FSPB_E_ARG, "count_pairs: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const long nv = (long)g->P.nx * g->P.ny * g->P.nz;
    int rc = settle(g, s);
    if (rc) return rc;
    // without per-voxel counts, one count per brick of the tile's shape
    long max_bricks = 0;
    for (int sh = 0; sh < kNumShapes; ++sh) max_bricks = std::max(max_bricks, brick_count(g->P, sh));
    if (!counts && !g->counts)
        if ((rc = g->alloc((void**)&g->counts, sizeof(int) * max_bricks)) != FSPB_OK) return rc;
    if (!g->partial) {
        if ((rc = g->alloc((void**)&g->partial, sizeof(unsigned long long) * kCountParts)) != FSPB_OK)
            return rc;
        if ((rc = g->alloc((void**)&g->total, sizeof(unsigned long long))) != FSPB_OK) return rc;
    }
    const DoseArgs a = g->args();
    if (counts) {
        launch_count(a, g->tile, g->order, fluence, counts, s);
        HIP_TRY(hipGetLastError());
        launch_sum_counts(counts, nv, g->partial, kCountParts, g->total, s);
    } else {
        launch_count_bricks(a, g->tile, g->order, fluence, g->counts, s);
        HIP_TRY(hipGetLastError());
        launch_sum_counts(g->counts, brick_count(g->P, g->tile.shape), g->partial, kCountParts,
                          g->total, s);
    }
    HIP_TRY(hipGetLastError());
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, g->total, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *total = h;
    return FSPB_OK;
}

// ---- the pair count without allocation ------------------------------------
// Scratch of fspb_count_pairs_noalloc: per-brick counts, then the partial
// sums.  One copy per device, held until the process ends; kernels take its
// device address (scratch_ptr), never the host-side name.
constexpr long kNoAllocMaxBricks = 1L << 20;
constexpr size_t kNoAllocPartOff = sizeof(int) * kNoAllocMaxBricks;
constexpr size_t kNoAllocScratchBytes = kNoAllocPartOff + sizeof(unsigned long long) * kCountParts;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the current device), looked up
// once per device.
static int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(FSPB_E_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FSPB_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FSPB_OK;
}

int fspb_count_pairs_noalloc(fspb_geometry* g, const float* fluence, unsigned long long* total,
                             void* stream) {
    if (!g || !total) return fail(FSPB_E_ARG, "count_pairs_noalloc: NULL argument");
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != g->device)
        return fail(FSPB_E_ARG, "count_pairs_noalloc: the handle belongs to device %d, the current "
                                "device is %d", g->device, cur);
    const long nb = brick_count(g->P, g->tile.shape);
    if (nb > kNoAllocMaxBricks)
        return fail(FSPB_E_ARG, "count_pairs_noalloc: %ld bricks exceed the static scratch of %ld",
                    nb, kNoAllocMaxBricks);
    void* base = nullptr;
    int rc = scratch_ptr(cur, &base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = settle(g, s)) != FSPB_OK) return rc;
    // every brick and every partial is written: nothing needs clearing
    int* bc = reinterpret_cast<int*>(base);
    auto* part = reinterpret_cast<unsigned long long*>(static_cast<unsigned char*>(base) + kNoAllocPartOff);
    launch_count_bricks(g->args(), g->tile, g->order, fluence, bc, s);
    HIP_TRY(hipGetLastError());
    launch_sum_counts(bc, nb, part, kCountParts, total, s);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_set_dc(fspb_geometry* g, int enabled) {
    if (!g) return fail(FSPB_E_ARG, "set_dc: NULL handle");
    if (enabled != 0 && enabled != 1) return fail(FSPB_E_ARG, "set_dc: enabled must be 0 or 1");
    if (enabled && !g->dc_created)
        return fail(FSPB_E_STATE, "set_dc: handle was created without density correction");
    g->dc_enabled = enabled;
    return FSPB_OK;
}

int fspb_drift_tables(const fspb_tables* t, float* ratio) {
    if (!t || !t->b1.v || !t->b2.v || t->b1.n < 1 || t->b2.n < 1)
        return fail(FSPB_E_ARG, "drift_tables: NULL tables or empty b1 / b2");
    float c = 0.0f;
    const bool one = drift_proportional(t->b1, t->b2, &c);
    if (ratio) *ratio = one ? c : 0.0f;
    return one ? 1 : 2;
}

int fspb_geometry_info(const fspb_geometry* g, fspb_info* info) {
    if (!g || !info) return fail(FSPB_E_ARG, "geometry_info: NULL argument");
    int rc = g->fetch_host();
    if (rc) return rc;
    memset(info, 0, sizeof *info);
    info->n_beams = g->n_beams;
    info->n_beamlets = g->n_beamlets;
    info->nx = g->P.nx;
    info->ny = g->P.ny;
    info->nz = g->P.nz;
    info->n_vox = (long long)g->P.nx * g->P.ny * g->P.nz;
    info->k_stride = g->k_stride;
    info->k_max = g->k_max;
    info->n_hit = g->n_hit;
    info->n_entry_ambiguous = g->n_amb;
    for (int a = 0; a < 3; ++a) info->smooth_radius[a] = g->smooth_r[a];
    info->sample_step = g->sample_step;
    info->dc_enabled = g->dc_enabled;
    info->device_bytes = (long long)g->device_bytes;
    info->drift_tables = g->P.w2_one ? 1 : 2;
    info->drift_ratio = g->P.w2_one ? g->P.w2c : 0.0f;
    return FSPB_OK;
}

int fspb_smoothed_density(const fspb_geometry* g, float* out, void* stream) {
    if (!g || !out) return fail(FSPB_E_ARG, "smoothed_density: NULL argument");
    if (!g->rhohat) return fail(FSPB_E_STATE, "smoothed_density: handle has no density correction");
    int rc = settle(const_cast<fspb_geometry*>(g), (hipStream_t)stream);
    if (rc) return rc;
    const long nv = (long)g->P.nx * g->P.ny * g->P.nz;
    HIP_TRY(hipMemcpyAsync(out, g->rhohat, sizeof(float) * nv, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return FSPB_OK;
}

int fspb_beamlet(const fspb_geometry* g, int i, fspb_beamlet_info* info, float* T, float* W1,
                 float* W2, int max_k) {
    if (!g) return fail(FSPB_E_ARG, "beamlet: NULL handle");
    if (i < 0 || i >= g->n_beamlets) return fail(FSPB_E_ARG, "beamlet: index %d out of range", i);
    int rc = g->fetch_host();
    if (rc) return rc;
    const BeamletDesc& d = g->h_desc[i];
    const Frame64& f = g->h_frames[i];
    const TraceInfo& ti = g->h_info[i];
    if (info) {
        memset(info, 0, sizeof *info);
        info->hit = d.hit;
        info->k_entry = ti.k_entry;
        info->n_samples = ti.n_samples;
        info->K = d.K;
        info->s_in = f.s_in;
        info->s_entry = ti.s_entry;
        info->theta = f.theta;
        for (int q = 0; q < 3; ++q) {
            info->src[q] = f.src[q];
            info->dir[q] = f.d[q];
            info->ex[q] = f.ex[q];
            info->ey[q] = f.ey[q];
        }
        info->entry_margin = ti.margin;
        for (int q = 0; q < 3; ++q) {
            info->pair_t[q] = d.d[q];
            info->pair_x[q] = d.ex[q];
            info->pair_y[q] = d.ey[q];
        }
        info->pair_t[3] = d.c_t;
        info->pair_x[3] = d.c_x;
        info->pair_y[3] = d.c_y;
    }
    int n = std::min(max_k, d.K);
    if (n > 0 && (T || W1 || W2) && g->siddon)
        return fail(FSPB_E_STATE, "beamlet: the sampled tables are not kept with exact depth tables");
    if (n > 0 && (T || W1 || W2)) {
        std::vector<float2> tt(n);
        HIP_TRY(hipMemcpy(tt.data(), g->tT + d.tab_off, sizeof(float2) * n, hipMemcpyDeviceToHost));
        if (T)
            for (int j = 0; j < n; ++j) T[j] = tt[j].x;
        if ((W1 || W2) && g->tTW) {
            std::vector<float4> tw(n);
            std::vector<float2> tw2(n);
            HIP_TRY(hipMemcpy(tw.data(), g->tTW + d.tab_off, sizeof(float4) * n, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(tw2.data(), g->tW2 + d.tab_off, sizeof(float2) * n, hipMemcpyDeviceToHost));
            for (int j = 0; j < n; ++j) {
                if (W1) W1[j] = tw[j].z;
                if (W2) W2[j] = tw2[j].x;
            }
        }
    }
    return FSPB_OK;
}

void fspb_destroy(fspb_geometry* g) {
    if (!g) return;
    // with the queued work on a few known streams, the buffers return to the
    // pool once the work on each is done, without waiting here; at most
    // kMaxPendingReleases handles wait so
    constexpr size_t kMaxPendingReleases = 2;
    bool deferred = false;
    if (!g->streams.empty() && !g->many_streams) {
        std::vector<hipEvent_t> evs;
        bool ok = true;
        for (hipStream_t st : g->streams) {
            hipEvent_t ev = nullptr;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                ok = false;
                break;
            }
            evs.push_back(ev);
            if (hipEventRecord(ev, st) != hipSuccess) {
                ok = false;
                break;
            }
        }
        if (ok) {
            std::lock_guard<std::mutex> lk(pool().mu);
            pool().deferred.push_back({g->device, std::move(evs), std::move(g->blocks)});
            g->blocks.clear();
            reap_locked(kMaxPendingReleases);
            deferred = true;
        } else {
            for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
        }
    }
    if (!deferred) {
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
    }
    g->release();
    delete g;
}

int fspb_release_cached_memory(void) {
    HIP_TRY(hipDeviceSynchronize());
    {
        std::lock_guard<std::mutex> lk(pool().mu);
        reap_locked(0);
    }
    {
        std::lock_guard<std::mutex> lk(g_tables_mu);
        auto& sets = table_sets();
        for (auto it = sets.begin(); it != sets.end();) {
            if ((*it)->refs == 0) {
                free_table_set(*it);
                it = sets.erase(it);
            } else {
                ++it;
            }
        }
    }
    std::vector<void*> drop;
    {
        std::lock_guard<std::mutex> lk(pool().mu);
        for (auto& kv : pool().free_blocks) {
            drop.insert(drop.end(), kv.second.begin(), kv.second.end());
            kv.second.clear();
        }
        pool().cached = 0;
    }
    for (void* p : drop) HIP_TRY(hipFree(p));
    return FSPB_OK;
}


int fspb_tile_shapes(int* dims, int max_shapes) {
    if (dims)
        for (int q = 0; q < std::min(max_shapes, kNumShapes); ++q) shape_dims(q, dims + 3 * q);
    return kNumShapes;
}

int fspb_set_tile(fspb_geometry* g, int shape, int waves_per_block, void* stream) {
    if (!g) return fail(FSPB_E_ARG, "set_tile: NULL handle");
    if (shape < 0 || shape >= kNumShapes) return fail(FSPB_E_ARG, "set_tile: shape %d out of range", shape);
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4 &&
        waves_per_block != kLdsWaves)
        return fail(FSPB_E_ARG, "set_tile: waves_per_block must be 1, 2, 4 or 8");
    hipStream_t s = (hipStream_t)stream;
    int rc = settle(g, s);
    if (rc) return rc;
    const bool rebuild = shape != g->tile.shape;
    g->tile.shape = shape;
    g->tile.waves_per_block = waves_per_block;
    if (!rebuild) return FSPB_OK;
    if ((rc = build_order(g, s)) != FSPB_OK) return rc;
    // like the creation work, the new schedule is awaited by other streams
    // (outside graph capture; a captured rebuild is ordered by its graph)
    if (g->ready && !capturing(s)) {
        HIP_TRY(hipEventRecord(g->ready, s));
        g->ready_stream = s;
        g->pending = true;
    }
    return FSPB_OK;
}

int fspb_get_tile(const fspb_geometry* g, int* shape, int* waves_per_block) {
    if (!g || !shape || !waves_per_block) return fail(FSPB_E_ARG, "get_tile: NULL argument");
    *shape = g->tile.shape;
    *waves_per_block = g->tile.waves_per_block;
    return FSPB_OK;
}

int fspb_set_schedule(fspb_geometry* g, int per_beam, void* stream) {
    if (!g) return fail(FSPB_E_ARG, "set_schedule: NULL handle");
    if (per_beam != 0 && per_beam != 1) return fail(FSPB_E_ARG, "set_schedule: per_beam must be 0 or 1");
    if (per_beam && g->siddon)
        return fail(FSPB_E_STATE, "set_schedule: not available with exact depth tables");
    hipStream_t s = (hipStream_t)stream;
    int rc = settle(g, s);
    if (rc) return rc;
    if (per_beam == g->tile.per_beam) return FSPB_OK;
    g->tile.per_beam = per_beam;
    if (!per_beam) return FSPB_OK;
    if ((rc = build_order(g, s)) != FSPB_OK) return rc;
    if (g->ready && !capturing(s)) {
        HIP_TRY(hipEventRecord(g->ready, s));
        g->ready_stream = s;
        g->pending = true;
    }
    return FSPB_OK;
}

int fspb_get_schedule(const fspb_geometry* g, int* per_beam) {
    if (!g || !per_beam) return fail(FSPB_E_ARG, "get_schedule: NULL argument");
    *per_beam = g->tile.per_beam;
    return FSPB_OK;
}

int fspb_autotune(fspb_geometry* g, const float* fluence, float* dose_scratch, int reps,
                  void* stream, fspb_tune_result* results, int max_results, int* n_results) {
    if (!g || !fluence || !dose_scratch || reps < 1)
        return fail(FSPB_E_ARG, "autotune: NULL argument or reps < 1");
    hipStream_t s = (hipStream_t)stream;
    if (int rc0 = settle(g, s)) return rc0;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int wpbs[4] = {1, 2, 4, kLdsWaves};
    TileCfg best = g->tile;
    float best_ms = 1e30f;
    int n = 0, rc = FSPB_OK;
    const int n_sched = g->siddon ? 1 : 2;
    for (int pb = 0; pb < n_sched && rc == FSPB_OK; ++pb)
    for (int sh = 0; sh < kNumShapes && rc == FSPB_OK; ++sh) {
        for (int w = 0; w < 4 && rc == FSPB_OK; ++w) {
            rc = fspb_set_schedule(g, pb, stream);
            if (rc == FSPB_OK) rc = fspb_set_tile(g, sh, wpbs[w], stream);
            if (rc) break;
            std::vector<float> ms;
            enqueue_forward(g, fluence, dose_scratch, s);
            for (int r = 0; r < reps; ++r) {
                (void)hipEventRecord(e0, s);
                enqueue_forward(g, fluence, dose_scratch, s);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(FSPB_E_HIP, "autotune: forward failed");
                    break;
                }
                float t = 0;
                (void)hipEventElapsedTime(&t, e0, e1);
                ms.push_back(t);
            }
            if (rc) break;
            std::sort(ms.begin(), ms.end());
            const float med = ms[ms.size() / 2];
            if (results && n < max_results) {
                results[n].shape = sh;
                shape_dims(sh, results[n].dims);
                results[n].waves_per_block = wpbs[w];
                results[n].ms = med;
                results[n].per_beam = pb;
            }
            ++n;
            if (med < best_ms) {
                best_ms = med;
                best = g->tile;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (n_results) *n_results = n;
    if ((rc = fspb_set_schedule(g, best.per_beam, stream)) != FSPB_OK) return rc;
    return fspb_set_tile(g, best.shape, best.waves_per_block, stream);
}

int fspb_autotune_adjoint(fspb_geometry* g, const float* voxel_weight, float* grad_scratch,
                          int reps, void* stream, int* planes, float* ms, int max_results,
                          int* n_results) {
    if (!g || !voxel_weight || !grad_scratch || reps < 1)
        return fail(FSPB_E_ARG, "autotune_adjoint: NULL argument or reps < 1");
    if (g->siddon) return fail(FSPB_E_STATE, "autotune_adjoint: not available with exact depth tables");
    hipStream_t s = (hipStream_t)stream;
    if (int rc0 = settle(g, s)) return rc0;
    // the default thickness, half and two and four times it, and the whole grid
    const int d = adjoint_slab(g->P), lo = adjoint_min_slab(g->P), nz = g->P.nz;
    std::vector<int> cand;
    for (int c : {d / 2, d, 2 * d, 4 * d, nz}) {
        c = std::min(std::max(c, std::max(lo, 1)), nz);
        if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    }
    std::sort(cand.begin(), cand.end());
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int keep = g->adj_slab;
    int best = d, n = 0, rc = FSPB_OK;
    float best_ms = 1e30f;
    for (int c : cand) {
        g->adj_slab = c;
        std::vector<float> t_ms;
        launch_adjoint(g->args(), g->dc_enabled != 0, g->n_beamlets, voxel_weight, grad_scratch,
                       g->adj_part, g->adj_queue, c, g->n_cu, s);
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            launch_adjoint(g->args(), g->dc_enabled != 0, g->n_beamlets, voxel_weight,
                           grad_scratch, g->adj_part, g->adj_queue, c, g->n_cu, s);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(FSPB_E_HIP, "autotune_adjoint: adjoint failed");
                break;
            }
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            t_ms.push_back(t);
        }
        if (rc) break;
        std::sort(t_ms.begin(), t_ms.end());
        const float med = t_ms[t_ms.size() / 2];
        if (n < max_results) {
            if (planes) planes[n] = c;
            if (ms) ms[n] = med;
        }
        ++n;
        if (med < best_ms) {
            best_ms = med;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        g->adj_slab = keep;
        return rc;
    }
    if (n_results) *n_results = n;
    g->adj_slab = best;
    return FSPB_OK;
}

int fspb_wait_ready(fspb_geometry* g, void* stream) {
    if (!g) return fail(FSPB_E_ARG, "wait_ready: NULL handle");
    return settle(g, (hipStream_t)stream);
}

int fspb_update_density(fspb_geometry* g, const float* density, void* stream) {
    if (!g || !density) return fail(FSPB_E_ARG, "update_density: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (int rc0 = settle(g, s)) return rc0;
    const PlanConst& P = g->P;
    if (g->dc_created) {
        launch_smooth(density, nullptr, nullptr, g->tmp0, g->tmp1, g->rhohat, g->fac, P.nx, P.ny,
                      P.nz, g->w3, g->smooth_r, g->denstab, g->dens, s);
        HIP_TRY(hipGetLastError());
    }
    launch_trace(g->frames, g->n_beamlets, density, g->tg, g->tp, g->denstab, g->dens, g->tT,
                 g->tTW, g->tW2, g->desc, g->tinfo, s);
    HIP_TRY(hipGetLastError());
    if (g->siddon) {
        launch_siddon(g->frames, g->n_beamlets, density, g->tg, g->tp, g->sid_stride, g->denstab,
                      g->dens, g->sid, g->desc, g->tinfo, s);
        HIP_TRY(hipGetLastError());
    }
    g->host_ready = false;
    return FSPB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many plans in one persistent launch.
struct fspb_batch {
    int device = 0;
    int n_plans = 0, n_waves = 0;
    int dc = kPlain;                 // correction mode shared by every plan
    TileCfg tile;
    std::vector<fspb_geometry*> plans;
    std::vector<std::pair<void*, size_t>> blocks;
    const float4* water = nullptr;   // the water table all plans share, else null
    int water_n = 0;
    DoseArgs* d_args = nullptr;
    int2* d_items = nullptr;
    int* d_begin = nullptr;
    unsigned long long* ts_done = nullptr;
    unsigned long long* ts_start = nullptr;
    long n_items = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double clock_khz = 100000.0;

    int alloc(void** p, size_t bytes) {
        size_t cls = 0;
        int rc = pool_alloc(device, p, bytes, &cls);
        if (rc == FSPB_OK) blocks.push_back({*p, cls});
        return rc;
    }
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        for (auto& b : blocks) pool_free(device, b.first, b.second);
        blocks.clear();
    }
};

static int batch_enqueue(fspb_batch* b, const float* const* fluence, float* const* dose,
                         const float* const* density, hipStream_t s) {
    for (int p = 0; p < b->n_plans; ++p)
        if (!fluence[p] || !dose[p]) return fail(FSPB_E_ARG, "batch: NULL fluence or dose of plan %d", p);
    if (density)
        for (int p = 0; p < b->n_plans; ++p) {
            int rc = fspb_update_density(b->plans[p], density[p], s);
            if (rc) return rc;
        }
    BatchPtrs ptrs = {};
    for (int p = 0; p < b->n_plans; ++p) {
        ptrs.fluence[p] = fluence[p];
        ptrs.dose[p] = dose[p];
    }
    launch_fill_u64(b->ts_done, (long)b->n_plans * b->n_waves, 0ULL, s);
    HIP_TRY(hipGetLastError());
    launch_forward_batch(b->dc, b->tile, b->d_args, b->d_items, b->d_begin, b->n_waves, ptrs,
                         b->ts_done, b->ts_start, b->water, b->water_n, s);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

extern "C" {

int fspb_batch_create(int n, fspb_geometry* const* geoms, int shape, int waves_per_block,
                      int waves_per_cu, int policy, void* stream, fspb_batch** out) {
    if (!out) return fail(FSPB_E_ARG, "batch_create: out is NULL");
    *out = nullptr;
    if (n < 1 || !geoms) return fail(FSPB_E_ARG, "batch_create: need n >= 1 geometries");
    if (n > kMaxBatchPlans) return fail(FSPB_E_ARG, "batch_create: at most %d plans", kMaxBatchPlans);
    if (shape < 0 || shape >= kNumShapes) return fail(FSPB_E_ARG, "batch_create: bad shape");
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4 &&
        waves_per_block != kLdsWaves)
        return fail(FSPB_E_ARG, "batch_create: waves_per_block must be 1, 2, 4 or 8");
    if (waves_per_cu < 1 || waves_per_cu > 32)
        return fail(FSPB_E_ARG, "batch_create: waves_per_cu must be 1..32");
    if (policy != FSPB_SCHEDULE_THROUGHPUT && policy != FSPB_SCHEDULE_LATENCY)
        return fail(FSPB_E_ARG, "batch_create: unknown schedule policy %d", policy);
    for (int p = 0; p < n; ++p) {
        if (!geoms[p]) return fail(FSPB_E_ARG, "batch_create: geometry %d is NULL", p);
        if (int rc = settle_host(geoms[p])) return rc;   // the batch may run on any stream
        if (geoms[p]->siddon)
            return fail(FSPB_E_STATE, "batch_create: geometry %d uses exact depth tables", p);
        if (geoms[p]->dc_enabled != geoms[0]->dc_enabled)
            return fail(FSPB_E_ARG, "batch_create: plans must share the density-correction mode");
    }
    hipStream_t s = (hipStream_t)stream;
    fspb_batch* B = new (std::nothrow) fspb_batch();
    if (!B) return fail(FSPB_E_NOMEM, "host allocation failed");
    B->device = geoms[0]->device;
    B->n_plans = n;
    B->dc = kPlain;
    if (geoms[0]->dc_enabled) {
        B->dc = kDcOneDrift;
        for (int p = 0; p < n; ++p)
            if (!geoms[p]->P.w2_one) B->dc = kDcTwoDrift;
    }
    B->tile.shape = shape;
    B->tile.waves_per_block = waves_per_block;
    B->plans.assign(geoms, geoms + n);
    // one shared water table (plans built from the same commissioned tables
    // share the device copy) can be staged in LDS by the persistent kernel
    B->water = geoms[0]->dtab;
    B->water_n = geoms[0]->P.dt_n;
    for (int p = 1; p < n; ++p)
        if (geoms[p]->dtab != B->water) B->water = nullptr;
    auto bail = [&](int rc) {
        (void)hipStreamSynchronize(s);
        B->release();
        delete B;
        return rc;
    };
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, B->device) == hipSuccess) cus = prop.multiProcessorCount;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, B->device) == hipSuccess && khz > 0)
            B->clock_khz = khz;
    }
    B->n_waves = waves_per_cu * cus;
    // items: every brick of every plan with its estimated work for the batch
    // shape; longest-processing-time-first assignment to the waves
    struct Item {
        int plan, brick, cost;
    };
    std::vector<Item> items;
    for (int p = 0; p < n; ++p) {
        fspb_geometry* g = geoms[p];
        if (g->tile.shape != shape) {
            int rc = fspb_set_tile(g, shape, g->tile.waves_per_block, stream);
            if (rc) return bail(rc);
        }
        const long nb = brick_count(g->P, shape);
        int rc = fetch_cost(g, (hipStream_t)stream);
        if (rc) return bail(rc);
        for (long q = 0; q < nb; ++q) items.push_back({p, (int)q, g->h_cost[q] + 4});
    }
    if (policy == FSPB_SCHEDULE_THROUGHPUT) {
        // one longest-first list over all plans: shortest makespan
        std::stable_sort(items.begin(), items.end(),
                         [](const Item& x, const Item& y) { return x.cost > y.cost; });
    } else {
        // plans in increasing order of total work, each plan's bricks
        // longest-first: small plans complete early
        std::vector<long long> tot(n, 0);
        for (const Item& it : items) tot[it.plan] += it.cost;
        std::vector<int> rank(n);
        std::vector<int> ord(n);
        for (int p = 0; p < n; ++p) ord[p] = p;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return tot[x] < tot[y]; });
        for (int r = 0; r < n; ++r) rank[ord[r]] = r;
        std::stable_sort(items.begin(), items.end(), [&](const Item& x, const Item& y) {
            if (rank[x.plan] != rank[y.plan]) return rank[x.plan] < rank[y.plan];
            return x.cost > y.cost;
        });
    }
    std::vector<std::vector<int2>> per(B->n_waves);
    std::vector<std::pair<long long, int>> heap;
    heap.reserve(B->n_waves);
    for (int w = 0; w < B->n_waves; ++w) heap.push_back({0LL, w});
    auto cmp = [](const std::pair<long long, int>& a, const std::pair<long long, int>& b) {
        return a.first > b.first || (a.first == b.first && a.second > b.second);
    };
    std::make_heap(heap.begin(), heap.end(), cmp);
    for (const Item& it : items) {
        std::pop_heap(heap.begin(), heap.end(), cmp);
        auto& top = heap.back();
        per[top.second].push_back(make_int2(it.plan, it.brick));
        top.first += it.cost;
        std::push_heap(heap.begin(), heap.end(), cmp);
    }
    std::vector<int2> flat;
    std::vector<int> begin(B->n_waves + 1, 0);
    for (int w = 0; w < B->n_waves; ++w) {
        begin[w] = (int)flat.size();
        flat.insert(flat.end(), per[w].begin(), per[w].end());
    }
    begin[B->n_waves] = (int)flat.size();
    B->n_items = (long)flat.size();
    std::vector<DoseArgs> args(n);
    for (int p = 0; p < n; ++p) args[p] = geoms[p]->args();
    int rc;
    if ((rc = B->alloc((void**)&B->d_args, sizeof(DoseArgs) * n))) return bail(rc);
    if ((rc = B->alloc((void**)&B->d_items, sizeof(int2) * std::max<size_t>(flat.size(), 1)))) return bail(rc);
    if ((rc = B->alloc((void**)&B->d_begin, sizeof(int) * begin.size()))) return bail(rc);
    if ((rc = B->alloc((void**)&B->ts_done, sizeof(unsigned long long) * (size_t)n * B->n_waves))) return bail(rc);
    if ((rc = B->alloc((void**)&B->ts_start, sizeof(unsigned long long) * B->n_waves))) return bail(rc);
    if (hipMemcpyAsync(B->d_args, args.data(), sizeof(DoseArgs) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(B->d_items, flat.data(), sizeof(int2) * flat.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(B->d_begin, begin.data(), sizeof(int) * begin.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(FSPB_E_HIP, "batch_create: copy failed"));
    *out = B;
    return FSPB_OK;
}

int fspb_batch_forward(fspb_batch* b, const float* const* fluence, float* const* dose, void* stream) {
    if (!b || !fluence || !dose) return fail(FSPB_E_ARG, "batch_forward: NULL argument");
    return batch_enqueue(b, fluence, dose, nullptr, (hipStream_t)stream);
}

int fspb_batch_capture(fspb_batch* b, const float* const* fluence, float* const* dose,
                       const float* const* density, void* stream) {
    if (!b || !fluence || !dose) return fail(FSPB_E_ARG, "batch_capture: NULL argument");
    if (!stream) return fail(FSPB_E_ARG, "batch_capture: capture needs a non-null stream");
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = batch_enqueue(b, fluence, dose, density, s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(FSPB_E_HIP, "batch_capture: %s", hipGetErrorString(e));
    b->graph = graph;
    HIP_TRY(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    return FSPB_OK;
}

int fspb_batch_replay(fspb_batch* b, void* stream) {
    if (!b) return fail(FSPB_E_ARG, "batch_replay: NULL batch");
    if (!b->exec) return fail(FSPB_E_STATE, "batch_replay: nothing captured");
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return FSPB_OK;
}

int fspb_batch_latencies(const fspb_batch* b, double* plan_ms, double* total_ms, void* stream) {
    if (!b) return fail(FSPB_E_ARG, "batch_latencies: NULL batch");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    std::vector<unsigned long long> done((size_t)b->n_plans * b->n_waves), start(b->n_waves);
    HIP_TRY(hipMemcpy(done.data(), b->ts_done, sizeof(unsigned long long) * done.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(start.data(), b->ts_start, sizeof(unsigned long long) * start.size(), hipMemcpyDeviceToHost));
    unsigned long long t0 = ~0ULL, tend = 0;
    for (unsigned long long v : start) t0 = std::min(t0, v);
    for (int p = 0; p < b->n_plans; ++p) {
        unsigned long long m = 0;
        for (int w = 0; w < b->n_waves; ++w) m = std::max(m, done[(size_t)p * b->n_waves + w]);
        tend = std::max(tend, m);
        if (plan_ms) plan_ms[p] = m > t0 ? (double)(m - t0) / b->clock_khz : 0.0;
    }
    if (total_ms) *total_ms = tend > t0 ? (double)(tend - t0) / b->clock_khz : 0.0;
    return FSPB_OK;
}

int fspb_batch_info(const fspb_batch* b, int* n_waves, long long* n_items) {
    if (!b) return fail(FSPB_E_ARG, "batch_info: NULL batch");
    if (n_waves) *n_waves = b->n_waves;
    if (n_items) *n_items = b->n_items;
    return FSPB_OK;
}

void fspb_batch_destroy(fspb_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    b->release();
    delete b;
}

}  // extern "C"

// ===========================================================================
// Learned surrogate: network state and the surrogate entry points.
struct fspb_mlp {
    int device = 0;
    float* master = nullptr;   // FP32 parameters (flat layout of fspb.h)
    float* am = nullptr;       // Adam moments
    float* av = nullptr;
    __bf16* w1t = nullptr;     // BF16 copies in the layouts the kernels read
    __bf16* w2t = nullptr;
    __bf16* w2r = nullptr;
    __bf16* w3t = nullptr;
    __bf16* w3r = nullptr;
    float* grad_parts = nullptr;   // per-workgroup gradients of one launch
    float* loss_parts = nullptr;
    int part_tiles = 0;
    size_t grad_cls = 0, loss_cls = 0;
    long long step = 0;
    SurrogateScale sc{};
    SurrogateGuard gd{};
    std::vector<std::pair<void*, size_t>> blocks;

    int alloc(void** p, size_t bytes) {
        size_t cls = 0;
        int rc = pool_alloc(device, p, bytes, &cls);
        if (rc == FSPB_OK) blocks.push_back({*p, cls});
        return rc;
    }
    MlpWeights weights() const {
        MlpWeights W;
        W.w1t = W.w1t_rw = w1t;
        W.w2t = W.w2t_rw = w2t;
        W.w2r = W.w2r_rw = w2r;
        W.w3t = W.w3t_rw = w3t;
        W.w3r = W.w3r_rw = w3r;
        W.b1 = master + kOffB1;
        W.b2 = master + kOffB2;
        W.b3 = master + kOffB3;
        return W;
    }
    // per-workgroup scratch for a launch over n rows (grown on demand; the
    // old buffers are returned only after the device has finished with them)
    int ensure_parts(long long n) {
        const int tiles = mlp_tiles((long)n);
        if (tiles <= part_tiles) return FSPB_OK;
        HIP_TRY(hipDeviceSynchronize());
        pool_free(device, grad_parts, grad_cls);
        pool_free(device, loss_parts, loss_cls);
        grad_parts = loss_parts = nullptr;
        part_tiles = 0;
        int rc = pool_alloc(device, (void**)&grad_parts, sizeof(float) * (size_t)tiles * kMlpParams,
                            &grad_cls);
        if (rc != FSPB_OK) return rc;
        rc = pool_alloc(device, (void**)&loss_parts, sizeof(float) * (size_t)tiles, &loss_cls);
        if (rc != FSPB_OK) {
            pool_free(device, grad_parts, grad_cls);
            grad_parts = nullptr;
            return rc;
        }
        part_tiles = tiles;
        return FSPB_OK;
    }
    void release() {
        pool_free(device, grad_parts, grad_cls);
        pool_free(device, loss_parts, loss_cls);
        for (auto& b : blocks) pool_free(device, b.first, b.second);
        blocks.clear();
    }
};

namespace {

int check_rows(long long n, bool allow_zero, const char* what) {
    if (n < (allow_zero ? 0 : 1) || n > FSPB_MLP_MAX_ROWS)
        return fail(FSPB_E_ARG, "%s: row count %lld outside [%d, %d]", what, n, allow_zero ? 0 : 1,
                    FSPB_MLP_MAX_ROWS);
    return FSPB_OK;
}

int check_same_device(int dev, const char* what) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) return fail(FSPB_E_STATE, "%s: handle lives on device %d, current is %d", what, dev, cur);
    return FSPB_OK;
}

int upload_state(fspb_mlp* m, const float* params, const float* am, const float* av) {
    std::vector<float> zero(kMlpParams, 0.0f);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(m->master, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->am, am ? am : zero.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->av, av ? av : zero.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    launch_mlp_sync(m->master, m->weights(), 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    return FSPB_OK;
}

int check_finite(const float* v, int n, const char* what) {
    for (int q = 0; q < n; ++q)
        if (!isfinite(v[q])) return fail(FSPB_E_ARG, "%s: value %d is not finite", what, q);
    return FSPB_OK;
}

}  // namespace

extern "C" {

int fspb_mlp_create(const float* params, fspb_mlp** out) {
    if (!out) return fail(FSPB_E_ARG, "mlp_create: NULL out");
    *out = nullptr;
    if (!params) return fail(FSPB_E_ARG, "mlp_create: NULL params");
    int rc = check_finite(params, kMlpParams, "mlp_create: params");
    if (rc != FSPB_OK) return rc;
    int dev = 0;
    if ((rc = check_device(&dev)) != FSPB_OK) return rc;
    fspb_mlp* m = new (std::nothrow) fspb_mlp();
    if (!m) return fail(FSPB_E_NOMEM, "mlp_create: host allocation failed");
    m->device = dev;
    for (int c = 0; c < kMlpOut; ++c) {
        m->sc.mean[c] = 0.0f;
        m->sc.stdev[c] = 1.0f;
        m->gd.band_lo[c] = -FLT_MAX;
        m->gd.band_hi[c] = FLT_MAX;
    }
    m->gd.rho_lo = -FLT_MAX;
    m->gd.rho_hi = FLT_MAX;
    m->gd.het_max = FLT_MAX;
    const size_t fp = sizeof(float) * kMlpParams;
    if ((rc = m->alloc((void**)&m->master, fp)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->am, fp)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->av, fp)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w1t, sizeof(__bf16) * kW1tN)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w2t, sizeof(__bf16) * kW2N)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w2r, sizeof(__bf16) * kW2N)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w3t, sizeof(__bf16) * kW3tN)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w3r, sizeof(__bf16) * kW3rN)) != FSPB_OK ||
        (rc = upload_state(m, params, nullptr, nullptr)) != FSPB_OK) {
        m->release();
        delete m;
        return rc;
    }
    *out = m;
    return FSPB_OK;
}

int fspb_mlp_set_scaling(fspb_mlp* m, const float* mean, const float* stdev) {
    if (!m || !mean || !stdev) return fail(FSPB_E_ARG, "mlp_set_scaling: NULL argument");
    for (int c = 0; c < kMlpOut; ++c)
        if (!isfinite(mean[c]) || !finite_pos(stdev[c]))
            return fail(FSPB_E_ARG, "mlp_set_scaling: output %d needs a finite mean and std > 0", c);
    for (int c = 0; c < kMlpOut; ++c) {
        m->sc.mean[c] = mean[c];
        m->sc.stdev[c] = stdev[c];
    }
    return FSPB_OK;
}

int fspb_mlp_set_guard(fspb_mlp* m, const fspb_surrogate_guard* g) {
    if (!m || !g) return fail(FSPB_E_ARG, "mlp_set_guard: NULL argument");
    if (std::isnan(g->rho_lo) || std::isnan(g->rho_hi) || std::isnan(g->het_max))
        return fail(FSPB_E_ARG, "mlp_set_guard: NaN bound");
    for (int c = 0; c < kMlpOut; ++c)
        if (std::isnan(g->band_lo[c]) || std::isnan(g->band_hi[c]))
            return fail(FSPB_E_ARG, "mlp_set_guard: NaN band for output %d", c);
    m->gd.rho_lo = g->rho_lo;
    m->gd.rho_hi = g->rho_hi;
    m->gd.het_max = g->het_max;
    for (int c = 0; c < kMlpOut; ++c) {
        m->gd.band_lo[c] = g->band_lo[c];
        m->gd.band_hi[c] = g->band_hi[c];
    }
    return FSPB_OK;
}

int fspb_mlp_loss_grad(fspb_mlp* m, const uint16_t* x, const float* t, long long n, float* grad,
                       float* loss, void* stream) {
    if (!m || !x || !t) return fail(FSPB_E_ARG, "mlp_loss_grad: NULL argument");
    int rc;
    if ((rc = check_rows(n, false, "mlp_loss_grad")) != FSPB_OK) return rc;
    if ((rc = check_same_device(m->device, "mlp_loss_grad")) != FSPB_OK) return rc;
    if ((rc = m->ensure_parts(n)) != FSPB_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int tiles = mlp_tiles((long)n);
    launch_mlp_train((const __bf16*)x, t, (long)n, m->weights(), m->grad_parts, m->loss_parts, s);
    HIP_TRY(hipGetLastError());
    if (grad) launch_mlp_grad_sum(m->grad_parts, tiles, grad, s);
    if (loss) launch_mlp_loss_sum(m->loss_parts, tiles, loss, s);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_mlp_train_step(fspb_mlp* m, const uint16_t* x, const float* t, long long n,
                        const fspb_adam* opt, float* loss, void* stream) {
    if (!m || !x || !t || !opt) return fail(FSPB_E_ARG, "mlp_train_step: NULL argument");
    if (!finite_pos(opt->lr) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
        !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !finite_pos(opt->eps))
        return fail(FSPB_E_ARG, "mlp_train_step: needs lr > 0, 0 <= beta < 1, eps > 0");
    int rc;
    if ((rc = check_rows(n, false, "mlp_train_step")) != FSPB_OK) return rc;
    if ((rc = check_same_device(m->device, "mlp_train_step")) != FSPB_OK) return rc;
    if ((rc = m->ensure_parts(n)) != FSPB_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int tiles = mlp_tiles((long)n);
    const MlpWeights W = m->weights();
    launch_mlp_train((const __bf16*)x, t, (long)n, W, m->grad_parts, m->loss_parts, s);
    HIP_TRY(hipGetLastError());
    if (loss) launch_mlp_loss_sum(m->loss_parts, tiles, loss, s);
    const long long k = m->step + 1;
    AdamParams ap;
    ap.lr = opt->lr;
    ap.beta1 = opt->beta1;
    ap.beta2 = opt->beta2;
    ap.eps = opt->eps;
    ap.bc1 = (float)(1.0 - pow((double)opt->beta1, (double)k));
    ap.bc2 = (float)(1.0 - pow((double)opt->beta2, (double)k));
    launch_mlp_adam(m->grad_parts, tiles, W, m->master, m->am, m->av, ap, s);
    HIP_TRY(hipGetLastError());
    m->step = k;
    return FSPB_OK;
}

int fspb_mlp_predict(fspb_mlp* m, const uint16_t* x, long long n, float* y, void* stream) {
    if (!m) return fail(FSPB_E_ARG, "mlp_predict: NULL handle");
    int rc;
    if ((rc = check_rows(n, true, "mlp_predict")) != FSPB_OK) return rc;
    if (n == 0) return FSPB_OK;
    if (!x || !y) return fail(FSPB_E_ARG, "mlp_predict: NULL argument");
    if ((rc = check_same_device(m->device, "mlp_predict")) != FSPB_OK) return rc;
    launch_mlp_forward((const __bf16*)x, (long)n, m->weights(), y, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_mlp_get_state(const fspb_mlp* m, float* params, float* adam_m, float* adam_v,
                       long long* step) {
    if (!m) return fail(FSPB_E_ARG, "mlp_get_state: NULL handle");
    HIP_TRY(hipDeviceSynchronize());
    const size_t fp = sizeof(float) * kMlpParams;
    if (params) HIP_TRY(hipMemcpy(params, m->master, fp, hipMemcpyDeviceToHost));
    if (adam_m) HIP_TRY(hipMemcpy(adam_m, m->am, fp, hipMemcpyDeviceToHost));
    if (adam_v) HIP_TRY(hipMemcpy(adam_v, m->av, fp, hipMemcpyDeviceToHost));
    if (step) *step = m->step;
    return FSPB_OK;
}

int fspb_mlp_set_state(fspb_mlp* m, const float* params, const float* adam_m,
                       const float* adam_v, long long step) {
    if (!m || !params) return fail(FSPB_E_ARG, "mlp_set_state: NULL argument");
    if (step < 0) return fail(FSPB_E_ARG, "mlp_set_state: negative step");
    int rc = check_finite(params, kMlpParams, "mlp_set_state: params");
    if (rc == FSPB_OK && adam_m) rc = check_finite(adam_m, kMlpParams, "mlp_set_state: adam_m");
    if (rc == FSPB_OK && adam_v) rc = check_finite(adam_v, kMlpParams, "mlp_set_state: adam_v");
    if (rc != FSPB_OK) return rc;
    if ((rc = check_same_device(m->device, "mlp_set_state")) != FSPB_OK) return rc;
    if ((rc = upload_state(m, params, adam_m, adam_v)) != FSPB_OK) return rc;
    m->step = step;
    return FSPB_OK;
}

void fspb_mlp_destroy(fspb_mlp* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    m->release();
    delete m;
}

static int check_surrogate_geometry(const fspb_geometry* g, const char* what) {
    if (!g) return fail(FSPB_E_ARG, "%s: NULL geometry", what);
    if (!g->dc_created)
        return fail(FSPB_E_STATE, "%s: the geometry was created without density correction", what);
    if (g->siddon) return fail(FSPB_E_STATE, "%s: not available with exact depth tables", what);
    // row ids are 32-bit, the gathers address the CT with 32-bit byte offsets
    // and index its rows with 24-bit multiplies
    const long long nv = (long long)g->P.nx * g->P.ny * g->P.nz;
    if (nv >= (1LL << 30) || nv * g->n_beams >= (1LL << 32) ||
        (long long)g->P.ny * g->P.nz >= (1LL << 24) || g->P.nx >= (1 << 24))
        return fail(FSPB_E_ARG, "%s: %lld voxels x %d beams exceed the surrogate's row range", what,
                    nv, g->n_beams);
    return check_same_device(g->device, what);
}

int fspb_surrogate_samples(fspb_geometry* g, const float* density, const int* rows, long long n,
                           uint16_t* x, float* t, int* valid, void* stream) {
    int rc;
    if ((rc = check_surrogate_geometry(g, "surrogate_samples")) != FSPB_OK) return rc;
    if ((rc = settle(g, (hipStream_t)stream)) != FSPB_OK) return rc;
    if (n < 0 || n > (1LL << 30)) return fail(FSPB_E_ARG, "surrogate_samples: bad row count %lld", n);
    if (n == 0) return FSPB_OK;
    if (!density || !rows || !x || !t || !valid)
        return fail(FSPB_E_ARG, "surrogate_samples: NULL argument");
    launch_surrogate_samples(g->args(), density, (const int2*)rows, (long)n, (__bf16*)x, t, valid,
                             (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_surrogate_infer(fspb_geometry* g, const fspb_mlp* m, const float* density, float* prm,
                         void* stream) {
    int rc;
    if ((rc = check_surrogate_geometry(g, "surrogate_infer")) != FSPB_OK) return rc;
    if ((rc = settle(g, (hipStream_t)stream)) != FSPB_OK) return rc;
    if (!m || !density || !prm) return fail(FSPB_E_ARG, "surrogate_infer: NULL argument");
    if (m->device != g->device) return fail(FSPB_E_STATE, "surrogate_infer: handles on different devices");
    if (!g->surr_live) {
        const size_t rows = (size_t)g->P.nx * g->P.ny * g->P.nz * g->n_beams;
        if ((rc = g->alloc((void**)&g->surr_live, sizeof(unsigned) * rows)) != FSPB_OK ||
            (rc = g->alloc((void**)&g->surr_count, 256)) != FSPB_OK ||
            (rc = g->alloc((void**)&g->surr_quad,
                           sizeof(float4) * (size_t)g->P.nx * g->P.ny * g->P.nz)) != FSPB_OK)
            return rc;
    }
    launch_surrogate_infer(g->args(), density, g->rhohat, m->weights(), m->sc, m->gd,
                           (float4*)prm, g->surr_quad, g->surr_live, g->surr_count,
                           (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_forward_surrogate(fspb_geometry* g, const float* fluence, const float* prm, float* dose,
                           void* stream) {
    int rc;
    if ((rc = check_surrogate_geometry(g, "forward_surrogate")) != FSPB_OK) return rc;
    if ((rc = settle(g, (hipStream_t)stream)) != FSPB_OK) return rc;
    if (!fluence || !prm || !dose) return fail(FSPB_E_ARG, "forward_surrogate: NULL argument");
    launch_forward_surrogate(g->args(), g->tile, g->order, fluence, (const float4*)prm, dose,
                             (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

}  // extern "C"

// ===========================================================================
// Gamma index.
extern "C" int fspb_gamma(const float* ref, const float* eval, int nx, int ny, int nz, float dx,
                          float dy, float dz, const fspb_gamma_params* params, float* gamma,
                          fspb_gamma_stats* stats, void* stream) {
    if (!ref || !eval) return fail(FSPB_E_ARG, "gamma: NULL dose grid");
    if (nx < 1 || ny < 1 || nz < 1) return fail(FSPB_E_ARG, "gamma: grid sizes must be >= 1");
    const long long nv = (long long)nx * ny * nz;
    if (nv > (1LL << 31) - 1) return fail(FSPB_E_ARG, "gamma: grid of %lld voxels exceeds 2^31-1", nv);
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
        return fail(FSPB_E_ARG, "gamma: voxel spacing must be finite and > 0");
    fspb_gamma_params p{};
    if (params) p = *params;
    if (p.dist == 0) p.dist = 0.3f;
    if (p.dose_frac == 0) p.dose_frac = 0.03f;
    if (p.gamma_cap == 0) p.gamma_cap = 5.0f;
    if (p.iso_frac == 0) p.iso_frac = 0.5f;
    if (!finite_pos(p.dist) || !finite_pos(p.dose_frac) || !finite_pos(p.gamma_cap) ||
        !isfinite(p.dose_max) || !isfinite(p.iso_frac))
        return fail(FSPB_E_ARG, "gamma: criteria must be finite and > 0");
    // offsets of the search sphere, shortest first
    const double R = (double)p.gamma_cap * p.dist;
    const int mx = (int)floor(R / dx), my = (int)floor(R / dy), mz = (int)floor(R / dz);
    struct Off {
        int i, j, k;
        double d2;
    };
    std::vector<Off> offs;
    for (int k = -mz; k <= mz; ++k)
        for (int j = -my; j <= my; ++j)
            for (int i = -mx; i <= mx; ++i) {
                const double d2 = (i * (double)dx) * (i * (double)dx) + (j * (double)dy) * (j * (double)dy) +
                                  (k * (double)dz) * (k * (double)dz);
                if (d2 <= R * R) offs.push_back({i, j, k, d2});
            }
    if ((int)offs.size() > kMaxGammaOffsets)
        return fail(FSPB_E_ARG, "gamma: search sphere of %zu offsets exceeds %d (reduce the cap)",
                    offs.size(), kMaxGammaOffsets);
    std::stable_sort(offs.begin(), offs.end(), [](const Off& a, const Off& b) { return a.d2 < b.d2; });
    std::vector<int4> hoff(offs.size());
    const double inv_dd2 = 1.0 / ((double)p.dist * p.dist);
    for (size_t q = 0; q < offs.size(); ++q) {
        const float d2 = (float)(offs[q].d2 * inv_dd2);
        int bits;
        memcpy(&bits, &d2, 4);
        hoff[q] = make_int4(offs[q].i, offs[q].j, offs[q].k, bits);
    }
    int dev = 0, rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int n_part = 512;
    struct Scratch {
        int dev;
        std::vector<std::pair<void*, size_t>> b;
        ~Scratch() {
            for (auto& x : b) pool_free(dev, x.first, x.second);
        }
        int get(void** p, size_t bytes) {
            size_t cls = 0;
            int r = pool_alloc(dev, p, bytes, &cls);
            if (r == FSPB_OK) b.push_back({*p, cls});
            return r;
        }
    } S{dev, {}};
    int4* doff = nullptr;
    float* fpart = nullptr;
    float* dmax = nullptr;
    GammaPart* gpart = nullptr;
    GammaPart* gout = nullptr;
    float* g = gamma;
    if ((rc = S.get((void**)&doff, sizeof(int4) * hoff.size())) ||
        (rc = S.get((void**)&fpart, sizeof(float) * n_part)) ||
        (rc = S.get((void**)&dmax, sizeof(float))) ||
        (rc = S.get((void**)&gpart, sizeof(GammaPart) * n_part)) ||
        (rc = S.get((void**)&gout, sizeof(GammaPart))) || (!g && (rc = S.get((void**)&g, sizeof(float) * nv))))
        return rc;
    HIP_TRY(hipMemcpyAsync(doff, hoff.data(), sizeof(int4) * hoff.size(), hipMemcpyHostToDevice, s));
    float D = p.dose_max;
    if (!(D > 0.0f)) {
        launch_grid_max(ref, (long)nv, fpart, n_part, dmax, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&D, dmax, sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!(D > 0.0f)) return fail(FSPB_E_ARG, "gamma: the reference dose has no positive value");
    }
    GammaArgs a;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    const double dD = (double)p.dose_frac * D;
    a.inv_dD2 = (float)(1.0 / (dD * dD));
    a.cap2 = p.gamma_cap * p.gamma_cap;
    a.n_off = (int)hoff.size();
    launch_gamma(ref, eval, doff, a, g, s);
    HIP_TRY(hipGetLastError());
    GammaPart h{};
    if (stats) {
        launch_gamma_stats(g, ref, (long)nv, p.iso_frac * D, gpart, n_part, gout, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&h, gout, sizeof(GammaPart), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));   // scratch goes back to the pool after this
    if (stats) {
        stats->gamma_max = h.max;
        stats->n_iso = h.n;
        stats->gamma_avg_iso = h.n ? h.sum / (double)h.n : 0.0;
        stats->pass_rate_iso = h.n ? (double)h.pass / (double)h.n : 0.0;
        stats->dose_max = D;
    }
    return FSPB_OK;
}
