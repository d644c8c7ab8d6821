// fspb_api.hip -- host side of libfspb: the geometry handle's entry points
// of the C ABI in include/fspb.h (creation, forward, adjoint, pair counts,
// inspection, tiling and schedules, density updates, release) and the
// device-memory pool and table sets behind them.  The batch, surrogate and
// gamma entry points are in api_batch.hip, api_mlp.hip and api_gamma.hip;
// error reporting and the shared checks in api_common.hip.
//
// Responsibilities: argument validation (pure host, before any HIP call),
// device buffers owned by the geometry handle, packing of the commissioned
// tables into the layouts the kernels read, and kernel launches.  All of the
// method's per-voxel and per-beamlet arithmetic runs in the kernels.
#include "api_internal.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <deque>
#include <functional>
#include <map>
#include <new>

namespace fspb {

namespace {

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

}  // namespace

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
    if (e == hipSuccess) log_msg(2, "pool: %zu bytes from the HIP runtime on device %d", cls, dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        log_msg(2, "pool: hipMalloc of %zu bytes failed; returning cached blocks of device %d", cls, dev);
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

std::mutex g_tables_mu;

namespace {

constexpr int kMaxIdleTableSets = 8;
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

}  // namespace

}  // namespace fspb

// Waits (on the host) for the handle's creation work.
int settle_host(fspb_geometry* g) {
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
int settle(fspb_geometry* g, hipStream_t s) {
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

int fetch_cost(fspb_geometry* G, hipStream_t s) {
    if (G->h_cost_valid) return FSPB_OK;
    const long nb = brick_count(G->P, G->tile.shape);
    G->h_cost.assign(nb, 0);
    HIP_TRY(hipMemcpyAsync(G->h_cost.data(), G->cost, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    G->h_cost_valid = true;
    return FSPB_OK;
}

extern "C" {


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
                (rc = G->alloc((void**)&G->split.queue, sizeof(int) * 8 * kSplitQueueInts)) != FSPB_OK ||
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
    G->n_cu = device_cu_count(dev);
    rc = create_impl(ct, n_beams, beams, tables, opts, (hipStream_t)stream, G);
    if (rc) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        G->release();
        delete G;
        return rc;
    }
    *out = G;
    log_msg(2, "geometry %p: %dx%dx%d voxels, %d beams, %d beamlets, %s, %s tables, tile %d/%d waves, "
               "%s schedule, device %d", (void*)G, G->P.nx, G->P.ny, G->P.nz, n_beams, G->n_beamlets,
            G->dc_enabled ? "DC" : "plain", G->siddon ? "exact" : "uniform", G->tile.shape,
            G->tile.waves_per_block, G->tile.per_beam ? "per-beam" : "brick-major", dev);
    clear_last_error();
    return FSPB_OK;
}

// The forward of a handle, with its depth tables' kind.
static void enqueue_forward(fspb_geometry* g, const float* fluence, float* dose, hipStream_t s) {
    if (g->siddon)
        launch_forward_siddon(g->args(), g->dc_enabled != 0, g->tile, g->order, fluence, dose, s);
    else if (g->tile.per_beam)
        launch_forward_split(g->args(), g->dc_enabled != 0, g->tile, g->split, fluence, g->planes,
                             dose, g->n_cu, s);
    else
        launch_forward(g->args(), g->dc_enabled != 0, g->tile, g->order, fluence, dose, s);
}

int fspb_forward(fspb_geometry* g, const float* fluence, float* dose, void* stream) {
    if (!g || !fluence || !dose) return fail(FSPB_E_ARG, "forward: NULL argument");
    int rc = settle(g, (hipStream_t)stream);
    if (rc) return rc;
    enqueue_forward(g, fluence, dose, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    log_msg(3, "forward: geometry %p, stream %p", (void*)g, stream);
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
    log_msg(3, "adjoint: geometry %p, stream %p, %d-plane slabs", (void*)g, stream, adj_slab_of(g));
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
    log_msg(2, "geometry %p released", (void*)g);
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
    log_msg(2, "pool: %zu cached blocks returned to the HIP runtime", drop.size());
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
    log_msg(2, "autotune: geometry %p, %d configurations timed, best %s schedule, shape %d, "
               "%d waves per workgroup, %.4f ms", (void*)g, n,
            best.per_beam ? "per-beam" : "brick-major", best.shape, best.waves_per_block, best_ms);
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
    log_msg(2, "autotune_adjoint: geometry %p, %d thicknesses timed, best %d planes, %.4f ms",
            (void*)g, n, best, best_ms);
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

