// api_internal.h -- what the host-side sources of the C ABI share: error
// reporting, the per-device caching pool of device memory, the device
// checks, the commissioned-table sets and the geometry handle (the struct
// behind include/fspb.h's opaque fspb_geometry).  Host code only.
#pragma once

#include "fspb.h"
#include "kernels.h"

#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace fspb {

// Records a printf-style message for fspb_last_error (per thread) and
// returns code.
int fail(int code, const char* fmt, ...);
// Diagnostic line on stderr when the log level (fspb_set_log_level,
// FSPB_LOG_LEVEL) is at least `level`.
int log_level();
void log_msg(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_last_error();

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(FSPB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// Device memory from the per-device caching pool (sizes rounded up to
// classes at most 1/8 above the request; *cls_out gets the class size, which
// pool_free takes back).
int pool_alloc(int dev, void** p, size_t bytes, size_t* cls_out);
void pool_free(int dev, void* p, size_t cls);

bool finite_pos(float v);
// A table is usable: n >= 1 values, finite start, step > 0 when n > 1.
int check_table(const fspb_table1d& t, const char* name);
// The current device, which must be a gfx950 (FSPB_E_UNSUPPORTED otherwise).
int check_device(int* dev);
// Compute units of a device that passed check_device (cached; 0 if unknown).
int device_cu_count(int dev);
// The current device is dev (FSPB_E_STATE otherwise).
int check_same_device(int dev, const char* what);

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

extern std::mutex g_tables_mu;   // guards the table sets and their use counts

}  // namespace fspb

using namespace fspb;

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

// Waits on the host for the handle's creation work.
int settle_host(fspb_geometry* g);
// Orders work on stream s after the handle's creation work.
int settle(fspb_geometry* g, hipStream_t s);
// Host copy of the brick costs for the batch scheduler (synchronises s).
int fetch_cost(fspb_geometry* G, hipStream_t s);
