// api_batch.hip -- host side of libfspb: the batch entry points of the C
// ABI (many plans in one persistent launch, captured into a HIP graph with
// their density updates).
#include "api_internal.h"

#include <algorithm>
#include <queue>
#include <vector>

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
    log_msg(2, "batch %p: %d plans, %zu work items over %d waves, shape %d, %d waves per workgroup, "
               "%s policy", (void*)B, n, flat.size(), B->n_waves, shape, waves_per_block,
            policy == FSPB_SCHEDULE_LATENCY ? "latency" : "throughput");
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
    log_msg(3, "batch_replay: batch %p, stream %p", (void*)b, stream);
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

