// Batched frames: every view's rays in ONE traversal launch, every display
// in ONE reconstruction launch, optionally replayed from a hipGraph whose
// node parameters are updated per frame, and an autotuner for the launch
// shape.  Path-mode views run in phases: bounces 0-1 in the traversal
// launch, each later bounce in a launch of its own over the paths still
// alive (a compacted list per view), so that the waves of those launches
// are full of live paths; between bounces every path's state lives in
// memory, so none is held in registers across a traversal.
//
// Per frame the host writes the view descriptors into one slot of a ring of
// pinned staging buffers; the slot is copied to its device twin on the
// stream ahead of the kernels, and an event marks when the slot may be
// reused.  With four slots the host runs up to three frames ahead.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "vafr_internal.h"

namespace vafr {
namespace {

constexpr int kSlots = 4;
constexpr int kMaxBatchViews = 256;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Slot {
    char* host = nullptr;   // pinned staging
    char* dev = nullptr;    // device twin
    int32_t* order = nullptr;   // planned dispatch order of this slot's traversal launch
    float4* state = nullptr;    // path state of the phased path-mode views (4 float4 per path)
    int32_t* list = nullptr;    // two lists of path ids per path-mode view
    int64_t state_cap = 0;      // capacity in paths
    hipEvent_t done = nullptr;
    bool used = false;
    uint64_t frame = 0;         // number of the frame that last used the slot
    // stage timing (when profiling): before upload, after upload, after
    // traversal, after reconstruction
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
};

// A graph for one launch shape.
struct GraphEntry {
    int n_trace = 0, n_recon = 0, trace_blocks = 0, recon_blocks = 0, trace_block = 0, recon_rows = 0, stack = 0;
    int queue_blocks = 0, bounces = 0;   // queue launches: one per bounce 1 .. bounces
    bool lambert = false;   // traversal kernel without the path-tracing code
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr, kplan = nullptr, ktrace = nullptr, krecon = nullptr;
    hipGraphNode_t kqueue[vafr::kMaxBounces] = {};
    bool timed = false;
    hipGraphNode_t evn[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t last_frame = 0;   // frame that last launched the graph, and its slot
    int last_slot = -1;
};

// Launch shapes kept as graphs; past this the least recently used goes.
constexpr size_t kGraphCache = 32;

}  // namespace
}  // namespace vafr

struct vafr_batch_s {
    int32_t max_views = 0;
    vafr_batch_config cfg{vafr::kTraceBlockDefault, vafr::kBatchReconRowsDefault, 1};
    int device = -1;
    // staging layout: TraceView[], traversal block ends, ReconView[],
    // reconstruction block ends, queue-pass block ends, per view the counts
    // of listed paths per bounce (they stay zero on the host, so every
    // upload clears them)
    size_t off_tb = 0, off_rv = 0, off_rb = 0, off_qb = 0, off_qc = 0, bytes = 0;
    vafr::Slot slot[vafr::kSlots];
    int next = 0;
    uint64_t frames = 0;             // frames run so far
    std::vector<vafr::GraphEntry> graphs;
    std::mutex mu;
    // host-side descriptors of the frame being prepared
    std::vector<vafr::TraceView> tv;
    std::vector<vafr::ReconView> rv;
    int stack = vafr::kStackShort;   // stack class of the frame's traversal launch
    bool lambert = true;             // no view of the frame is path-traced
    std::vector<int32_t> tb, rb, qb;
    std::vector<int64_t> qoff;       // first path-state entry of each view
    int64_t queue_items = 0;         // path-state entries the frame needs
    int bounces = 0;                 // most bounces of a path-mode view of the frame
    bool profiling = false;
    double stage_sum[3] = {0, 0, 0};   // accumulated stage times (ms)
    int64_t stage_frames = 0;
    // longest-first dispatch: block durations of the last traversal launch
    // (shared by the slots; only an ordering hint) and the capacity of it
    // and of every slot's order buffer, in blocks
    uint32_t* cost = nullptr;
    int32_t plan_cap = 0;
};

namespace vafr {
namespace {

int check_config(const vafr_batch_config* c) {
    if (!trace_block_ok(c->trace_block)) return fail(VAFR_E_ARG, "trace_block must be 64, 128 or 256");
    if (!recon_rows_ok(c->recon_rows)) return fail(VAFR_E_ARG, "recon_rows must be 1, 2, 4 or 8");
    if (c->use_graph != 0 && c->use_graph != 1) return fail(VAFR_E_ARG, "use_graph must be 0 or 1");
    return VAFR_OK;
}

void free_graphs(vafr_batch b) {
    for (auto& g : b->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    b->graphs.clear();
}

// Views whose reconstruction can share one pass: VaFR views with the same
// layout tables, gaze and display (the two eyes of a binocular frame), the
// first not yet paired.
bool pairable(const ReconView& a, const ReconView& b) {
    return a.mode == kModeVafr && b.mode == kModeVafr && !a.lp2 && a.u_of_rho == b.u_of_rho && a.col == b.col &&
           a.n_cols == b.n_cols && a.lp_bytes == b.lp_bytes && a.width == b.width && a.height == b.height &&
           a.sx == b.sx && a.sy == b.sy && a.cx == b.cx && a.cy == b.cy && a.rho_scale == b.rho_scale &&
           a.img != b.img;
}

// Descriptors of one frame into b->tv/tb/rv/rb.  A view whose reconstruction
// pairs with the previous reconstruction descriptor rides along in it.
int describe(vafr_batch b, const vafr_view* views, int32_t n, int32_t* trace_blocks, int32_t* recon_blocks,
             int32_t* queue_blocks) {
    b->tv.clear();
    b->rv.clear();
    b->tb.clear();
    b->rb.clear();
    b->qb.clear();
    b->qoff.clear();
    b->queue_items = 0;
    b->bounces = 0;
    int64_t tsum = 0, rsum = 0, qsum = 0;
    b->stack = kStackShort;
    b->lambert = true;
    for (int32_t i = 0; i < n; ++i) {
        const vafr_view& w = views[i];
        TraceView t;
        int rc;
        if (w.kind == VAFR_VIEW_FULL) {
            if (!w.img_rgba_dev) return fail(VAFR_E_ARG, "view %d: img_rgba_dev is NULL", i);
            rc = make_trace_view(-1, w.scene, &w.camera, w.gaze, &w.shading, nullptr, &w.display, w.img_rgba_dev,
                                 w.hit_id_dev, &t);
        } else if (w.kind == VAFR_VIEW_VAFR || w.kind == VAFR_VIEW_LMFR || w.kind == VAFR_VIEW_LAFR) {
            if (!w.lp_rgba_dev) return fail(VAFR_E_ARG, "view %d: lp_rgba_dev is NULL", i);
            const int lk = w.kind == VAFR_VIEW_VAFR ? VAFR_LAYOUT_VAFR
                         : w.kind == VAFR_VIEW_LMFR ? VAFR_LAYOUT_LMFR : VAFR_LAYOUT_LAFR;
            rc = make_trace_view(lk, w.scene, &w.camera,
                                 w.gaze, &w.shading, w.layout, nullptr, w.lp_rgba_dev, w.hit_id_dev, &t);
        } else {
            return fail(VAFR_E_ARG, "view %d: unknown kind %d", i, w.kind);
        }
        if (rc) return rc;
        tsum += (t.n_items + b->cfg.trace_block - 1) / b->cfg.trace_block;
        if (tsum > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "too many rays in one batch");
        b->stack = std::max(b->stack, (int)t.stack);
        // path mode runs in phases (state and list pointers are filled in
        // per slot)
        b->qoff.push_back(b->queue_items);
        if (t.shade_mode == VAFR_SHADE_PATH) {
            if (t.n_items > 0x7fffffff)
                return fail(VAFR_E_UNSUPPORTED, "view %d: path-mode views hold fewer than 2^31 rays", i);
            b->lambert = false;
            t.pt_phased = 1;
            b->queue_items += t.n_items;
            b->bounces = std::max(b->bounces, (int)t.bounces);
            if (t.bounces > kPathFuse) qsum += (t.n_items + kQueueBlock - 1) / kQueueBlock;
            if (qsum > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "too many rays in one batch");
        }
        b->qb.push_back((int32_t)qsum);
        b->tv.push_back(t);
        b->tb.push_back((int32_t)tsum);
        if (w.kind != VAFR_VIEW_FULL && w.img_rgba_dev) {
            ReconView r;
            if (int rc2 = make_recon_view(w.layout, w.gaze, w.lp_rgba_dev, w.img_rgba_dev, &r)) return rc2;
            if (!b->rv.empty() && pairable(b->rv.back(), r)) {
                b->rv.back().lp2 = r.lp;
                b->rv.back().img2 = r.img;
                continue;
            }
            rsum += recon_blocks_of(r, b->cfg.recon_rows);
            if (rsum > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "too many pixels in one batch");
            b->rv.push_back(r);
            b->rb.push_back((int32_t)rsum);
        }
    }
    *trace_blocks = (int32_t)tsum;
    *recon_blocks = (int32_t)rsum;
    *queue_blocks = (int32_t)qsum;
    return VAFR_OK;
}

// Room for the state and lists of `items` paths in slot s (the slot is idle
// when called).
int ensure_state(Slot& s, int64_t items) {
    if (items <= s.state_cap) return VAFR_OK;
    (void)hipFree(s.state);
    (void)hipFree(s.list);
    s.state = nullptr;
    s.list = nullptr;
    s.state_cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&s.state), 4 * sizeof(float4) * (size_t)items) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s.list), 2 * sizeof(int32_t) * (size_t)items) != hipSuccess)
        return fail(VAFR_E_OOM, "path state allocation failed");
    s.state_cap = items;
    return VAFR_OK;
}

// Kernel arguments of one queue launch (bounce >= 1); the pointed-to values
// must outlive the call that consumes the parameters.
struct QueueArgs {
    const TraceView* v;
    const int32_t* qe;
    int32_t n;
    int32_t bounce;
    void* p[4];
};

hipKernelNodeParams queue_params(vafr_batch b, const GraphEntry& g, char* dev, int bounce, QueueArgs& a) {
    a.v = reinterpret_cast<const TraceView*>(dev);
    a.qe = reinterpret_cast<const int32_t*>(dev + b->off_qb);
    a.n = g.n_trace;
    a.bounce = bounce;
    a.p[0] = &a.v;
    a.p[1] = &a.qe;
    a.p[2] = &a.n;
    a.p[3] = &a.bounce;
    void** args = a.p;
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(trace_queue_batch_kernel(g.stack));
    p.gridDim = dim3((unsigned)g.queue_blocks);
    p.blockDim = dim3((unsigned)kQueueBlock);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

// Kernel arguments of a batched traversal node; the pointed-to values must
// outlive the call that consumes the parameters.
struct TraceArgs {
    const TraceView* v;
    const int32_t* be;
    int32_t n;
    unsigned long long* cnt;
    const int32_t* order;
    uint32_t* cost;
    void* p[6];
};

hipKernelNodeParams trace_params(vafr_batch b, const GraphEntry& g, const Slot& s, TraceArgs& a) {
    a.v = reinterpret_cast<const TraceView*>(s.dev);
    a.be = reinterpret_cast<const int32_t*>(s.dev + b->off_tb);
    a.n = g.n_trace;
    a.cnt = nullptr;
    const bool planned = trace_plan_ok(g.trace_blocks);
    a.order = planned ? s.order : nullptr;
    a.cost = planned ? b->cost : nullptr;
    a.p[0] = &a.v;
    a.p[1] = &a.be;
    a.p[2] = &a.n;
    a.p[3] = &a.cnt;
    a.p[4] = &a.order;
    a.p[5] = &a.cost;
    void** args = a.p;
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(trace_batch_kernel(g.trace_block, g.stack, !g.lambert, g.lambert));
    p.gridDim = dim3((unsigned)g.trace_blocks);
    p.blockDim = dim3((unsigned)g.trace_block);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

struct PlanArgs {
    uint32_t* cost;
    int32_t* order;
    int32_t blocks;
    void* p[3];
};

hipKernelNodeParams plan_params(vafr_batch b, const GraphEntry& g, const Slot& s, PlanArgs& a) {
    a.cost = b->cost;
    a.order = s.order;
    a.blocks = g.trace_blocks;
    a.p[0] = &a.cost;
    a.p[1] = &a.order;
    a.p[2] = &a.blocks;
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(trace_plan_kernel());
    p.gridDim = dim3(8u);
    p.blockDim = dim3(1024u);
    p.sharedMemBytes = 0;
    p.kernelParams = a.p;
    p.extra = nullptr;
    return p;
}

// Makes room for a traversal launch of `blocks` workgroups in the duration
// buffer and in every slot's order buffer (waits for the slots in flight and
// drops the graphs, which hold the old addresses, when it grows).
int ensure_plan(vafr_batch b, int32_t blocks) {
    if (blocks <= b->plan_cap) return VAFR_OK;
    for (auto& sl : b->slot)
        if (sl.used) VAFR_HIP(hipEventSynchronize(sl.done));
    free_graphs(b);
    const int32_t cap = std::max(blocks, 2 * b->plan_cap);
    (void)hipFree(b->cost);
    b->cost = nullptr;
    for (auto& sl : b->slot) {
        (void)hipFree(sl.order);
        sl.order = nullptr;
    }
    b->plan_cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&b->cost), sizeof(uint32_t) * cap) != hipSuccess)
        return fail(VAFR_E_OOM, "dispatch plan allocation failed");
    VAFR_HIP(hipMemset(b->cost, 0, sizeof(uint32_t) * cap));
    for (auto& sl : b->slot)
        if (hipMalloc(reinterpret_cast<void**>(&sl.order), sizeof(int32_t) * cap) != hipSuccess)
            return fail(VAFR_E_OOM, "dispatch plan allocation failed");
    b->plan_cap = cap;
    return VAFR_OK;
}

hipKernelNodeParams recon_params(vafr_batch b, const GraphEntry& g, char* dev, void** args, const ReconView** v,
                                 const int32_t** be, int32_t* n) {
    *v = reinterpret_cast<const ReconView*>(dev + b->off_rv);
    *be = reinterpret_cast<const int32_t*>(dev + b->off_rb);
    *n = g.n_recon;
    args[0] = v;
    args[1] = be;
    args[2] = n;
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(recon_batch_kernel(g.recon_rows));
    p.gridDim = dim3((unsigned)g.recon_blocks);
    p.blockDim = dim3((unsigned)kReconThreads);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

int graph_for(vafr_batch b, int32_t trace_blocks, int32_t recon_blocks, int32_t queue_blocks, Slot& s,
              GraphEntry** out) {
    const int nt = (int)b->tv.size(), nr = (int)b->rv.size();
    for (auto& g : b->graphs)
        if (g.n_trace == nt && g.n_recon == nr && g.trace_blocks == trace_blocks && g.recon_blocks == recon_blocks &&
            g.queue_blocks == queue_blocks && g.bounces == (queue_blocks > 0 ? b->bounces : 0) &&
            g.lambert == b->lambert && g.trace_block == b->cfg.trace_block &&
            g.recon_rows == b->cfg.recon_rows && g.stack == b->stack && g.timed == b->profiling) {
            *out = &g;
            return VAFR_OK;
        }
    if (b->graphs.size() >= kGraphCache) {
        // Evict the least recently used shape.  Its last launch can only be
        // in flight if its slot has not been reused since, so at most that
        // one frame is waited for (serving mixes change the launch shape
        // often; waiting for every frame in flight here would stall the
        // caller for several frames).
        auto victim = std::min_element(b->graphs.begin(), b->graphs.end(), [](const GraphEntry& x,
                                                                              const GraphEntry& y) {
            return x.last_frame < y.last_frame;
        });
        if (victim->last_slot >= 0) {
            const Slot& sl = b->slot[victim->last_slot];
            if (sl.used && sl.frame == victim->last_frame) VAFR_HIP(hipEventSynchronize(sl.done));
        }
        if (victim->exec) (void)hipGraphExecDestroy(victim->exec);
        if (victim->graph) (void)hipGraphDestroy(victim->graph);
        b->graphs.erase(victim);
    }
    GraphEntry g;
    g.n_trace = nt;
    g.n_recon = nr;
    g.trace_blocks = trace_blocks;
    g.recon_blocks = recon_blocks;
    g.queue_blocks = queue_blocks;
    g.bounces = queue_blocks > 0 ? b->bounces : 0;
    g.lambert = b->lambert;
    g.trace_block = b->cfg.trace_block;
    g.recon_rows = b->cfg.recon_rows;
    g.stack = b->stack;
    g.timed = b->profiling;
    VAFR_HIP(hipGraphCreate(&g.graph, 0));
    hipError_t e = hipSuccess;
    if (g.timed) e = hipGraphAddEventRecordNode(&g.evn[0], g.graph, nullptr, 0, s.ev[0]);
    if (e == hipSuccess)
        e = hipGraphAddMemcpyNode1D(&g.copy, g.graph, g.evn[0] ? &g.evn[0] : nullptr, g.evn[0] ? 1 : 0, s.dev, s.host,
                                    b->bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && g.timed) e = hipGraphAddEventRecordNode(&g.evn[1], g.graph, &g.copy, 1, s.ev[1]);
    TraceArgs ta;
    PlanArgs pa;
    if (e == hipSuccess && trace_blocks > 0) {
        hipGraphNode_t dep = g.timed ? g.evn[1] : g.copy;
        if (trace_plan_ok(trace_blocks)) {
            hipKernelNodeParams pp = plan_params(b, g, s, pa);
            e = hipGraphAddKernelNode(&g.kplan, g.graph, &dep, 1, &pp);
            dep = g.kplan;
        }
        if (e == hipSuccess) {
            hipKernelNodeParams p = trace_params(b, g, s, ta);
            e = hipGraphAddKernelNode(&g.ktrace, g.graph, &dep, 1, &p);
        }
    }
    QueueArgs qa[kMaxBounces];
    hipGraphNode_t traced = g.ktrace;
    for (int k = kPathFuse + 1; e == hipSuccess && traced && k <= g.bounces; ++k) {
        hipKernelNodeParams p = queue_params(b, g, s.dev, k, qa[k - 1]);
        e = hipGraphAddKernelNode(&g.kqueue[k - 1], g.graph, &traced, 1, &p);
        traced = g.kqueue[k - 1];
    }
    if (e == hipSuccess && g.timed) {
        hipGraphNode_t dep = traced ? traced : g.evn[1];
        e = hipGraphAddEventRecordNode(&g.evn[2], g.graph, &dep, 1, s.ev[2]);
    }
    void* ra[3];
    const ReconView* rvp;
    const int32_t* rbe;
    int32_t rn;
    if (e == hipSuccess && recon_blocks > 0) {
        hipKernelNodeParams p = recon_params(b, g, s.dev, ra, &rvp, &rbe, &rn);
        hipGraphNode_t dep = g.timed ? g.evn[2] : (traced ? traced : g.copy);
        e = hipGraphAddKernelNode(&g.krecon, g.graph, &dep, 1, &p);
    }
    if (e == hipSuccess && g.timed) {
        hipGraphNode_t dep = g.krecon ? g.krecon : g.evn[2];
        e = hipGraphAddEventRecordNode(&g.evn[3], g.graph, &dep, 1, s.ev[3]);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g.graph) (void)hipGraphDestroy(g.graph);
        return hip_fail(e, "building the frame graph");
    }
    b->graphs.push_back(g);
    *out = &b->graphs.back();
    return VAFR_OK;
}

// Adds a finished timed frame's stage durations to the accumulators.
int fold_slot(vafr_batch b, Slot& s) {
    if (!s.used || !s.timed) return VAFR_OK;
    VAFR_HIP(hipEventSynchronize(s.ev[3]));
    for (int k = 0; k < 3; ++k) {
        float ms = 0.0f;
        VAFR_HIP(hipEventElapsedTime(&ms, s.ev[k], s.ev[k + 1]));
        b->stage_sum[k] += ms;
    }
    ++b->stage_frames;
    s.timed = false;
    return VAFR_OK;
}

// One frame with the batch's current configuration (caller holds b->mu).
int run_locked(vafr_batch b, const vafr_view* views, int32_t n, hipStream_t stream) {
    if (!views || n < 1 || n > b->max_views) return fail(VAFR_E_ARG, "n_views must be in [1, %d]", b->max_views);
    int dev = -1;
    VAFR_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(VAFR_E_ARG, "batch was created on device %d, current is %d", b->device, dev);
    int32_t tblocks = 0, rblocks = 0, qblocks = 0;
    if (int rc = describe(b, views, n, &tblocks, &rblocks, &qblocks)) return rc;
    // launches too large to plan keep the fixed XCD order
    const bool planned = trace_plan_ok(tblocks);
    if (planned)
        if (int rc = ensure_plan(b, tblocks)) return rc;
    const int si = b->next;
    Slot& s = b->slot[si];
    b->next = (b->next + 1) % kSlots;
    const uint64_t fno = ++b->frames;
    if (s.used) {
        VAFR_HIP(hipEventSynchronize(s.done));
        if (int rc = fold_slot(b, s)) return rc;
    }
    if (b->queue_items > 0) {
        if (int rc = ensure_state(s, b->queue_items)) return rc;
        uint32_t* counters = reinterpret_cast<uint32_t*>(s.dev + b->off_qc);
        for (size_t i = 0; i < b->tv.size(); ++i)
            if (b->tv[i].pt_phased) {
                b->tv[i].pt_state = s.state + 4 * b->qoff[i];
                b->tv[i].pt_list = s.list + 2 * b->qoff[i];
                b->tv[i].pt_count = counters + i * (kMaxBounces + 1);
            }
    }
    std::memcpy(s.host, b->tv.data(), sizeof(TraceView) * b->tv.size());
    std::memcpy(s.host + b->off_qb, b->qb.data(), sizeof(int32_t) * b->qb.size());
    std::memcpy(s.host + b->off_tb, b->tb.data(), sizeof(int32_t) * b->tb.size());
    if (!b->rv.empty()) {
        std::memcpy(s.host + b->off_rv, b->rv.data(), sizeof(ReconView) * b->rv.size());
        std::memcpy(s.host + b->off_rb, b->rb.data(), sizeof(int32_t) * b->rb.size());
    }
    if (b->cfg.use_graph) {
        GraphEntry* g;
        if (int rc = graph_for(b, tblocks, rblocks, qblocks, s, &g)) return rc;
        VAFR_HIP(hipGraphExecMemcpyNodeSetParams1D(g->exec, g->copy, s.dev, s.host, b->bytes, hipMemcpyHostToDevice));
        if (g->timed)
            for (int k = 0; k < 4; ++k) VAFR_HIP(hipGraphExecEventRecordNodeSetEvent(g->exec, g->evn[k], s.ev[k]));
        TraceArgs ta;
        PlanArgs pa;
        if (g->ktrace) {
            if (g->kplan) {
                hipKernelNodeParams pp = plan_params(b, *g, s, pa);
                VAFR_HIP(hipGraphExecKernelNodeSetParams(g->exec, g->kplan, &pp));
            }
            hipKernelNodeParams p = trace_params(b, *g, s, ta);
            VAFR_HIP(hipGraphExecKernelNodeSetParams(g->exec, g->ktrace, &p));
        }
        QueueArgs qa[kMaxBounces];
        for (int k = kPathFuse + 1; k <= g->bounces; ++k) {
            hipKernelNodeParams p = queue_params(b, *g, s.dev, k, qa[k - 1]);
            VAFR_HIP(hipGraphExecKernelNodeSetParams(g->exec, g->kqueue[k - 1], &p));
        }
        void* ra[3];
        const ReconView* rvp;
        const int32_t* rbe;
        int32_t rn;
        if (g->krecon) {
            hipKernelNodeParams p = recon_params(b, *g, s.dev, ra, &rvp, &rbe, &rn);
            VAFR_HIP(hipGraphExecKernelNodeSetParams(g->exec, g->krecon, &p));
        }
        VAFR_HIP(hipGraphLaunch(g->exec, stream));
        g->last_frame = fno;
        g->last_slot = si;
    } else {
        if (b->profiling) VAFR_HIP(hipEventRecord(s.ev[0], stream));
        VAFR_HIP(hipMemcpyAsync(s.dev, s.host, b->bytes, hipMemcpyHostToDevice, stream));
        if (b->profiling) VAFR_HIP(hipEventRecord(s.ev[1], stream));
        if (planned)
            if (int rc = launch_trace_plan(b->cost, s.order, tblocks, stream)) return rc;
        if (int rc = launch_trace_batch(reinterpret_cast<const TraceView*>(s.dev),
                                        reinterpret_cast<const int32_t*>(s.dev + b->off_tb), (int32_t)b->tv.size(),
                                        tblocks, b->cfg.trace_block, b->stack, !b->lambert, b->lambert, stream,
                                        nullptr,
                                        planned ? s.order : nullptr, planned ? b->cost : nullptr))
            return rc;
        for (int k = kPathFuse + 1; qblocks > 0 && k <= b->bounces; ++k)
            if (int rc = launch_trace_queue_batch(reinterpret_cast<const TraceView*>(s.dev),
                                                  reinterpret_cast<const int32_t*>(s.dev + b->off_qb),
                                                  (int32_t)b->tv.size(), qblocks, b->stack, k, stream))
                return rc;
        if (b->profiling) VAFR_HIP(hipEventRecord(s.ev[2], stream));
        if (int rc = launch_reconstruct_batch(reinterpret_cast<const ReconView*>(s.dev + b->off_rv),
                                              reinterpret_cast<const int32_t*>(s.dev + b->off_rb),
                                              (int32_t)b->rv.size(), rblocks, b->cfg.recon_rows, stream))
            return rc;
        if (b->profiling) VAFR_HIP(hipEventRecord(s.ev[3], stream));
    }
    VAFR_HIP(hipEventRecord(s.done, stream));
    s.used = true;
    s.frame = fno;
    s.timed = b->profiling;
    return VAFR_OK;
}

}  // namespace
}  // namespace vafr

using namespace vafr;

extern "C" int vafr_batch_create(int32_t max_views, const vafr_batch_config* cfg, vafr_batch* out) {
    if (!out) return fail(VAFR_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_views < 1 || max_views > kMaxBatchViews) return fail(VAFR_E_ARG, "max_views must be in [1, %d]", kMaxBatchViews);
    if (cfg)
        if (int rc = check_config(cfg)) return rc;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0) return fail(VAFR_E_HIP, "no HIP device available");
    vafr_batch b = new (std::nothrow) vafr_batch_s;
    if (!b) return fail(VAFR_E_OOM, "batch allocation failed");
    if (cfg) b->cfg = *cfg;
    b->max_views = max_views;
    b->off_tb = align256(sizeof(TraceView) * max_views);
    b->off_rv = b->off_tb + align256(sizeof(int32_t) * max_views);
    b->off_rb = b->off_rv + align256(sizeof(ReconView) * max_views);
    b->off_qb = b->off_rb + align256(sizeof(int32_t) * max_views);
    b->off_qc = b->off_qb + align256(sizeof(int32_t) * max_views);
    b->bytes = b->off_qc + align256(sizeof(uint32_t) * (kMaxBounces + 1) * max_views);
    auto bail = [&](int code) {
        vafr_batch_destroy(b);
        return code;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return bail(fail(VAFR_E_HIP, "hipGetDevice failed"));
    for (auto& s : b->slot) {
        if (hipHostMalloc(reinterpret_cast<void**>(&s.host), b->bytes, hipHostMallocDefault) != hipSuccess)
            return bail(fail(VAFR_E_OOM, "pinned staging allocation failed"));
        std::memset(s.host, 0, b->bytes);
        if (hipMalloc(reinterpret_cast<void**>(&s.dev), b->bytes) != hipSuccess)
            return bail(fail(VAFR_E_OOM, "device descriptor table allocation failed"));
        if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
            return bail(fail(VAFR_E_HIP, "event creation failed"));
        for (auto& ev : s.ev)
            if (hipEventCreate(&ev) != hipSuccess) return bail(fail(VAFR_E_HIP, "event creation failed"));
    }
    try {
        b->tv.reserve(max_views);
        b->rv.reserve(max_views);
        b->tb.reserve(max_views);
        b->rb.reserve(max_views);
        b->qb.reserve(max_views);
        b->qoff.reserve(max_views);
    } catch (const std::bad_alloc&) {
        return bail(fail(VAFR_E_OOM, "batch allocation failed"));
    }
    *out = b;
    return VAFR_OK;
}

extern "C" int vafr_batch_run(vafr_batch b, const vafr_view* views, int32_t n_views, hipStream_t stream) {
    if (!b) return fail(VAFR_E_ARG, "batch is NULL");
    std::lock_guard<std::mutex> lock(b->mu);
    return run_locked(b, views, n_views, stream);
}

extern "C" int vafr_batch_get_config(vafr_batch b, vafr_batch_config* out) {
    if (!b || !out) return fail(VAFR_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(b->mu);
    *out = b->cfg;
    return VAFR_OK;
}

extern "C" int vafr_batch_set_config(vafr_batch b, const vafr_batch_config* cfg) {
    if (!b || !cfg) return fail(VAFR_E_ARG, "NULL argument");
    if (int rc = check_config(cfg)) return rc;
    std::lock_guard<std::mutex> lock(b->mu);
    b->cfg = *cfg;
    return VAFR_OK;
}

extern "C" int vafr_batch_autotune(vafr_batch b, const vafr_view* views, int32_t n_views, int32_t reps,
                                   hipStream_t stream, vafr_batch_config* chosen) {
    if (!b) return fail(VAFR_E_ARG, "batch is NULL");
    if (reps < 1 || reps > 1000) return fail(VAFR_E_ARG, "reps must be in [1, 1000]");
    std::lock_guard<std::mutex> lock(b->mu);
    hipEvent_t e0, e1;
    VAFR_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VAFR_E_HIP, "event creation failed");
    }
    const vafr_batch_config start = b->cfg;
    auto time_cfg = [&](const vafr_batch_config& c, float* ms) -> int {
        b->cfg = c;
        if (int rc = run_locked(b, views, n_views, stream)) return rc;   // warm-up (and graph build)
        VAFR_HIP(hipEventRecord(e0, stream));
        for (int r = 0; r < reps; ++r)
            if (int rc = run_locked(b, views, n_views, stream)) return rc;
        VAFR_HIP(hipEventRecord(e1, stream));
        VAFR_HIP(hipEventSynchronize(e1));
        VAFR_HIP(hipEventElapsedTime(ms, e0, e1));
        return VAFR_OK;
    };
    int rc = VAFR_OK;
    vafr_batch_config best = start;
    float best_ms = 1e30f;
    // traversal workgroup size first (the reconstruction shape fixed), then
    // the reconstruction tile height with the chosen traversal shape
    for (int tbk : {64, 128, 256}) {
        vafr_batch_config c = best;
        c.trace_block = tbk;
        float ms;
        if ((rc = time_cfg(c, &ms))) break;
        if (ms < best_ms) { best_ms = ms; best = c; }
    }
    if (!rc) {
        const vafr_batch_config base = best;
        for (int rows : {1, 2, 4, 8}) {
            vafr_batch_config c = base;
            c.recon_rows = rows;
            if (c.recon_rows == base.recon_rows) continue;
            float ms;
            if ((rc = time_cfg(c, &ms))) break;
            if (ms < best_ms) { best_ms = ms; best = c; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->cfg = rc ? start : best;
    if (!rc && chosen) *chosen = best;
    return rc;
}

extern "C" int vafr_batch_set_profiling(vafr_batch b, int32_t on) {
    if (!b) return fail(VAFR_E_ARG, "batch is NULL");
    if (on != 0 && on != 1) return fail(VAFR_E_ARG, "on must be 0 or 1");
    std::lock_guard<std::mutex> lock(b->mu);
    for (auto& s : b->slot) {
        if (s.used) VAFR_HIP(hipEventSynchronize(s.done));
        s.timed = false;
    }
    b->profiling = on == 1;
    b->stage_sum[0] = b->stage_sum[1] = b->stage_sum[2] = 0.0;
    b->stage_frames = 0;
    return VAFR_OK;
}

extern "C" int vafr_batch_stage_ms(vafr_batch b, float* mean3, int64_t* frames) {
    if (!b || !mean3) return fail(VAFR_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(b->mu);
    for (auto& s : b->slot)
        if (int rc = fold_slot(b, s)) return rc;
    if (frames) *frames = b->stage_frames;
    for (int k = 0; k < 3; ++k) mean3[k] = b->stage_frames ? (float)(b->stage_sum[k] / b->stage_frames) : 0.0f;
    return VAFR_OK;
}

extern "C" void vafr_batch_destroy(vafr_batch b) {
    if (!b) return;
    int cur = -1;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (b->device >= 0) (void)hipSetDevice(b->device);
    for (auto& s : b->slot) {
        if (s.done) {
            if (s.used) (void)hipEventSynchronize(s.done);
            (void)hipEventDestroy(s.done);
        }
        for (auto& ev : s.ev)
            if (ev) (void)hipEventDestroy(ev);
        if (s.dev) (void)hipFree(s.dev);
        if (s.order) (void)hipFree(s.order);
        if (s.state) (void)hipFree(s.state);
        if (s.list) (void)hipFree(s.list);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (b->cost) (void)hipFree(b->cost);
    free_graphs(b);
    if (have) (void)hipSetDevice(cur);
    delete b;
}
