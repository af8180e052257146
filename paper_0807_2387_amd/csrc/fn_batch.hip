// Batches of independent point sets (one mesh each) and HIP-graph capture of
// evaluation sequences.
//
// A batch holds one context per member with their workspaces carved from one
// caller buffer; inputs and outputs are the members' arrays concatenated (CSR
// offsets).  Members may use different parameters (the grid is normally chosen per
// member from its size).  An evaluation is a set of tasks (a member's forward, its H
// adjoint or its phi adjoint; a member's forward and adjoints use separate scratch)
// spread over a few lanes -- streams the batch owns, forked from the batch stream with
// one event and joined back with one event per lane -- by longest-processing-time
// first on a cost model (near-field pairs, points, grid cells), so the kernels of small
// members run side by side instead of leaving most CUs idle one after the other.  The
// call stays ordered on the batch stream, and a whole batch evaluation records into a
// single graph (fn_graph_*) once the lanes exist.
#include "fn_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

struct fn_batch {
    hipStream_t stream = nullptr;
    int nlanes = 4;                    // lanes of an evaluation (fn_batch_set_lanes)
    std::vector<hipStream_t> lanes;    // created on the first evaluation, default priority
    std::vector<hipEvent_t> lane_ev;   // join event per lane
    hipEvent_t ev_fork = nullptr;
    std::vector<fn_ctx *> ctx;
    std::vector<int64_t> toff, soff;  // host copies of the offsets of the last geometry
    std::vector<size_t> wsoff;        // workspace offset of each member
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool geom_ready = false;
    std::string err;
};

struct fn_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static thread_local std::string g_batch_create_err;
static thread_local std::string g_graph_err;

#define BATCH_ERR(b, code, msg) \
    do {                        \
        (b)->err = (msg);       \
        return (code);          \
    } while (0)

static int member_err(fn_batch *b, int i, int rc)
{
    b->err = "member " + std::to_string(i) + ": " + fn_last_error(b->ctx[i]);
    return rc;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static int batch_layout(fn_batch *b, const int64_t *toff, const int64_t *soff, std::vector<size_t> *offs, size_t *total)
{
    const int B = (int)b->ctx.size();
    if (!toff || !soff) BATCH_ERR(b, FN_E_INVAL, "NULL offsets");
    if (toff[0] != 0 || soff[0] != 0) BATCH_ERR(b, FN_E_INVAL, "offsets must start at 0");
    size_t o = 0;
    if (offs) offs->assign(B, 0);
    for (int i = 0; i < B; ++i) {
        const int64_t nt = toff[i + 1] - toff[i], ns = soff[i + 1] - soff[i];
        if (nt < 0 || ns < 0) BATCH_ERR(b, FN_E_INVAL, "offsets must be non-decreasing");
        size_t by = 0;
        int rc = fn_workspace_size(b->ctx[i], nt, ns, &by);
        if (rc) return member_err(b, i, rc);
        if (offs) (*offs)[i] = o;
        o = al256(o + by);
    }
    *total = o;
    return FN_OK;
}

extern "C" {

int fn_batch_create(int32_t count, const fn_params *params, void *stream, fn_batch **out)
{
    if (!out) { g_batch_create_err = "out is NULL"; return FN_E_INVAL; }
    *out = nullptr;
    if (count < 1 || !params) { g_batch_create_err = "need count >= 1 and a params array"; return FN_E_INVAL; }
    fn_batch *b = new (std::nothrow) fn_batch();
    if (!b) { g_batch_create_err = "out of host memory"; return FN_E_NOMEM; }
    b->stream = static_cast<hipStream_t>(stream);
    for (int i = 0; i < count; ++i) {
        fn_ctx *c = nullptr;
        int rc = fn_create(&params[i], stream, &c);
        if (rc) {
            g_batch_create_err = "member " + std::to_string(i) + ": " + fn_last_error(nullptr);
            for (fn_ctx *x : b->ctx) fn_destroy(x);
            delete b;
            return rc;
        }
        b->ctx.push_back(c);
    }
    *out = b;
    return FN_OK;
}

int fn_batch_destroy(fn_batch *batch)
{
    if (batch) {
        for (fn_ctx *c : batch->ctx) fn_destroy(c);
        for (hipStream_t l : batch->lanes) {
            hipStreamSynchronize(l);
            hipStreamDestroy(l);
        }
        for (hipEvent_t e : batch->lane_ev) hipEventDestroy(e);
        if (batch->ev_fork) hipEventDestroy(batch->ev_fork);
    }
    delete batch;
    return FN_OK;
}

int fn_batch_workspace_size(fn_batch *batch, const int64_t *tgt_off, const int64_t *src_off, size_t *bytes)
{
    if (!batch || !bytes) return FN_E_INVAL;
    return batch_layout(batch, tgt_off, src_off, nullptr, bytes);
}

int fn_batch_set_workspace(fn_batch *batch, void *dev_ptr, size_t bytes)
{
    if (!batch) return FN_E_INVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255))
        BATCH_ERR(batch, FN_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    batch->ws = dev_ptr;
    batch->ws_bytes = bytes;
    batch->geom_ready = false;
    return FN_OK;
}

int fn_set_geometry_batch(fn_batch *batch, const int64_t *tgt_off, const double *tgt_xy, const int64_t *src_off,
                          const double *src_xy, const double *src_w)
{
    return fn_set_geometry_batch_split(batch, tgt_off, tgt_xy, src_off, src_xy, src_w, nullptr);
}

int fn_set_geometry_batch_split(fn_batch *batch, const int64_t *tgt_off, const double *tgt_xy,
                                const int64_t *src_off, const double *src_xy, const double *src_w,
                                const int64_t *n_surf)
{
    if (!batch) return FN_E_INVAL;
    fn_batch *b = batch;
    if (!b->ws) BATCH_ERR(b, FN_E_STATE, "fn_batch_set_workspace must be called before fn_set_geometry_batch");
    b->geom_ready = false;
    std::vector<size_t> offs;
    size_t total = 0;
    int rc = batch_layout(b, tgt_off, src_off, &offs, &total);
    if (rc) return rc;
    if (total > b->ws_bytes) BATCH_ERR(b, FN_E_NOMEM, "batch workspace too small");
    const int B = (int)b->ctx.size();
    char *base = static_cast<char *>(b->ws);
    for (int i = 0; i < B; ++i) {
        const int64_t nt = tgt_off[i + 1] - tgt_off[i], ns = src_off[i + 1] - src_off[i];
        const size_t sz = (i + 1 < B ? offs[i + 1] : total) - offs[i];
        rc = fn_set_workspace(b->ctx[i], base + offs[i], sz);
        if (rc) return member_err(b, i, rc);
        rc = fn_set_geometry_split(b->ctx[i], nt, nt ? tgt_xy + 2 * tgt_off[i] : nullptr, ns,
                                   ns ? src_xy + 2 * src_off[i] : nullptr, ns ? src_w + src_off[i] : nullptr,
                                   n_surf ? n_surf[i] : 0);
        if (rc) return member_err(b, i, rc);
    }
    b->toff.assign(tgt_off, tgt_off + B + 1);
    b->soff.assign(src_off, src_off + B + 1);
    b->wsoff = offs;
    b->geom_ready = true;
    return FN_OK;
}

int fn_batch_set_charges(fn_batch *batch, const double *q)
{
    if (!batch) return FN_E_INVAL;
    if (!batch->geom_ready) BATCH_ERR(batch, FN_E_STATE, "fn_set_geometry_batch must succeed first");
    for (size_t i = 0; i < batch->ctx.size(); ++i) {
        int rc = fn_set_charges(batch->ctx[i], q ? q + batch->soff[i] : nullptr);
        if (rc) return member_err(batch, (int)i, rc);
    }
    return FN_OK;
}

}  // extern "C"

namespace {

enum { TASK_FWD = 0, TASK_ADJ_H = 1, TASK_ADJ_PHI = 2 };
struct Task {
    int member, kind;
    double cost;
};

// Relative cost of a member's task: near-field pairs (the dominant work), points through
// spread and gather, grid cells through the FFT passes.
double task_cost(const fn_ctx *c, int kind)
{
    const double pairs = (double)c->geom.near_pairs + (double)c->geom.near_pairs_s;
    const double pts = (double)c->geom.nt + (double)c->geom.ns;
    const double G = c->plan.G, cells = (double)c->geom.ext[0] * c->geom.ext[1];
    const double lg = std::log2(G);
    return (kind == TASK_FWD ? 1.5 : 1.0) * pairs + 150.0 * pts + 60.0 * (cells + 0.5 * G * G / 4 * lg / 13.0);
}

// The lanes exist (created all or none, outside capture)
int ensure_lanes(fn_batch *b)
{
    if ((int)b->lanes.size() == b->nlanes && b->ev_fork) return FN_OK;
    if (stream_capturing(b->stream))
        BATCH_ERR(b, FN_E_STATE, "evaluate the batch once before capturing it (the first evaluation creates its lanes)");
    for (hipStream_t l : b->lanes) {
        hipStreamSynchronize(l);
        hipStreamDestroy(l);
    }
    for (hipEvent_t e : b->lane_ev) hipEventDestroy(e);
    b->lanes.clear();
    b->lane_ev.clear();
    hipError_t e = hipSuccess;
    if (!b->ev_fork) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    for (int l = 0; l < b->nlanes && e == hipSuccess; ++l) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (s) b->lanes.push_back(s);
        if (ev) b->lane_ev.push_back(ev);
    }
    if (e != hipSuccess || (int)b->lanes.size() != b->nlanes || (int)b->lane_ev.size() != b->nlanes) {
        for (hipStream_t l : b->lanes) hipStreamDestroy(l);
        for (hipEvent_t ev : b->lane_ev) hipEventDestroy(ev);
        b->lanes.clear();
        b->lane_ev.clear();
        BATCH_ERR(b, FN_E_DEVICE, std::string("creating the batch lanes: ") + hipGetErrorString(e));
    }
    return FN_OK;
}

// Enqueue the tasks over the lanes (longest first, each to the least loaded lane), forked
// from and joined back into the batch stream.  Arguments were checked by the caller.
int run_tasks(fn_batch *b, std::vector<Task> &tasks, double *phi, double *H, const double *in, int comps, double *u)
{
    int rc = ensure_lanes(b);
    if (rc) return rc;
    std::stable_sort(tasks.begin(), tasks.end(), [](const Task &x, const Task &y) { return x.cost > y.cost; });
    hipError_t e = hipEventRecord(b->ev_fork, b->stream);
    for (int l = 0; l < b->nlanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lanes[l], b->ev_fork, 0);
    if (e != hipSuccess) BATCH_ERR(b, FN_E_DEVICE, std::string("fork: ") + hipGetErrorString(e));
    std::vector<double> load(b->nlanes, 0.0);
    for (const Task &t : tasks) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[l] += t.cost;
        fn_ctx *c = b->ctx[t.member];
        const int64_t to = b->toff[t.member], so = b->soff[t.member];
        if (t.kind == TASK_FWD)
            rc = fn_internal_eval_on_stream(c, phi ? phi + to : nullptr, H ? H + 2 * to : nullptr, b->lanes[l]);
        else if (t.kind == TASK_ADJ_H)
            rc = fn_internal_adjoint_H_on_stream(c, in ? in + 2 * to : nullptr, u ? u + so : nullptr, b->lanes[l]);
        else
            rc = fn_internal_adjoint_phi_on_stream(c, in ? in + comps * to : nullptr, u ? u + so : nullptr, b->lanes[l]);
        if (rc) {
            rc = member_err(b, t.member, rc);
            break;
        }
    }
    // join every lane even after an error, so that the batch stream never runs ahead of it
    hipError_t ej = hipSuccess;
    for (int l = 0; l < b->nlanes; ++l) {
        const hipError_t e1 = hipEventRecord(b->lane_ev[l], b->lanes[l]);
        const hipError_t e2 = hipStreamWaitEvent(b->stream, b->lane_ev[l], 0);
        if (ej == hipSuccess) ej = e1 != hipSuccess ? e1 : e2;
    }
    if (rc) return rc;
    if (ej != hipSuccess) BATCH_ERR(b, FN_E_DEVICE, std::string("join: ") + hipGetErrorString(ej));
    return FN_OK;
}

// Batch-wide argument checks, before anything is enqueued.
int check_eval_args(fn_batch *b, bool fwd, bool need_phi_or_H, const void *phi, const void *H, bool adj,
                    const void *in, const void *u)
{
    if (!b->geom_ready) BATCH_ERR(b, FN_E_STATE, "fn_set_geometry_batch must succeed first");
    const size_t B = b->ctx.size();
    const int64_t nt = b->toff[B] - b->toff[0], ns = b->soff[B] - b->soff[0];
    if (fwd)
        for (size_t i = 0; i < B; ++i)
            if (!b->ctx[i]->charges_ready) {
                b->err = "member " + std::to_string(i) + ": fn_batch_set_charges must be called before evaluation";
                return FN_E_STATE;
            }
    if (fwd && need_phi_or_H && nt > 0 && !phi && !H) BATCH_ERR(b, FN_E_INVAL, "both outputs are NULL");
    if (adj && ((nt > 0 && !in) || (ns > 0 && !u))) BATCH_ERR(b, FN_E_INVAL, "NULL input or output");
    return FN_OK;
}

}  // namespace

extern "C" {

int fn_batch_set_lanes(fn_batch *batch, int32_t lanes)
{
    if (!batch) return FN_E_INVAL;
    if (lanes < 1 || lanes > 8) BATCH_ERR(batch, FN_E_INVAL, "lanes must be in [1, 8]");
    if (stream_capturing(batch->stream)) BATCH_ERR(batch, FN_E_STATE, "not during graph capture");
    batch->nlanes = lanes;
    return ensure_lanes(batch);
}

int fn_batch_eval(fn_batch *batch, double *phi, double *H)
{
    if (!batch) return FN_E_INVAL;
    int rc = check_eval_args(batch, true, true, phi, H, false, nullptr, nullptr);
    if (rc) return rc;
    std::vector<Task> tasks;
    for (size_t i = 0; i < batch->ctx.size(); ++i)
        if (batch->toff[i + 1] > batch->toff[i]) tasks.push_back({(int)i, TASK_FWD, task_cost(batch->ctx[i], TASK_FWD)});
    return run_tasks(batch, tasks, phi, H, nullptr, 0, nullptr);
}

static int batch_adjoint(fn_batch *batch, const double *in, int comps, double *u, bool h)
{
    if (!batch) return FN_E_INVAL;
    int rc = check_eval_args(batch, false, false, nullptr, nullptr, true, in, u);
    if (rc) return rc;
    std::vector<Task> tasks;
    const int kind = h ? TASK_ADJ_H : TASK_ADJ_PHI;
    for (size_t i = 0; i < batch->ctx.size(); ++i)
        if (batch->soff[i + 1] > batch->soff[i]) tasks.push_back({(int)i, kind, task_cost(batch->ctx[i], kind)});
    return run_tasks(batch, tasks, nullptr, nullptr, in, comps, u);
}

int fn_batch_eval_H_adjoint(fn_batch *batch, const double *V, double *u) { return batch_adjoint(batch, V, 2, u, true); }

int fn_batch_eval_with_H_adjoint(fn_batch *batch, double *phi, double *H, const double *V, double *u)
{
    if (!batch) return FN_E_INVAL;
    int rc = check_eval_args(batch, true, true, phi, H, true, V, u);
    if (rc) return rc;
    std::vector<Task> tasks;
    for (size_t i = 0; i < batch->ctx.size(); ++i) {
        if (batch->soff[i + 1] > batch->soff[i])
            tasks.push_back({(int)i, TASK_ADJ_H, task_cost(batch->ctx[i], TASK_ADJ_H)});
        if (batch->toff[i + 1] > batch->toff[i])
            tasks.push_back({(int)i, TASK_FWD, task_cost(batch->ctx[i], TASK_FWD)});
    }
    return run_tasks(batch, tasks, phi, H, V, 2, u);
}

int fn_batch_eval_phi_adjoint(fn_batch *batch, const double *v, double *u)
{
    return batch_adjoint(batch, v, 1, u, false);
}

int fn_batch_member(fn_batch *batch, int32_t i, fn_ctx **out)
{
    if (!batch || !out || i < 0 || i >= (int32_t)batch->ctx.size()) return FN_E_INVAL;
    *out = batch->ctx[i];
    return FN_OK;
}

const char *fn_batch_last_error(const fn_batch *batch)
{
    if (!batch) return g_batch_create_err.c_str();
    return batch->err.c_str();
}

// ---------------------------------------------------------------------------
// graph capture of library calls issued on one stream

int fn_graph_begin(void *stream)
{
    if (!stream) { g_graph_err = "graph capture needs a non-NULL stream"; return FN_E_INVAL; }
    hipError_t e = hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { g_graph_err = std::string("hipStreamBeginCapture: ") + hipGetErrorString(e); return FN_E_DEVICE; }
    return FN_OK;
}

int fn_graph_end(void *stream, fn_graph **out)
{
    if (!stream || !out) { g_graph_err = "NULL stream or out"; return FN_E_INVAL; }
    *out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &g);
    if (e != hipSuccess || !g) {
        g_graph_err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
        if (g) hipGraphDestroy(g);
        return FN_E_DEVICE;
    }
    fn_graph *G = new (std::nothrow) fn_graph();
    if (!G) { hipGraphDestroy(g); g_graph_err = "out of host memory"; return FN_E_NOMEM; }
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g_graph_err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        hipGraphDestroy(g);
        delete G;
        return FN_E_DEVICE;
    }
    *out = G;
    return FN_OK;
}

int fn_graph_launch(fn_graph *graph, void *stream)
{
    if (!graph) { g_graph_err = "graph is NULL"; return FN_E_INVAL; }
    hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) { g_graph_err = std::string("hipGraphLaunch: ") + hipGetErrorString(e); return FN_E_DEVICE; }
    return FN_OK;
}

int fn_graph_destroy(fn_graph *graph)
{
    if (graph) {
        if (graph->exec) hipGraphExecDestroy(graph->exec);
        if (graph->graph) hipGraphDestroy(graph->graph);
    }
    delete graph;
    return FN_OK;
}

const char *fn_graph_last_error(void) { return g_graph_err.c_str(); }

}  // extern "C"
