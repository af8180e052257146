// Batches of independent point sets (one mesh each) and HIP-graph capture of
// evaluation sequences.
//
// A batch holds one context per member, all on the batch's stream, with their
// workspaces carved from one caller buffer; inputs and outputs are the members'
// arrays concatenated (CSR offsets).  Members may use different parameters (the
// grid is normally chosen per member from its size).  Every member call is
// enqueued on the one stream, so a whole batch evaluation can be captured into
// a single graph and replayed with one launch (fn_graph_*), which removes the
// per-kernel launch cost that dominates small members.
#include "fn_internal.h"

#include <cstring>
#include <new>
#include <string>
#include <vector>

struct fn_batch {
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;  // second stream of fn_batch_eval_with_H_adjoint (created on first use)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
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
        if (batch->stream2) {
            hipStreamSynchronize(batch->stream2);
            hipStreamDestroy(batch->stream2);
        }
        if (batch->ev_fork) hipEventDestroy(batch->ev_fork);
        if (batch->ev_join) hipEventDestroy(batch->ev_join);
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

int fn_batch_eval(fn_batch *batch, double *phi, double *H)
{
    if (!batch) return FN_E_INVAL;
    if (!batch->geom_ready) BATCH_ERR(batch, FN_E_STATE, "fn_set_geometry_batch must succeed first");
    for (size_t i = 0; i < batch->ctx.size(); ++i) {
        if (batch->toff[i + 1] == batch->toff[i]) continue;
        int rc = fn_eval(batch->ctx[i], phi ? phi + batch->toff[i] : nullptr, H ? H + 2 * batch->toff[i] : nullptr);
        if (rc) return member_err(batch, (int)i, rc);
    }
    return FN_OK;
}

static int batch_adjoint(fn_batch *batch, const double *in, int comps, double *u, bool h)
{
    if (!batch) return FN_E_INVAL;
    if (!batch->geom_ready) BATCH_ERR(batch, FN_E_STATE, "fn_set_geometry_batch must succeed first");
    for (size_t i = 0; i < batch->ctx.size(); ++i) {
        if (batch->soff[i + 1] == batch->soff[i]) continue;
        const double *pi = in ? in + comps * batch->toff[i] : nullptr;
        double *pu = u ? u + batch->soff[i] : nullptr;
        int rc = h ? fn_eval_H_adjoint(batch->ctx[i], pi, pu) : fn_eval_phi_adjoint(batch->ctx[i], pi, pu);
        if (rc) return member_err(batch, (int)i, rc);
    }
    return FN_OK;
}

int fn_batch_eval_H_adjoint(fn_batch *batch, const double *V, double *u) { return batch_adjoint(batch, V, 2, u, true); }

int fn_batch_eval_with_H_adjoint(fn_batch *batch, double *phi, double *H, const double *V, double *u)
{
    if (!batch) return FN_E_INVAL;
    if (!batch->geom_ready) BATCH_ERR(batch, FN_E_STATE, "fn_set_geometry_batch must succeed first");
    // every argument is checked before anything is enqueued, so that an error leaves the
    // outputs untouched
    {
        const size_t B = batch->ctx.size();
        const int64_t nt = batch->toff[B] - batch->toff[0], ns = batch->soff[B] - batch->soff[0];
        for (size_t i = 0; i < B; ++i)
            if (!batch->ctx[i]->charges_ready) {
                batch->err = "member " + std::to_string(i) + ": fn_batch_set_charges must be called before evaluation";
                return FN_E_STATE;
            }
        if (nt > 0 && !phi && !H) BATCH_ERR(batch, FN_E_INVAL, "both outputs are NULL");
        if ((nt > 0 && !V) || (ns > 0 && !u)) BATCH_ERR(batch, FN_E_INVAL, "NULL input or output");
    }
    if (!batch->stream2) {
        if (stream_capturing(batch->stream))
            BATCH_ERR(batch, FN_E_STATE, "call fn_batch_eval_with_H_adjoint once before capturing it (it creates its stream)");
        hipStream_t s2 = nullptr;
        hipEvent_t e1 = nullptr, e2 = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&e2, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (e2) hipEventDestroy(e2);
            if (e1) hipEventDestroy(e1);
            if (s2) hipStreamDestroy(s2);
            BATCH_ERR(batch, FN_E_DEVICE, std::string("creating the second stream: ") + hipGetErrorString(e));
        }
        batch->stream2 = s2;
        batch->ev_fork = e1;
        batch->ev_join = e2;
    }
    // one fork for the whole batch: every member's adjoint on the second stream, its
    // forward on the batch stream, one join at the end
    hipError_t e = hipEventRecord(batch->ev_fork, batch->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(batch->stream2, batch->ev_fork, 0);
    if (e != hipSuccess) BATCH_ERR(batch, FN_E_DEVICE, std::string("fork: ") + hipGetErrorString(e));
    int rc = FN_OK;
    for (size_t i = 0; i < batch->ctx.size() && rc == FN_OK; ++i) {
        const int64_t nt = batch->toff[i + 1] - batch->toff[i], ns = batch->soff[i + 1] - batch->soff[i];
        if (ns > 0) {
            rc = fn_internal_adjoint_H_on_stream(batch->ctx[i], V ? V + 2 * batch->toff[i] : nullptr,
                                                 u ? u + batch->soff[i] : nullptr, batch->stream2);
            if (rc) rc = member_err(batch, (int)i, rc);
        }
        if (rc == FN_OK && nt > 0) {
            rc = fn_internal_eval_on_stream(batch->ctx[i], phi ? phi + batch->toff[i] : nullptr,
                                            H ? H + 2 * batch->toff[i] : nullptr, batch->stream);
            if (rc) rc = member_err(batch, (int)i, rc);
        }
    }
    // join even after an error, so that the batch stream never runs ahead of the fork
    const hipError_t e1 = hipEventRecord(batch->ev_join, batch->stream2);
    const hipError_t e2 = hipStreamWaitEvent(batch->stream, batch->ev_join, 0);
    if (rc) return rc;
    if (e1 != hipSuccess || e2 != hipSuccess)
        BATCH_ERR(batch, FN_E_DEVICE, std::string("join: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return FN_OK;
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
