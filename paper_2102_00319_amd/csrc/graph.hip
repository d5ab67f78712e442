// graph.hip -- capture of launch sequences into one HIP graph, over one or more
// contexts (one per parameter set, each on its own stream).
//
// Between fhe_graph_begin and fhe_graph_end every library call enqueues work
// as usual, but nothing runs: the work of all the contexts' streams becomes one
// graph (their streams fork from and join into the first context's stream).
// Pointer tables built during capture are kept in an arena whose device copy
// is written once, after capture, and belongs to the graph; the scratch and
// layer workspace the captured launches use are handed over to the graph as
// well, so that later calls on the contexts cannot move them.  Replays read
// and write the same device buffers as the captured calls.
#include <cstring>

#include "fhe_internal.h"

struct fhe_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t stream;
    std::vector<void *> dev;     // device memory owned by the graph
    struct Lent {                // buffers from a context's caller-supplied allocator
        void *p;
        fhe_free_fn free_fn;
        void *user;
    };
    std::vector<Lent> lent;
    std::vector<void *> host;    // pinned staging
    std::vector<hipEvent_t> events;
};

static void graph_free(fhe_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (void *p : g->dev)
        if (p) (void)hipFree(p);
    for (const fhe_graph::Lent &b : g->lent) b.free_fn(b.p, b.user);
    for (void *p : g->host)
        if (p) (void)hipHostFree(p);
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    delete g;
}

static void end_capture_state(fhe_ctx *const *ctxs, uint32_t n)
{
    for (uint32_t i = 0; i < n; ++i) {
        ctxs[i]->capturing = false;
        ctxs[i]->cap_host = ctxs[i]->cap_dev = nullptr;
        ctxs[i]->cap_bytes = ctxs[i]->cap_used = 0;
    }
}

extern "C" {

fhe_status fhe_graph_begin(fhe_ctx *const *ctxs, uint32_t n, uint64_t table_bytes, fhe_graph **out)
{
    if (!ctxs || !n || !out) return fhe_fail(FHE_EINVAL, "fhe_graph_begin: null or empty");
    *out = nullptr;
    for (uint32_t i = 0; i < n; ++i) {
        if (!ctxs[i]) return fhe_fail(FHE_EINVAL, "fhe_graph_begin: null context");
        if (ctxs[i]->capturing) return fhe_fail(FHE_EINVAL, "fhe_graph_begin: context already capturing");
        if (ctxs[i]->prof) return fhe_fail(FHE_EINVAL, "fhe_graph_begin: disable profiling before capture");
        for (uint32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fhe_fail(FHE_EINVAL, "fhe_graph_begin: context listed twice");
    }
    if (!table_bytes) table_bytes = (uint64_t)16 << 20;
    fhe_graph *g = new fhe_graph();
    g->stream = ctxs[0]->stream;
    for (uint32_t i = 0; i < n; ++i) {
        void *h = nullptr, *d = nullptr;
        if (hipHostMalloc(&h, table_bytes) != hipSuccess || hipMalloc(&d, table_bytes) != hipSuccess) {
            if (h) (void)hipHostFree(h);
            graph_free(g);
            end_capture_state(ctxs, i);
            return fhe_fail(FHE_ENOMEM, "fhe_graph_begin: cannot allocate the pointer-table arena");
        }
        g->host.push_back(h);
        g->dev.push_back(d);
        // finish pending work (and pending table copies) before capture starts
        if (hipStreamSynchronize(ctxs[i]->stream) != hipSuccess) {
            graph_free(g);
            end_capture_state(ctxs, i);
            return fhe_fail(FHE_EDEVICE, "fhe_graph_begin: stream synchronisation failed");
        }
        ctxs[i]->cap_host = (uint8_t *)h;
        ctxs[i]->cap_dev = (uint8_t *)d;
        ctxs[i]->cap_bytes = table_bytes;
        ctxs[i]->cap_used = 0;
        ctxs[i]->cap_error = 0;
    }
    hipError_t e = hipStreamBeginCapture(ctxs[0]->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        graph_free(g);
        end_capture_state(ctxs, n);
        return fhe_hip_check(e, "hipStreamBeginCapture");
    }
    for (uint32_t i = 0; i < n; ++i) ctxs[i]->capturing = true;
    // fork: the other streams join the capture
    for (uint32_t i = 1; i < n; ++i) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ctxs[0]->cap_error = FHE_EDEVICE;
            break;
        }
        g->events.push_back(ev);
        if (hipEventRecord(ev, ctxs[0]->stream) != hipSuccess ||
            hipStreamWaitEvent(ctxs[i]->stream, ev, 0) != hipSuccess) {
            ctxs[0]->cap_error = FHE_EDEVICE;
            break;
        }
    }
    *out = g;
    return FHE_OK;
}

fhe_status fhe_graph_end(fhe_ctx *const *ctxs, uint32_t n, fhe_graph *g)
{
    if (!ctxs || !n || !g) return fhe_fail(FHE_EINVAL, "fhe_graph_end: null or empty");
    int err = 0;
    // join the other streams back into the capturing one
    for (uint32_t i = 1; i < n; ++i) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            err = FHE_EDEVICE;
            continue;
        }
        g->events.push_back(ev);
        if (hipEventRecord(ev, ctxs[i]->stream) != hipSuccess ||
            hipStreamWaitEvent(ctxs[0]->stream, ev, 0) != hipSuccess)
            err = FHE_EDEVICE;
    }
    for (uint32_t i = 0; i < n; ++i)
        if (ctxs[i]->cap_error) err = ctxs[i]->cap_error;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctxs[0]->stream, &graph);
    g->graph = graph;
    std::vector<size_t> used(n);
    for (uint32_t i = 0; i < n; ++i) used[i] = ctxs[i]->cap_used;
    end_capture_state(ctxs, n);
    if (e != hipSuccess || err || !graph) {
        graph_free(g);
        if (e != hipSuccess) return fhe_hip_check(e, "hipStreamEndCapture");
        return fhe_fail(err ? err : FHE_EDEVICE, "fhe_graph_end: a call failed during capture");
    }
    if ((e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        graph_free(g);
        return fhe_hip_check(e, "hipGraphInstantiate");
    }
    // the tables' device home, then hand the contexts' scratch over to the graph
    for (uint32_t i = 0; i < n; ++i) {
        if (used[i] && (e = hipMemcpy(g->dev[i], g->host[i], used[i], hipMemcpyHostToDevice)) != hipSuccess) {
            graph_free(g);
            return fhe_hip_check(e, "hipMemcpy");
        }
        fhe_ctx *c = ctxs[i];
        for (uint8_t *b : {c->scratch, c->wksp}) {
            if (!b) continue;
            if (c->alloc_fn) g->lent.push_back(fhe_graph::Lent{b, c->free_fn, c->alloc_user});
            else g->dev.push_back(b);
        }
        c->used -= c->scratch_bytes + c->wksp_bytes;
        c->scratch = c->wksp = nullptr;
        c->scratch_bytes = c->wksp_bytes = 0;
    }
    for (void *h : g->host) (void)hipHostFree(h);
    g->host.clear();
    return FHE_OK;
}

fhe_status fhe_graph_launch(fhe_graph *g, void *hip_stream)
{
    if (!g || !g->exec) return fhe_fail(FHE_EINVAL, "fhe_graph_launch: null graph");
    HIPCHK(hipGraphLaunch(g->exec, hip_stream ? (hipStream_t)hip_stream : g->stream));
    return FHE_OK;
}

void fhe_graph_destroy(fhe_graph *g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();   // replays may have gone to any stream
    graph_free(g);
}

}  // extern "C"
