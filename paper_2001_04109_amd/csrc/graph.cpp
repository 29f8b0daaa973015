// Batched calls recorded once as HIP graphs and replayed.
//
// A graph is made by running the batched driver with a capture context
// installed: the host planning (schedules, level grouping, task and
// descriptor tables) happens once, the driver's workspace and staging
// buffers are allocated for the graph before the capture begins, and every
// kernel launch and table copy of the call is recorded.  A replay re-runs
// the recorded work on the operands at the recorded addresses, with no
// host planning and one launch call.
#include <hip/hip_runtime.h>

#include <vector>

#include "batch.h"
#include "ffp.h"
#include "ldlt.h"
#include "runtime.h"

struct ffp_graph_s {
    int device = 0;
    ffp::CaptureCtx ctx;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;   // null: the batch had no work
};

namespace {

using namespace ffp;

void destroy(ffp_graph_s* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->ctx.free_all();
    delete g;
}

// Runs enqueue() on stream s under a capture context and instantiates what
// it recorded.
template <class F>
int record(hipStream_t s, F&& enqueue, ffp_graph* out)
{
    if (!out) return FFP_EINVAL;
    *out = nullptr;
    if (s == nullptr) return FFP_EINVAL;   // the null stream cannot be captured
    ffp_graph_s* g = new ffp_graph_s();
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return FFP_EDEVICE;
    }
    g->ctx.stream = s;
    set_capture_ctx(&g->ctx);
    int st = enqueue();
    set_capture_ctx(nullptr);
    if (g->ctx.capturing) {
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        g->ctx.capturing = false;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (st == FFP_OK) st = FFP_EDEVICE;
        }
        g->graph = graph;
        if (st == FFP_OK) {
            if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGetLastError();
                g->exec = nullptr;
                st = FFP_EDEVICE;
            }
        }
    }
    if (st != FFP_OK) {
        destroy(g);
        return st;
    }
    *out = g;
    return FFP_OK;
}

}  // namespace

extern "C" {

int ffp_graph_syrk_batched(int njobs, const ffp_job* jobs, unsigned flags, void* stream, ffp_graph* out)
{
    hipStream_t s = (hipStream_t)stream;
    return record(s, [&]() { return batched_run(njobs, jobs, flags, s); }, out);
}

int ffp_graph_ldlt_batched(int njobs, const ffp_ldlt_job* jobs, void* stream, ffp_graph* out)
{
    hipStream_t s = (hipStream_t)stream;
    return record(s, [&]() { return fldlt_modp_batched(njobs, jobs, stream); }, out);
}

int ffp_graph_launch(ffp_graph g, void* stream)
{
    if (!g) return FFP_EINVAL;
    if (!g->exec) return FFP_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FFP_EDEVICE;
    if (dev != g->device) return FFP_EINVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? FFP_OK : FFP_EDEVICE;
}

size_t ffp_graph_device_bytes(ffp_graph g) { return g ? g->ctx.dev_bytes : 0; }

size_t ffp_graph_nodes(ffp_graph g)
{
    if (!g || !g->graph) return 0;
    size_t n = 0;
    if (hipGraphGetNodes(g->graph, nullptr, &n) != hipSuccess) return 0;
    return n;
}

void ffp_graph_destroy(ffp_graph g) { destroy(g); }

}  // extern "C"
