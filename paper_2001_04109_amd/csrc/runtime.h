// Device workspace pool and plan executor.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "plan.h"

namespace ffp {

// A grow-only device buffer owned by the library, one per (device, stream).
// Growing waits for the stream so that no enqueued kernel still uses the
// old buffer.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    ProdTask* tasks = nullptr;   // device task table for grouped launches
    size_t task_cap = 0;
};

// Returns FFP_OK or FFP_ENOMEM / FFP_EDEVICE.  The returned workspace stays
// valid until the next call on the same stream that needs more memory.
int acquire_workspace(hipStream_t s, size_t bytes, size_t ntasks, Workspace** out);

// Pinned host staging plus a device buffer for kernel metadata (task and
// descriptor tables) of one call on stream s.  acquire_staging waits until
// the previous call's copies from the staging area have executed;
// release_staging marks the area busy until the work enqueued so far on s
// has run.
int acquire_staging(hipStream_t s, size_t bytes, char** host, char** dev);
int release_staging(hipStream_t s);

// A second stream paired with s (created on first use: non-blocking,
// default priority) and two events, for work that runs beside s inside one
// call: record `fork` on s, make `side` wait for it, enqueue on side, record
// `join` on side, make s wait for it.  Lives until the process ends.  Must
// be obtained before a capture begins (capture_point).
struct SideStream {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
int side_stream(hipStream_t s, SideStream** out);

// Records which HIP call failed (with its error name) for
// ffp_last_error_detail; returns e.
hipError_t note_hip(const char* where, hipError_t e);
const char* last_error_detail();

// Capture of a batched call into a HIP graph.  While a capture context is
// installed on the calling thread, acquire_workspace and acquire_staging
// allocate buffers that the context owns (they live as long as the graph)
// instead of using the per-stream pool, and nothing waits on the host.  The
// batched drivers acquire everything before their first launch and then
// call capture_point, which begins the stream capture; an acquisition after
// that point fails with FFP_EUNSUPPORTED (no allocation inside a capture).
struct CaptureCtx {
    hipStream_t stream = nullptr;
    bool capturing = false;
    std::vector<void*> dev;        // device buffers
    std::vector<void*> host;       // pinned host buffers
    std::vector<Workspace*> ws;
    size_t dev_bytes = 0;
    size_t host_bytes = 0;
    void free_all();
};
void set_capture_ctx(CaptureCtx* c);
CaptureCtx* capture_ctx();
// Begins the capture of stream s if a context is installed and not yet
// capturing; otherwise does nothing.
int capture_point(hipStream_t s);

// Enqueues every op of the plan on stream s.  a, c: caller buffers; ws:
// workspace of at least pl.ws_bytes.
int execute_plan(const Plan& pl, const void* a, void* c, void* ws, hipStream_t s, bool no_alloc = false);

int execute_op(const Plan& pl, const Op& o, const void* a, void* c, void* ws, hipStream_t s);

// Level scheduling of block operations.  Every op is placed on the
// earliest level after all earlier ops of its job that it depends on (it
// reads or writes memory that one of them writes, or writes memory that
// one of them reads; views are compared as rectangles).  The ops of one
// level are independent: the products of one class in a level run as one
// grouped launch of the product kernel (tiles longest first), the packs of
// one class pair as one grouped pack, other ops one by one.  Items of one
// job are consecutive and in program order; different jobs must touch
// disjoint memory.  Results are those of the program order.
struct SchedItem {
    const Plan* pl;
    const Op* op;
    const void* a;
    void* c;
    void* ws;
    int job;
};
// no_alloc: acquire no staging area (no pinned or device allocation): a
// level's product group of more than kInlineTasks tasks runs as several
// launches of at most kInlineTasks tasks (tables in the kernel arguments),
// and packs run one by one.
int run_leveled(const std::vector<SchedItem>& items, hipStream_t s, bool no_alloc = false);
// The level of every item (host only; also used by tests through the C ABI).
std::vector<int> schedule_levels(const std::vector<SchedItem>& items);
// 1: execute_plan runs the level scheduler (default); 0: ops in program order.
extern int g_leveled;
// 1 (default): products of small grouped launches move to a later level
// with a larger launch of their class when their dependents allow.
extern int g_merge_products;
// Size (in 128 x 128 tiles) under which a level's product launch counts as small.
extern int g_merge_tiles;
ProdTask make_task(const Plan& pl, const Op& o, const void* a, void* c, void* ws);
PackDesc make_pack(const Plan& pl, const Op& o, const void* a, void* c, void* ws);

hipError_t launch_products(int cls, ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                           hipStream_t s);
hipError_t launch_products_f64(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s);
hipError_t launch_products_i8(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s);
hipError_t launch_products_limb2(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s);
hipError_t launch_products_limb3(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s);

// Optional timing of product launches with HIP events (for the benchmark's
// roofline figures).  prof_read sums the elapsed times and algorithmic flops
// of the recorded launches of class cls (-1: all) and forgets them.
bool prof_enabled();
void prof_enable(bool on);
void prof_begin(hipStream_t s, hipEvent_t* e0);
void prof_end(hipStream_t s, hipEvent_t e0, double work, int cls);
int prof_read(int cls, double* ms, double* work, int64_t* launches);
int prof_read_variant(int cls, int variant, double* ms, double* work, int64_t* launches);

// Fills the product-kernel fields of a task from the field plan.
void init_task(ProdTask* t, const FieldPlan& f);

}  // namespace ffp
