// Workspace pool and plan executor of the product library.
#include "runtime.h"

#include <algorithm>
#include <map>
#include <vector>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>

#include "ffp.h"

namespace ffp {

namespace {

std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

void* at(const PView& v, const void* a, void* c, void* ws)
{
    char* base = nullptr;
    switch (v.buf) {
    case BUF_A: base = (char*)a; break;
    case BUF_C: base = (char*)c; break;
    default: base = (char*)ws; break;
    }
    return base + v.off;
}

DView dview(const PView& v, const void* a, void* c, void* ws)
{
    return DView{at(v, a, c, ws), v.ld, v.plane};
}

}  // namespace

namespace {
thread_local std::string g_err_detail;
}  // namespace

hipError_t note_hip(const char* where, hipError_t e)
{
    if (e != hipSuccess) {
        g_err_detail = std::string(where) + ": " + hipGetErrorName(e);
        (void)hipGetLastError();
    }
    return e;
}

const char* last_error_detail() { return g_err_detail.c_str(); }

namespace {
thread_local CaptureCtx* g_cap = nullptr;

int cap_dev_alloc(CaptureCtx* c, size_t bytes, void** out)
{
    *out = nullptr;
    if (c->capturing) return FFP_EUNSUPPORTED;
    if (bytes == 0) return FFP_OK;
    if (note_hip("hipMalloc (graph buffer)", hipMalloc(out, bytes)) != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return FFP_ENOMEM;
    }
    c->dev.push_back(*out);
    c->dev_bytes += bytes;
    return FFP_OK;
}
}  // namespace

void CaptureCtx::free_all()
{
    for (void* p : dev) (void)hipFree(p);
    for (void* p : host) (void)hipHostFree(p);
    for (Workspace* w : ws) delete w;
    dev.clear();
    host.clear();
    ws.clear();
    dev_bytes = host_bytes = 0;
}

void set_capture_ctx(CaptureCtx* c) { g_cap = c; }
CaptureCtx* capture_ctx() { return g_cap; }

int capture_point(hipStream_t s)
{
    CaptureCtx* c = g_cap;
    if (!c || c->capturing) return FFP_OK;
    if (s == nullptr || s != c->stream) return FFP_EINVAL;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return FFP_EDEVICE;
    }
    c->capturing = true;
    return FFP_OK;
}

namespace {
std::map<std::pair<int, hipStream_t>, SideStream> g_side;
}  // namespace

int side_stream(hipStream_t s, SideStream** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FFP_EDEVICE;
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    SideStream& ss = g_side[std::make_pair(dev, s)];
    if (!ss.side) {
        if (g_cap && g_cap->capturing) return FFP_EUNSUPPORTED;
        if (note_hip("hipStreamCreateWithFlags", hipStreamCreateWithFlags(&ss.side, hipStreamNonBlocking)) !=
                hipSuccess ||
            note_hip("hipEventCreateWithFlags", hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming)) !=
                hipSuccess ||
            note_hip("hipEventCreateWithFlags", hipEventCreateWithFlags(&ss.join, hipEventDisableTiming)) !=
                hipSuccess) {
            if (ss.side) (void)hipStreamDestroy(ss.side);
            if (ss.fork) (void)hipEventDestroy(ss.fork);
            ss = SideStream{};
            return FFP_EDEVICE;
        }
    }
    *out = &ss;
    return FFP_OK;
}

int acquire_workspace(hipStream_t s, size_t bytes, size_t ntasks, Workspace** out)
{
    if (CaptureCtx* c = g_cap) {
        Workspace* w = new Workspace();
        c->ws.push_back(w);
        int st = cap_dev_alloc(c, bytes, &w->ptr);
        if (st != FFP_OK) return st;
        w->bytes = bytes;
        if (ntasks > 0) {
            st = cap_dev_alloc(c, ntasks * sizeof(ProdTask), (void**)&w->tasks);
            if (st != FFP_OK) return st;
            w->task_cap = ntasks;
        }
        *out = w;
        return FFP_OK;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FFP_EDEVICE;
    // the lock covers the lookup only: a stream's workspace is used by one
    // thread at a time (the library is thread-safe across streams), and its
    // growth waits for the stream, which must not hold up other streams
    Workspace* wp;
    {
        std::lock_guard<std::mutex> lk(g_ws_mutex);
        wp = &g_ws[std::make_pair(dev, s)];
    }
    Workspace& w = *wp;
    if (bytes > w.bytes || ntasks > w.task_cap) {
        if (w.ptr || w.tasks) {
            if (note_hip("hipStreamSynchronize (workspace)", hipStreamSynchronize(s)) != hipSuccess)
                return FFP_EDEVICE;
        }
        if (bytes > w.bytes) {
            if (w.ptr) (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
            size_t want = bytes + bytes / 4 + 4096;
            if (note_hip("hipMalloc (workspace)", hipMalloc(&w.ptr, want)) != hipSuccess) {
                w.ptr = nullptr;
                (void)hipGetLastError();
                return FFP_ENOMEM;
            }
            w.bytes = want;
        }
        if (ntasks > w.task_cap) {
            if (w.tasks) (void)hipFree(w.tasks);
            w.tasks = nullptr;
            w.task_cap = 0;
            size_t cap = ntasks < 64 ? 64 : ntasks * 2;
            if (note_hip("hipMalloc (task table)", hipMalloc((void**)&w.tasks, cap * sizeof(ProdTask))) !=
                hipSuccess) {
                w.tasks = nullptr;
                (void)hipGetLastError();
                return FFP_ENOMEM;
            }
            w.task_cap = cap;
        }
    }
    *out = &w;
    return FFP_OK;
}

namespace {
struct Staging {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
std::map<std::pair<int, hipStream_t>, Staging> g_stage;
}  // namespace

int acquire_staging(hipStream_t s, size_t bytes, char** host, char** dev)
{
    if (CaptureCtx* c = g_cap) {
        *host = nullptr;
        *dev = nullptr;
        if (c->capturing) return FFP_EUNSUPPORTED;
        if (note_hip("hipHostMalloc (graph tables)", hipHostMalloc((void**)host, bytes, hipHostMallocDefault)) !=
            hipSuccess) {
            *host = nullptr;
            (void)hipGetLastError();
            return FFP_ENOMEM;
        }
        c->host.push_back(*host);
        c->host_bytes += bytes;
        return cap_dev_alloc(c, bytes, (void**)dev);
    }
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return FFP_EDEVICE;
    // lookup under the lock; the wait for the previous use of this stream's
    // staging area outside it (other streams' launches go on meanwhile)
    Staging* sp;
    {
        std::lock_guard<std::mutex> lk(g_ws_mutex);
        sp = &g_stage[std::make_pair(d, s)];
    }
    Staging& st = *sp;
    if (st.pending) {
        if (hipEventSynchronize(st.done) != hipSuccess) return FFP_EDEVICE;
        st.pending = false;
    }
    if (!st.done && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess)
        return FFP_EDEVICE;
    if (bytes > st.cap) {
        if (st.host) (void)hipHostFree(st.host);
        if (st.dev) (void)hipFree(st.dev);
        st.host = nullptr;
        st.dev = nullptr;
        st.cap = 0;
        const size_t want = bytes + bytes / 2 + 4096;
        if (note_hip("hipHostMalloc (staging)", hipHostMalloc((void**)&st.host, want, hipHostMallocDefault)) !=
                hipSuccess ||
            note_hip("hipMalloc (staging)", hipMalloc((void**)&st.dev, want)) != hipSuccess) {
            (void)hipGetLastError();
            return FFP_ENOMEM;
        }
        st.cap = want;
    }
    *host = st.host;
    *dev = st.dev;
    return FFP_OK;
}

int release_staging(hipStream_t s)
{
    if (g_cap) return FFP_OK;   // the graph owns its staging area
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return FFP_EDEVICE;
    Staging* sp;
    {
        std::lock_guard<std::mutex> lk(g_ws_mutex);
        sp = &g_stage[std::make_pair(d, s)];
    }
    Staging& st = *sp;
    if (!st.done) return FFP_OK;
    if (hipEventRecord(st.done, s) != hipSuccess) return FFP_EDEVICE;
    st.pending = true;
    return FFP_OK;
}

thread_local int g_tile_hint = 0;

namespace {
// Sets the tile hint for the launches made while it lives.
struct TileHint {
    int saved;
    explicit TileHint(int tile) : saved(g_tile_hint) { g_tile_hint = tile; }
    ~TileHint() { g_tile_hint = saved; }
};
}  // namespace

int64_t g_kblk_cap = 0;
int g_persistent = 2;
thread_local int g_last_variant = -1;

int resident_blocks(const void* kernel, int threads)
{
    // occupancy per (device, kernel, block size), queried once: launches
    // are frequent and the query is a runtime call
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, kernel, threads);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per <= 0) per = 1;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = per * cus;
    return per * cus;
}

// ---- optional per-launch timing (HIP events around each product launch) --
namespace {
struct ProfRec {
    hipEvent_t e0, e1;
    double work;   // algorithmic flops of the launch
    int cls;
    int variant;
};
std::mutex g_prof_mutex;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
}  // namespace

bool prof_enabled() { return g_prof_on && g_cap == nullptr; }

void prof_begin(hipStream_t s, hipEvent_t* e0)
{
    if (hipEventCreate(e0) != hipSuccess) { *e0 = nullptr; return; }
    (void)hipEventRecord(*e0, s);
}

namespace {
// end event recorded by a launcher between its main kernel and a follow-up
// kernel of the same launch (prof_mark_end), taken by the next prof_end
thread_local hipEvent_t g_prof_mid = nullptr;
}  // namespace

void prof_mark_end(hipStream_t s)
{
    if (!prof_enabled() || g_prof_mid != nullptr) return;
    if (hipEventCreate(&g_prof_mid) != hipSuccess) { g_prof_mid = nullptr; return; }
    (void)hipEventRecord(g_prof_mid, s);
}

void prof_end(hipStream_t s, hipEvent_t e0, double work, int cls)
{
    hipEvent_t e1 = g_prof_mid;
    g_prof_mid = nullptr;
    if (!e0) {
        if (e1) (void)hipEventDestroy(e1);
        return;
    }
    if (e1 == nullptr) {
        if (hipEventCreate(&e1) != hipSuccess) return;
        (void)hipEventRecord(e1, s);
    }
    std::lock_guard<std::mutex> lk(g_prof_mutex);
    g_prof.push_back(ProfRec{e0, e1, work, cls, g_last_variant});
}

void prof_enable(bool on)
{
    std::lock_guard<std::mutex> lk(g_prof_mutex);
    g_prof_on = on;
}

int prof_read(int cls, double* ms, double* work, int64_t* launches)
{
    return prof_read_variant(cls, -1, ms, work, launches);
}

int prof_read_variant(int cls, int variant, double* ms, double* work, int64_t* launches)
{
    std::lock_guard<std::mutex> lk(g_prof_mutex);
    double tms = 0.0, tw = 0.0;
    int64_t nl = 0;
    std::vector<ProfRec> keep;
    for (ProfRec& r : g_prof) {
        if ((cls >= 0 && r.cls != cls) || (variant >= 0 && r.variant != variant)) {
            keep.push_back(r);
            continue;
        }
        float t = 0.f;
        if (hipEventSynchronize(r.e1) != hipSuccess) return -1;
        if (hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) return -1;
        tms += t;
        tw += r.work;
        ++nl;
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_prof.swap(keep);
    *ms = tms;
    *work = tw;
    *launches = nl;
    return 0;
}

void init_task(ProdTask* t, const FieldPlan& f)
{
    t->p = f.p;
    t->half = (f.p - 1) / 2;
    t->pinv = f.pinv;
    t->kblk = (int32_t)f64_kblk(f.p);
}

hipError_t launch_products(int cls, ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                           hipStream_t s)
{
    switch (cls) {
    case CLS_F64: return launch_products_f64(tasks, ntasks, dev_task_buf, s);
    case CLS_I8: return launch_products_i8(tasks, ntasks, dev_task_buf, s);
    case CLS_LIMB2: return launch_products_limb2(tasks, ntasks, dev_task_buf, s);
    case CLS_LIMB3: return launch_products_limb3(tasks, ntasks, dev_task_buf, s);
    default: return hipErrorInvalidValue;
    }
}

int g_leveled = 1;

int execute_plan(const Plan& pl, const void* a, void* c, void* ws, hipStream_t s, bool no_alloc)
{
    if (g_leveled) {
        std::vector<SchedItem> items;
        items.reserve(pl.ops.size());
        for (const Op& o : pl.ops) items.push_back(SchedItem{&pl, &o, a, c, ws, 0});
        return run_leveled(items, s, no_alloc);
    }
    for (const Op& o : pl.ops) {
        int st = execute_op(pl, o, a, c, ws, s);
        if (st != FFP_OK) return st;
    }
    return FFP_OK;
}

namespace {

// Bytes [base + r ld, base + r ld + cols) for r < rows.
struct Region {
    uintptr_t base;
    int64_t ld, rows, cols;
};

bool overlap(const Region& x, const Region& y)
{
    if (x.rows <= 0 || x.cols <= 0 || y.rows <= 0 || y.cols <= 0) return false;
    const uintptr_t xe = x.base + (uintptr_t)((x.rows - 1) * x.ld + x.cols);
    const uintptr_t ye = y.base + (uintptr_t)((y.rows - 1) * y.ld + y.cols);
    if (xe <= y.base || ye <= x.base) return false;
    if (x.ld != y.ld || x.ld <= 0) return true;          // different pitch: spans overlap
    const int64_t ld = x.ld;
    const uintptr_t o = x.base < y.base ? x.base : y.base;
    const int64_t xr = (int64_t)((x.base - o) / (uintptr_t)ld), xc = (int64_t)((x.base - o) % (uintptr_t)ld);
    const int64_t yr = (int64_t)((y.base - o) / (uintptr_t)ld), yc = (int64_t)((y.base - o) % (uintptr_t)ld);
    if (xc + x.cols > ld || yc + y.cols > ld) return true; // a row wraps past the pitch
    return xr < yr + y.rows && yr < xr + x.rows && xc < yc + y.cols && yc < xc + x.cols;
}

struct OpRegions {
    std::vector<Region> rd, wr;
};

void add_view(std::vector<Region>& out, const PView& v, int64_t rows, int64_t cols, int64_t es,
              int planes, const SchedItem& it)
{
    const uintptr_t b = (uintptr_t)at(v, it.a, it.c, it.ws);
    const int64_t ld = (rows > 1 ? v.ld : cols) * es;
    for (int q = 0; q < planes; ++q) out.push_back(Region{b + (uintptr_t)(q * v.plane * es), ld, rows, cols * es});
}

int64_t class_es(int cls) { return cls == CLS_F64 ? 4 : 1; }

OpRegions regions_of(const SchedItem& it)
{
    const Op& o = *it.op;
    OpRegions r;
    const int64_t es = class_es(o.cls);
    const int pl = cls_planes(o.cls);
    switch (o.kind) {
    case OP_S1S2:
        for (int i = 0; i < 3; ++i) add_view(r.rd, o.v[i], o.m, o.k, es, pl, it);
        add_view(r.wr, o.v[3], o.m, o.k, es, pl, it);
        add_view(r.wr, o.v[4], o.m, o.k, es, pl, it);
        break;
    case OP_S34:
        for (int i = 0; i < 3; ++i) add_view(r.rd, o.v[i], o.m, o.k, es, pl, it);
        if (o.mode & 1) add_view(r.wr, o.v[3], o.m, o.k, es, pl, it);
        if (o.mode & 2) add_view(r.wr, o.v[4], o.m, o.k, es, pl, it);
        break;
    case OP_GEMM:
        add_view(r.rd, o.v[0], o.m, o.k, es, pl, it);
        add_view(r.rd, o.v[1], o.n, o.k, es, pl, it);
        add_view(r.wr, o.v[2], o.m, o.n, 4, 1, it);
        if (o.beta) add_view(r.rd, o.v[2], o.m, o.n, 4, 1, it);
        break;
    case OP_SYRK:
        add_view(r.rd, o.v[0], o.m, o.k, es, pl, it);
        add_view(r.wr, o.v[1], o.m, o.m, 4, 1, it);
        if (o.beta) add_view(r.rd, o.v[1], o.m, o.m, 4, 1, it);
        break;
    case OP_POSTADD:
        for (int i = 0; i < (o.beta ? 5 : 4); ++i) {
            add_view(r.rd, o.v[i], o.m, o.m, 4, 1, it);
            add_view(r.wr, o.v[i], o.m, o.m, 4, 1, it);
        }
        if (o.beta) {
            add_view(r.rd, o.v[5], 1, o.m, 4, 1, it);
            add_view(r.wr, o.v[5], 1, o.m, 4, 1, it);
        }
        break;
    case OP_ADDLOW:
        add_view(r.rd, o.v[0], o.m, o.m, 4, 1, it);
        add_view(r.rd, o.v[1], o.m, o.m, 4, 1, it);
        add_view(r.wr, o.v[2], o.m, o.m, 4, 1, it);
        break;
    case OP_SAVEC22:
        add_view(r.rd, o.v[0], o.m, o.m, 4, 1, it);
        add_view(r.wr, o.v[1], o.m, o.m, 4, 1, it);
        add_view(r.wr, o.v[2], 1, o.m, 4, 1, it);
        break;
    case OP_MIRROR:
        add_view(r.rd, o.v[0], o.m, o.m, 4, 1, it);
        add_view(r.wr, o.v[0], o.m, o.m, 4, 1, it);
        break;
    case OP_PACK:
        add_view(r.rd, o.v[0], o.m_src, o.k_src, class_es(o.src_cls), cls_planes(o.src_cls), it);
        add_view(r.wr, o.v[1], o.m, o.k, es, pl, it);
        break;
    case OP_COPY:
        add_view(r.rd, o.v[0], o.m, o.n, 4, 1, it);
        add_view(r.wr, o.v[1], o.m, o.n, 4, 1, it);
        break;
    case OP_LINCOMB:
        for (int i = 0; i < (o.mode & 7); ++i) add_view(r.rd, o.v[i], o.m, o.k, 4, 1, it);
        add_view(r.wr, o.v[5], o.m, o.k, 4, 1, it);
        break;
    case OP_LCT:
        for (int i = 0; i < (o.mode & 7); ++i) {
            const bool tr = (o.mode >> (3 + i)) & 1;
            add_view(r.rd, o.v[i], tr ? o.k : o.m, tr ? o.m : o.k, 4, 1, it);
        }
        add_view(r.wr, o.v[5], o.m, o.k, 4, 1, it);
        break;
    }
    return r;
}

bool any_overlap(const std::vector<Region>& x, const std::vector<Region>& y)
{
    for (const Region& a : x)
        for (const Region& b : y)
            if (overlap(a, b)) return true;
    return false;
}

// j (later) depends on i (earlier)
bool depends(const OpRegions& i, const OpRegions& j)
{
    return any_overlap(i.wr, j.rd) || any_overlap(i.wr, j.wr) || any_overlap(i.rd, j.wr);
}

bool longer_task(const ProdTask& a, const ProdTask& b)
{
    if (a.k != b.k) return a.k > b.k;
    return (int64_t)a.m * a.n > (int64_t)b.m * b.n;
}

int64_t rup256(int64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

// Products (GEMM, SYRK) of one representation class on one level form one
// grouped launch.  After the as-soon-as-possible levels are set, a product
// whose launch would be small (under g_merge_tiles tiles of 128 x 128, two
// rounds over the 256 CUs by default) moves to the later level, within
// the range its dependents allow, that already holds the most product work of
// its class: the leaves on blocks of A that are ready at once (the chains of
// P1 and P2) join a large launch instead of running on a fraction of the
// CUs.  Moving an operation later keeps every dependency satisfied as long as
// no operation that depends on it runs at or before its new level.
int g_merge_tiles = 512;

namespace {

bool is_product(const SchedItem& it) { return it.op->kind == OP_GEMM || it.op->kind == OP_SYRK; }

double product_area(const SchedItem& it)
{
    const Op& o = *it.op;
    return o.kind == OP_SYRK ? 0.5 * (double)o.m * (double)(o.m + 1) : (double)o.m * (double)o.n;
}

void merge_small_products(const std::vector<SchedItem>& items, const std::vector<OpRegions>& regs,
                          std::vector<int>& level)
{
    const size_t n = items.size();
    int maxlev = 0;
    for (int lv : level) maxlev = lv > maxlev ? lv : maxlev;
    std::vector<double> area((size_t)(maxlev + 1) * kNumCls, 0.0);
    auto slot = [&](int lv, int cls) -> double& { return area[(size_t)lv * kNumCls + cls]; };
    for (size_t i = 0; i < n; ++i)
        if (is_product(items[i])) slot(level[i], items[i].op->cls) += product_area(items[i]);
    std::vector<size_t> job_end(n);
    for (size_t i = n; i-- > 0;) job_end[i] = (i + 1 < n && items[i + 1].job == items[i].job) ? job_end[i + 1] : i + 1;
    for (size_t i = n; i-- > 0;) {
        if (!is_product(items[i])) continue;
        const int cls = items[i].op->cls, cur = level[i];
        if (slot(cur, cls) >= (double)g_merge_tiles * 128.0 * 128.0) continue;
        int alap = maxlev;
        for (size_t j = i + 1; j < job_end[i]; ++j)
            if (level[j] - 1 < alap && depends(regs[i], regs[j])) alap = level[j] - 1;
        int best = cur;
        for (int lv = cur + 1; lv <= alap; ++lv)
            if (slot(lv, cls) > slot(best, cls)) best = lv;
        if (best == cur || slot(best, cls) <= slot(cur, cls)) continue;
        const double a = product_area(items[i]);
        slot(cur, cls) -= a;
        slot(best, cls) += a;
        level[i] = best;
    }
}
}  // namespace

int g_merge_products = 1;

std::vector<int> schedule_levels(const std::vector<SchedItem>& items)
{
    const size_t n = items.size();
    std::vector<OpRegions> regs(n);
    for (size_t i = 0; i < n; ++i) regs[i] = regions_of(items[i]);
    std::vector<int> level(n, 0);
    size_t start = 0;
    for (size_t j = 0; j < n; ++j) {
        if (j > 0 && items[j].job != items[j - 1].job) start = j;
        int lv = 0;
        for (size_t i = start; i < j; ++i)
            if (level[i] + 1 > lv && depends(regs[i], regs[j])) lv = level[i] + 1;
        level[j] = lv;
    }
    if (g_merge_products) merge_small_products(items, regs, level);
    return level;
}

int run_leveled(const std::vector<SchedItem>& items, hipStream_t s, bool no_alloc)
{
    const size_t n = items.size();
    if (n == 0) return FFP_OK;
    const std::vector<int> level = schedule_levels(items);
    int maxlev = 0;
    for (int lv : level) maxlev = lv > maxlev ? lv : maxlev;
    std::vector<std::vector<size_t>> by_level(maxlev + 1);
    for (size_t j = 0; j < n; ++j) by_level[level[j]].push_back(j);

    // staging for the task and descriptor tables of grouped launches
    size_t meta = 0;
    for (const auto& lv : by_level) {
        size_t np[kNumCls] = {0}, nk[kNumCls * kNumCls] = {0};
        for (size_t j : lv) {
            const Op& o = *items[j].op;
            if (o.kind == OP_SYRK || o.kind == OP_GEMM) ++np[o.cls];
            else if (o.kind == OP_PACK) ++nk[o.src_cls * kNumCls + o.cls];
        }
        if (no_alloc) continue;
        for (size_t q : np)
            if (q > (size_t)kInlineTasks) meta += (size_t)rup256((int64_t)(q * sizeof(ProdTask)));
        for (size_t q : nk) if (q > 1) meta += (size_t)rup256((int64_t)(q * sizeof(PackDesc)));
    }
    char* host_meta = nullptr;
    char* dev_meta = nullptr;
    if (meta > 0) {
        int st = acquire_staging(s, meta, &host_meta, &dev_meta);
        if (st != FFP_OK) return st;
    }
    if (const int st = capture_point(s); st != FFP_OK) return st;
    size_t moff = 0;
    int status = FFP_OK;
    for (const auto& lv : by_level) {
        std::vector<size_t> prods[kNumCls], packs[kNumCls * kNumCls];
        for (size_t j : lv) {
            const SchedItem& it = items[j];
            const Op& o = *it.op;
            if (o.kind == OP_SYRK || o.kind == OP_GEMM) {
                prods[o.cls].push_back(j);
            } else if (o.kind == OP_PACK) {
                packs[o.src_cls * kNumCls + o.cls].push_back(j);
            } else {
                const int st = execute_op(*it.pl, o, it.a, it.c, it.ws, s);
                if (st != FFP_OK) { status = st; break; }
            }
        }
        if (status != FFP_OK) break;
        for (int cls = 0; cls < kNumCls && status == FFP_OK; ++cls) {
            const auto& g = prods[cls];
            if (g.empty()) continue;
            if (g.size() == 1) {
                const SchedItem& it = items[g[0]];
                status = execute_op(*it.pl, *it.op, it.a, it.c, it.ws, s);
                continue;
            }
            // up to kInlineTasks tasks travel in the kernel arguments
            std::vector<ProdTask> own;
            ProdTask inl[kInlineTasks];
            ProdTask* tasks = inl;
            ProdTask* dtasks = nullptr;
            if (no_alloc && g.size() > (size_t)kInlineTasks) {
                own.resize(g.size());
                tasks = own.data();
            } else if (g.size() > (size_t)kInlineTasks) {
                tasks = (ProdTask*)(host_meta + moff);
                dtasks = (ProdTask*)(dev_meta + moff);
                moff += (size_t)rup256((int64_t)(g.size() * sizeof(ProdTask)));
            }
            int nt = 0;
            double flops = 0.0;
            // a tuned tile applies to the products of one call; grouped
            // launches over several jobs keep the launch rule, which sizes
            // the tile from the whole group
            int tile = items[g[0]].pl->tile;
            for (size_t j : g)
                if (items[j].pl->tile != tile || items[j].job != items[g[0]].job) tile = 0;
            for (size_t j : g) {
                const SchedItem& it = items[j];
                ProdTask t = make_task(*it.pl, *it.op, it.a, it.c, it.ws);
                flops += t.syrk ? (double)t.m * (double)(t.m + 1) * (double)t.k
                                : 2.0 * (double)t.m * (double)t.n * (double)t.k;
                tasks[nt++] = t;
            }
            std::stable_sort(tasks, tasks + nt, longer_task);
            hipEvent_t e0 = nullptr;
            const bool prof = prof_enabled();
            if (prof) prof_begin(s, &e0);
            {
                TileHint hint(tile);
                if (no_alloc) {
                    // longest first, kInlineTasks per launch
                    for (int t0 = 0; t0 < nt && status == FFP_OK; t0 += kInlineTasks)
                        if (launch_products(cls, tasks + t0, std::min(kInlineTasks, nt - t0), nullptr, s) !=
                            hipSuccess)
                            status = FFP_EDEVICE;
                } else if (launch_products(cls, tasks, nt, dtasks, s) != hipSuccess) {
                    status = FFP_EDEVICE;
                }
            }
            if (prof) prof_end(s, e0, flops, cls);
        }
        for (int q = 0; q < kNumCls * kNumCls && status == FFP_OK; ++q) {
            const auto& g = packs[q];
            if (g.empty()) continue;
            if (no_alloc) {
                for (size_t j : g) {
                    const SchedItem& it = items[j];
                    status = execute_op(*it.pl, *it.op, it.a, it.c, it.ws, s);
                    if (status != FFP_OK) break;
                }
                continue;
            }
            if (g.size() == 1) {
                const SchedItem& it = items[g[0]];
                status = execute_op(*it.pl, *it.op, it.a, it.c, it.ws, s);
                continue;
            }
            PackDesc* d = (PackDesc*)(host_meta + moff);
            PackDesc* dd = (PackDesc*)(dev_meta + moff);
            moff += (size_t)rup256((int64_t)(g.size() * sizeof(PackDesc)));
            int nd = 0;
            for (size_t j : g) {
                const SchedItem& it = items[j];
                d[nd++] = make_pack(*it.pl, *it.op, it.a, it.c, it.ws);
            }
            if (launch_pack_grouped(q / kNumCls, q % kNumCls, d, nd, dd, s) != hipSuccess) status = FFP_EDEVICE;
        }
        if (status != FFP_OK) break;
    }
    if (meta > 0) {
        const int st = release_staging(s);
        if (status == FFP_OK) status = st;
    }
    return status;
}

ProdTask make_task(const Plan& pl, const Op& o, const void* a, void* c, void* ws)
{
    ProdTask t{};
    init_task(&t, pl.field);
    const bool syrk = o.kind == OP_SYRK;
    t.A = dview(o.v[0], a, c, ws);
    t.B = syrk ? t.A : dview(o.v[1], a, c, ws);
    const PView& cv = syrk ? o.v[1] : o.v[2];
    t.C = (uint32_t*)at(cv, a, c, ws);
    t.ldc = cv.ld;
    t.m = (int32_t)o.m;
    t.n = (int32_t)(syrk ? o.m : o.n);
    t.k = (int32_t)o.k;
    // a SYRK, or a general product restricted to the lower-triangle tiles
    t.syrk = (syrk || (o.kind == OP_GEMM && (o.mode & 1))) ? 1 : 0;
    t.alpha = o.alpha;
    t.beta = o.beta;
    return t;
}

PackDesc make_pack(const Plan& pl, const Op& o, const void* a, void* c, void* ws)
{
    PackDesc d{};
    d.src = dview(o.v[0], a, c, ws);
    d.dst = dview(o.v[1], a, c, ws);
    d.n = o.m_src;
    d.k = o.k_src;
    d.n_pad = o.m;
    d.k_pad = o.k;
    d.p = pl.field.p;
    d.pinv = pl.field.pinv;
    return d;
}

int execute_op(const Plan& pl, const Op& o, const void* a, void* c, void* ws, hipStream_t s)
{
    const FieldPlan& fpl = pl.field;
    const Fp f{fpl.p, (fpl.p - 1) / 2, fpl.pinv, fpl.ya, fpl.yb};
    {
        hipError_t e = hipSuccess;
        switch (o.kind) {
        case OP_S1S2:
            e = launch_preadd_s1s2(o.cls, f, o.m, o.k, dview(o.v[0], a, c, ws), dview(o.v[1], a, c, ws),
                                   dview(o.v[2], a, c, ws), dview(o.v[3], a, c, ws),
                                   dview(o.v[4], a, c, ws), s);
            break;
        case OP_S34:
            e = launch_preadd_s34(o.cls, f, o.mode, o.m, o.k, dview(o.v[0], a, c, ws),
                                  dview(o.v[1], a, c, ws), dview(o.v[2], a, c, ws),
                                  dview(o.v[3], a, c, ws), dview(o.v[4], a, c, ws), s);
            break;
        case OP_GEMM:
        case OP_SYRK: {
            const bool syrk = o.kind == OP_SYRK;
            ProdTask t = make_task(pl, o, a, c, ws);
            hipEvent_t e0 = nullptr;
            const bool prof = prof_enabled();
            if (prof) prof_begin(s, &e0);
            {
                TileHint hint(pl.tile);
                e = launch_products(o.cls, &t, 1, nullptr, s);
            }
            if (prof) {
                const double flops = syrk ? (double)t.m * (double)(t.m + 1) * (double)t.k
                                          : 2.0 * (double)t.m * (double)t.n * (double)t.k;
                prof_end(s, e0, flops, o.cls);
            }
            break;
        }
        case OP_POSTADD:
            e = launch_postadd(f, o.m, (const uint32_t*)at(o.v[0], a, c, ws), o.v[0].ld,
                               (const uint32_t*)at(o.v[1], a, c, ws), o.v[1].ld,
                               (uint32_t*)at(o.v[2], a, c, ws), o.v[2].ld,
                               (uint32_t*)at(o.v[3], a, c, ws), o.v[3].ld, o.beta,
                               o.beta ? (const uint32_t*)at(o.v[4], a, c, ws) : nullptr, o.v[4].ld,
                               o.beta ? (const uint32_t*)at(o.v[5], a, c, ws) : nullptr, s);
            break;
        case OP_ADDLOW:
            e = launch_add_lower(f, o.m, (const uint32_t*)at(o.v[0], a, c, ws), o.v[0].ld,
                                 (const uint32_t*)at(o.v[1], a, c, ws), o.v[1].ld,
                                 (uint32_t*)at(o.v[2], a, c, ws), o.v[2].ld, s);
            break;
        case OP_SAVEC22:
            e = launch_save_c22(o.m, (const uint32_t*)at(o.v[0], a, c, ws), o.v[0].ld,
                                (uint32_t*)at(o.v[1], a, c, ws), o.v[1].ld,
                                (uint32_t*)at(o.v[2], a, c, ws), s);
            break;
        case OP_MIRROR:
            e = (o.mode & 1) ? launch_mirror_lower_neg(fpl.p, o.m, (uint32_t*)at(o.v[0], a, c, ws), o.v[0].ld, s)
                             : launch_mirror_lower(o.m, (uint32_t*)at(o.v[0], a, c, ws), o.v[0].ld, s);
            break;
        case OP_PACK:
            e = launch_pack(f, o.src_cls, dview(o.v[0], a, c, ws), o.m_src, o.k_src, o.cls,
                            dview(o.v[1], a, c, ws), o.m, o.k, s);
            break;
        case OP_COPY:
            e = launch_copy_u32(o.m, o.n, (const uint32_t*)at(o.v[0], a, c, ws), o.v[0].ld,
                                (uint32_t*)at(o.v[1], a, c, ws), o.v[1].ld, o.mode & 1, s);
            break;
        case OP_LINCOMB: {
            DView in[5] = {};
            for (int i = 0; i < (o.mode & 7); ++i) in[i] = dview(o.v[i], a, c, ws);
            e = launch_lincomb(f, o.m, o.k, o.mode & 7, in, (unsigned)(o.mode >> 3), dview(o.v[5], a, c, ws), s);
            break;
        }
        case OP_LCT: {
            DView in[5] = {};
            for (int i = 0; i < (o.mode & 7); ++i) in[i] = dview(o.v[i], a, c, ws);
            e = launch_lct(f, o.m, o.k, o.mode & 7, in, o.coef, (unsigned)((o.mode >> 3) & 31), (o.mode >> 8) & 1,
                           dview(o.v[5], a, c, ws), s);
            break;
        }
        }
        if (e != hipSuccess) return FFP_EDEVICE;
    }
    return FFP_OK;
}

}  // namespace ffp
