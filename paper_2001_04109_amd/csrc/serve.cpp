// Request loop with continuous batching (see serve.h and include/ffp.h).
#include "serve.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

#include "batch.h"
#include "field.h"
#include "ldlt.h"
#include "tune.h"

namespace ffp {

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

int64_t result_ld(const ffp_request& r) { return rup(r.n > 0 ? r.n : 1, 4); }

size_t result_bytes(const ffp_request& r)
{
    size_t b = (size_t)r.n * (size_t)result_ld(r) * 4;
    if (r.kind == FFP_REQ_LDLT) b = (size_t)rup((int64_t)b, 256) + 256;   // + info
    return (size_t)rup((int64_t)b, 256);
}

}  // namespace

int g_serve_batch = 128;      // A*A^T requests per unit
int g_serve_ldlt_batch = 32;  // LDL^T requests per unit

namespace {

// Workspace the request needs while it runs (the same figure the batched
// launch and the LDL^T driver use for it).
ffp_job syrk_job(const ffp_request& r)
{
    ffp_job j{};
    j.n = r.n;
    j.k = r.k;
    j.p = r.p;
    j.alpha = r.alpha;
    j.beta = 0;
    j.a_dtype = FFP_U32;
    j.A = r.A;
    j.lda = r.lda;
    j.C = (uint32_t*)(uintptr_t)256;   // results are 256-byte aligned in the arena
    j.ldc = result_ld(r);
    return j;
}

// Flags that fix the request's depth and placements at submission (from
// the tuning table or the built-in rule).
unsigned pinned_flags(const ffp_request& r)
{
    if (r.kind != FFP_REQ_SYRK || r.n == 0) return 0;
    return pin_flags(syrk_job(r), 0);
}

// Workspace the request needs while it runs (the same figure the batched
// launch and the LDL^T driver use for it).
size_t workspace_bytes(const ffp_request& r, unsigned flags)
{
    if (r.n == 0) return 0;
    if (r.kind == FFP_REQ_LDLT) return (size_t)rup((int64_t)ldlt_workspace_bytes(r.n, r.p, result_ld(r)), 256);
    return (size_t)job_workspace_bytes(syrk_job(r), flags);
}

// ---- device backed by HIP --------------------------------------------------
class HipDevice : public DeviceIface {
public:
    ~HipDevice() override
    {
        for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
        if (arena_) (void)hipFree(arena_);
    }
    int init(size_t arena_bytes, int nstreams) override
    {
        if (hipGetDevice(&device_) != hipSuccess) return FFP_EDEVICE;
        if (hipMalloc((void**)&arena_, arena_bytes ? arena_bytes : 256) != hipSuccess) {
            arena_ = nullptr;
            (void)hipGetLastError();
            return FFP_ENOMEM;
        }
        for (int i = 0; i < nstreams; ++i) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return FFP_EDEVICE;
            streams_.push_back(s);
        }
        return FFP_OK;
    }
    void bind_thread() override { (void)hipSetDevice(device_); }
    char* arena() override { return arena_; }
    int launch_syrk(std::vector<ServeReq*>& batch, int s, UnitPart* u) override
    {
        std::vector<ffp_job> jobs;
        std::vector<char*> ws;
        std::vector<unsigned> flags;
        jobs.reserve(batch.size());
        for (ServeReq* r : batch) {
            ffp_job j{};
            j.n = r->rq.n;
            j.k = r->rq.k;
            j.p = r->rq.p;
            j.alpha = r->rq.alpha;
            j.beta = 0;
            j.a_dtype = FFP_U32;
            j.A = r->rq.A;
            j.lda = r->rq.lda;
            j.C = (uint32_t*)(arena_ + r->off);
            j.ldc = result_ld(r->rq);
            jobs.push_back(j);
            ws.push_back(r->ws_bytes ? arena_ + r->ws_off : nullptr);
            flags.push_back(r->flags);
        }
        int st = batched_run((int)jobs.size(), jobs.data(), 0, streams_[s], ws.data(), flags.data());
        if (st != FFP_OK) return st;
        return record(s, u);
    }
    int launch_ldlt(std::vector<ServeReq*>& batch, int s, UnitPart* u) override
    {
        std::vector<LdltJobSpec> jobs;
        jobs.reserve(batch.size());
        for (ServeReq* r : batch) {
            const int64_t n = r->rq.n, ld = result_ld(r->rq);
            uint32_t* S = (uint32_t*)(arena_ + r->off);
            int64_t* info = (int64_t*)(arena_ + r->off + rup(n * ld * 4, 256));
            if (n > 0 && hipMemcpy2DAsync(S, ld * 4, r->rq.A, r->rq.lda * 4, n * 4, n,
                                          hipMemcpyDeviceToDevice, streams_[s]) != hipSuccess)
                return FFP_EDEVICE;
            jobs.push_back(LdltJobSpec{n, r->rq.p, S, ld, info, arena_ + r->ws_off});
        }
        int st = ldlt_run_multi(jobs, streams_[s]);
        if (st != FFP_OK) return st;
        return record(s, u);
    }
    bool done(UnitPart* u) override
    {
        return hipEventQuery((hipEvent_t)u->event) == hipSuccess;
    }
    void sync_stream(int s) override { (void)hipStreamSynchronize(streams_[s]); }
    void release(UnitPart* u) override
    {
        if (u->event) (void)hipEventDestroy((hipEvent_t)u->event);
        u->event = nullptr;
    }

private:
    int record(int s, UnitPart* u)
    {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return FFP_EDEVICE;
        if (hipEventRecord(e, streams_[s]) != hipSuccess) return FFP_EDEVICE;
        u->event = e;
        return FFP_OK;
    }
    char* arena_ = nullptr;
    int device_ = 0;
    std::vector<hipStream_t> streams_;
};

// ---- simulated device: no computation, completion after a modelled time ----
class SimDevice : public DeviceIface {
public:
    SimDevice(double ns_per_op, double launch_us) : ns_(ns_per_op), launch_(launch_us) {}
    int init(size_t, int nstreams) override
    {
        free_at_.assign(nstreams, 0.0);
        return FFP_OK;
    }
    char* arena() override { return nullptr; }
    int launch_syrk(std::vector<ServeReq*>& batch, int s, UnitPart* u) override
    {
        double ops = 0;
        for (ServeReq* r : batch) ops += (double)r->rq.n * r->rq.n * r->rq.k;
        return finish(s, u, ops);
    }
    int launch_ldlt(std::vector<ServeReq*>& batch, int s, UnitPart* u) override
    {
        double ops = 0;
        for (ServeReq* r : batch) ops += (double)r->rq.n * r->rq.n * r->rq.n / 3.0;
        return finish(s, u, ops);
    }
    bool done(UnitPart* u) override { return now_s() >= u->sim_done; }
    void release(UnitPart*) override {}

private:
    int finish(int s, UnitPart* u, double ops)
    {
        const double start = std::max(now_s(), free_at_[s]);
        u->sim_done = start + launch_ * 1e-6 + ops * ns_ * 1e-9;
        free_at_[s] = u->sim_done;
        return FFP_OK;
    }
    double ns_, launch_;
    std::vector<double> free_at_;
};

}  // namespace

DeviceIface* make_hip_device() { return new HipDevice(); }
DeviceIface* make_sim_device(double ns_per_op, double launch_us)
{
    return new SimDevice(ns_per_op, launch_us);
}

Server::Server(DeviceIface* dev, size_t budget, int max_inflight, int nstreams)
    : dev_(dev), budget_(budget), max_inflight_(max_inflight), nstreams_(nstreams)
{
    stream_busy_.assign(nstreams, 0);
    pending_.assign(nstreams, nullptr);
    free_.push_back({0, budget});
}

Server::~Server()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (th_.joinable()) th_.join();   // returns once every unit has finished
    {
        std::lock_guard<std::mutex> lk(mu_);
        sched_done_ = true;
    }
    cv_launch_.notify_all();
    for (std::thread& t : launchers_)
        if (t.joinable()) t.join();
    // fetch events (only a HIP device has them): pending copies finish first
    for (Deferred& d : deferred_) {
        (void)hipEventSynchronize((hipEvent_t)d.ev);
        (void)hipEventDestroy((hipEvent_t)d.ev);
    }
    deferred_.clear();
    for (ServeReq& q : reqs_)
        if (q.fetch_ev) {
            (void)hipEventSynchronize((hipEvent_t)q.fetch_ev);
            (void)hipEventDestroy((hipEvent_t)q.fetch_ev);
            q.fetch_ev = nullptr;
        }
    delete dev_;
}

int Server::start()
{
    int st = dev_->init(budget_, nstreams_);
    if (st != FFP_OK) return st;
    for (int s = 0; s < nstreams_; ++s) launchers_.emplace_back([this, s] { launcher(s); });
    th_ = std::thread([this] { loop(); });
    return FFP_OK;
}

// Enqueues the units the scheduler hands to stream s.  Units of different
// streams are enqueued by their own threads, so the host work of one
// (schedules, thousands of launches for a batch of factorisations) does not
// hold up the others.
void Server::launcher(int s)
{
    dev_->bind_thread();
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        cv_launch_.wait(lk, [&] { return pending_[s] != nullptr || sched_done_; });
        Unit* u = pending_[s];
        if (!u) return;   // the scheduler has finished: nothing more to enqueue
        pending_[s] = nullptr;
        // the admitted entries are not touched by other threads while
        // RUNNING (reqs_ is a deque: addresses are stable), nor is the unit
        // until it is marked launched
        lk.unlock();
        int st[2] = {FFP_OK, FFP_OK};
        if (!u->batch[0].empty()) st[0] = dev_->launch_syrk(u->batch[0], s, &u->part[0]);
        if (!u->batch[1].empty()) st[1] = dev_->launch_ldlt(u->batch[1], s, &u->part[1]);
        if (st[0] != FFP_OK || st[1] != FFP_OK) dev_->sync_stream(s);   // nothing may still run
        lk.lock();
        for (int k = 0; k < 2; ++k)
            if (!u->batch[k].empty() && st[k] != FFP_OK) finish_part(u->part[k], st[k]);
        u->launched = true;
        cv_.notify_all();
        cv_done_.notify_all();
    }
}


bool Server::arena_alloc(size_t bytes, size_t* off)
{
    for (size_t i = 0; i < free_.size(); ++i) {
        if (free_[i].second >= bytes) {
            *off = free_[i].first;
            free_[i].first += bytes;
            free_[i].second -= bytes;
            if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
            return true;
        }
    }
    return false;
}

void Server::arena_free(size_t off, size_t bytes)
{
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
    it = free_.insert(it, {off, bytes});
    // coalesce with neighbours
    size_t i = (size_t)(it - free_.begin());
    if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
        free_[i].second += free_[i + 1].second;
        free_.erase(free_.begin() + (long)i + 1);
    }
    if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
        free_[i - 1].second += free_[i].second;
        free_.erase(free_.begin() + (long)i);
    }
}

// Marks the requests of a part done (with a failure status unless FFP_OK)
// and returns their workspace to the arena.  Called with the lock held.
void Server::finish_part(UnitPart& part, int status)
{
    const double t = now_s();
    for (uint64_t tk : part.tickets) {
        ServeReq& q = reqs_[tk - 1];
        if (status != FFP_OK) q.status = status;
        q.state = FFP_STATE_DONE;
        q.t_done = t;
        --inflight_;
        if (q.ws_bytes) {
            arena_free(q.ws_off, q.ws_bytes);
            used_ -= q.ws_bytes;
        }
        done_q_.push_back(tk);
    }
    part.finished = true;
    dev_->release(&part);
    cv_done_.notify_all();
}

int Server::submit(const ffp_request* r, uint64_t* ticket)
{
    if (!r || !ticket) return FFP_EINVAL;
    if (r->kind != FFP_REQ_SYRK && r->kind != FFP_REQ_LDLT) return FFP_EINVAL;
    if (r->n < 0 || r->n > ((int64_t)1 << 20)) return FFP_EINVAL;
    if (!supported_prime(r->p) || (r->kind == FFP_REQ_LDLT && r->p < 3)) return FFP_EPRIME;
    if (r->kind == FFP_REQ_SYRK) {
        if (r->k < 0 || r->alpha >= r->p) return FFP_EINVAL;
        if (r->n > 0 && r->k > 0 && (r->A == nullptr || r->lda < r->k)) return FFP_EINVAL;
    } else {
        if (r->n > 0 && (r->A == nullptr || r->lda < r->n)) return FFP_EINVAL;
    }
    ServeReq q;
    q.rq = *r;
    if (q.rq.kind == FFP_REQ_LDLT) q.rq.k = q.rq.n;
    q.bytes = result_bytes(q.rq);
    q.flags = pinned_flags(q.rq);
    q.ws_bytes = workspace_bytes(q.rq, q.flags);
    if (q.bytes + q.ws_bytes > budget_) return FFP_ENOMEM;
    if (!(r->timeout_s >= 0.0)) return FFP_EINVAL;
    {
        std::lock_guard<std::mutex> lk(mu_);
        q.ticket = reqs_.size() + 1;
        q.t_submit = now_s();
        if (r->timeout_s > 0.0) {
            q.deadline = q.t_submit + r->timeout_s;
            ++n_deadlines_;
        }
        reqs_.push_back(q);
        queue_.push_back(q.ticket);
        *ticket = q.ticket;
    }
    cv_.notify_all();
    return FFP_OK;
}

// A queued request leaves the queue as done with a failure status (cancel,
// deadline).  Called with the lock held; the caller removes it from queue_.
void Server::fail_queued(ServeReq& q, int status, double now)
{
    q.status = status;
    q.state = FFP_STATE_DONE;
    q.t_done = now;
    q.released = true;   // holds no memory
    if (q.deadline > 0.0) --n_deadlines_;
    done_q_.push_back(q.ticket);
}

int Server::cancel(uint64_t ticket)
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (ticket == 0 || ticket > reqs_.size()) return FFP_EINVAL;
        ServeReq& q = reqs_[ticket - 1];
        if (q.state != FFP_STATE_QUEUED) return FFP_EINVAL;   // admitted work is not interrupted
        auto it = std::find(queue_.begin(), queue_.end(), ticket);
        if (it == queue_.end()) return FFP_EINVAL;
        queue_.erase(it);
        fail_queued(q, FFP_ECANCELED, now_s());
    }
    cv_done_.notify_all();
    cv_.notify_all();
    return FFP_OK;
}

// Queued requests whose deadline has passed fail with FFP_ETIMEDOUT.  Called
// with the lock held.
void Server::expire_queued(double now)
{
    if (n_deadlines_ == 0 || now < next_expiry_check_) return;
    next_expiry_check_ = now + 1e-4;
    for (auto it = queue_.begin(); it != queue_.end();) {
        ServeReq& q = reqs_[*it - 1];
        if (q.deadline > 0.0 && now >= q.deadline) {
            fail_queued(q, FFP_ETIMEDOUT, now);
            it = queue_.erase(it);
        } else {
            ++it;
        }
    }
}

// Released results whose last fetch copy has executed return to the arena.
// Called with the lock held.
void Server::reap_deferred()
{
    for (size_t i = 0; i < deferred_.size();) {
        Deferred& d = deferred_[i];
        const hipError_t e = hipEventQuery((hipEvent_t)d.ev);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        (void)hipGetLastError();
        (void)hipEventDestroy((hipEvent_t)d.ev);
        arena_free(d.off, d.bytes);
        used_ -= d.bytes;
        deferred_[i] = deferred_.back();
        deferred_.pop_back();
    }
}

int Server::status(uint64_t ticket, ffp_result* out)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (ticket == 0 || ticket > reqs_.size() || !out) return FFP_EINVAL;
    const ServeReq& q = reqs_[ticket - 1];
    memset(out, 0, sizeof *out);
    out->state = q.status != FFP_OK ? q.status : q.state;
    out->t_submit = q.t_submit;
    out->t_admit = q.t_admit;
    out->t_done = q.t_done;
    char* base = dev_->arena();
    if (q.state != FFP_STATE_QUEUED && !q.released && base) {
        out->C = (uint32_t*)(base + q.off);
        out->ldc = result_ld(q.rq);
        if (q.rq.kind == FFP_REQ_LDLT)
            out->info = (int64_t*)(base + q.off + rup(q.rq.n * result_ld(q.rq) * 4, 256));
    }
    return FFP_OK;
}

int Server::release(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (ticket == 0 || ticket > reqs_.size()) return FFP_EINVAL;
    ServeReq& q = reqs_[ticket - 1];
    if (q.state != FFP_STATE_DONE) return FFP_EINVAL;
    if (!q.released) {
        q.released = true;
        if (q.fetch_ev) {
            // a fetch copy enqueued on the caller's stream may still read the
            // result: its memory returns to the arena once the copy has run
            deferred_.push_back(Deferred{q.off, q.bytes, q.fetch_ev});
            q.fetch_ev = nullptr;
        } else {
            arena_free(q.off, q.bytes);
            used_ -= q.bytes;
        }
    }
    cv_.notify_all();
    return FFP_OK;
}

int Server::drain(double timeout_s)
{
    std::unique_lock<std::mutex> lk(mu_);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(timeout_s));
    auto idle = [this] { return queue_.empty() && running_.empty(); };
    while (!idle()) {
        if (cv_done_.wait_until(lk, deadline) == std::cv_status::timeout && !idle()) return FFP_EDEVICE;
    }
    return FFP_OK;
}

int Server::poll(uint64_t* tickets, int max, double timeout_s, int* count)
{
    if (!tickets || !count || max < 1) return FFP_EINVAL;
    std::unique_lock<std::mutex> lk(mu_);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 0.0));
    while (done_q_.empty() && timeout_s > 0) {
        if (cv_done_.wait_until(lk, deadline) == std::cv_status::timeout) break;
    }
    int n = 0;
    while (n < max && !done_q_.empty()) {
        tickets[n++] = done_q_.front();
        done_q_.pop_front();
    }
    *count = n;
    return FFP_OK;
}

int Server::fetch(uint64_t ticket, uint32_t* dst, int64_t ldd, int64_t* info_dst, void* stream)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (ticket == 0 || ticket > reqs_.size()) return FFP_EINVAL;
    ServeReq& q = reqs_[ticket - 1];
    char* base = dev_->arena();
    if (!base || q.state != FFP_STATE_DONE || q.status != FFP_OK || q.released) return FFP_EINVAL;
    const int64_t n = q.rq.n, ld = result_ld(q.rq);
    if (n == 0) return FFP_OK;
    if (!dst || ldd < n) return FFP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpy2DAsync(dst, ldd * 4, base + q.off, ld * 4, n * 4, n, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return FFP_EDEVICE;
    if (q.rq.kind == FFP_REQ_LDLT && info_dst &&
        hipMemcpyAsync(info_dst, base + q.off + rup(n * ld * 4, 256), sizeof(int64_t),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return FFP_EDEVICE;
    // release() keeps the result's memory until these copies have executed
    if (!q.fetch_ev &&
        hipEventCreateWithFlags((hipEvent_t*)&q.fetch_ev, hipEventDisableTiming) != hipSuccess) {
        q.fetch_ev = nullptr;
        return FFP_EDEVICE;
    }
    if (hipEventRecord((hipEvent_t)q.fetch_ev, s) != hipSuccess) return FFP_EDEVICE;
    return FFP_OK;
}

int Server::stats(ffp_serve_stats* out)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (!out) return FFP_EINVAL;
    memset(out, 0, sizeof *out);
    out->submitted = (int64_t)reqs_.size();
    for (const ServeReq& q : reqs_) out->completed += q.state == FFP_STATE_DONE;
    out->units = units_;
    out->batched_jobs = batched_jobs_;
    out->max_batch = max_batch_;
    out->peak_inflight = peak_inflight_;
    out->overlapped_units = overlap_units_;
    out->peak_bytes = peak_used_;
    return FFP_OK;
}

void Server::loop()
{
    dev_->bind_thread();
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool progress = false;
        if (!deferred_.empty()) reap_deferred();
        {
            const size_t before = done_q_.size();
            expire_queued(now_s());
            if (done_q_.size() != before) progress = true;
        }
        // completions, part by part (of enqueued units)
        for (auto it = running_.begin(); it != running_.end();) {
            Unit& u = *it;
            if (!u.launched) {
                ++it;
                continue;
            }
            bool all = true;
            for (UnitPart& part : u.part) {
                if (part.tickets.empty() || part.finished) continue;
                if (dev_->done(&part)) {
                    finish_part(part, FFP_OK);
                    progress = true;
                } else {
                    all = false;
                }
            }
            if (all) {
                stream_busy_[u.stream] = 0;
                it = running_.erase(it);
                progress = true;
            } else {
                ++it;
            }
        }
        if (progress) cv_done_.notify_all();
        // admission and launch, one unit per free stream
        for (int s = 0; s < nstreams_ && !queue_.empty(); ++s) {
            if (stream_busy_[s]) continue;
            // a unit: the requests at the head of the queue, in arrival order,
            // while they fit (A*A^T and LDL^T requests go to their own batch)
            std::vector<ServeReq*> batch[2];
            while (!queue_.empty()) {
                ServeReq& q = reqs_[queue_.front() - 1];
                const int kind = q.rq.kind == FFP_REQ_LDLT ? 1 : 0;
                if ((int)batch[kind].size() >= (kind ? g_serve_ldlt_batch : g_serve_batch)) break;
                const size_t need = q.bytes + q.ws_bytes;
                size_t off = 0, ws_off = 0;
                if (inflight_ >= max_inflight_ || used_ + need > budget_ || !arena_alloc(q.bytes, &off))
                    break;
                if (q.ws_bytes && !arena_alloc(q.ws_bytes, &ws_off)) {
                    arena_free(off, q.bytes);
                    break;
                }
                q.off = off;
                q.ws_off = ws_off;
                used_ += need;
                peak_used_ = std::max(peak_used_, used_);
                q.state = FFP_STATE_RUNNING;
                q.t_admit = now_s();
                ++inflight_;
                peak_inflight_ = std::max<int64_t>(peak_inflight_, inflight_);
                queue_.pop_front();
                batch[kind].push_back(&q);
            }
            if (batch[0].empty() && batch[1].empty()) break;
            running_.emplace_back();
            Unit& u = running_.back();
            u.stream = s;
            u.t_launch = now_s();
            for (int k = 0; k < 2; ++k) {
                for (ServeReq* q : batch[k]) u.part[k].tickets.push_back(q->ticket);
                batched_jobs_ += (int64_t)batch[k].size();
                max_batch_ = std::max<int64_t>(max_batch_, (int64_t)batch[k].size());
                u.batch[k] = std::move(batch[k]);
            }
            if (running_.size() > 1) ++overlap_units_;
            ++units_;
            stream_busy_[s] = 1;
            // the stream's launch thread enqueues it
            pending_[s] = &u;
            cv_launch_.notify_all();
            progress = true;
        }
        if (stop_ && running_.empty()) break;
        if (!progress) cv_.wait_for(lk, std::chrono::microseconds(running_.empty() ? 2000 : 20));
    }
}

}  // namespace ffp

using ffp::Server;

struct ffp_server {
    Server* impl;
};

extern "C" {

int ffp_server_create(size_t hbm_budget, int max_inflight, int nstreams, ffp_server** out)
{
    if (!out || max_inflight < 1 || nstreams < 1 || nstreams > 16 || hbm_budget == 0) return FFP_EINVAL;
    Server* s = new Server(ffp::make_hip_device(), hbm_budget, max_inflight, nstreams);
    int st = s->start();
    if (st != FFP_OK) {
        delete s;
        return st;
    }
    *out = new ffp_server{s};
    return FFP_OK;
}

int ffp_server_create_simulated(size_t budget, int max_inflight, int nstreams, double ns_per_op,
                                double launch_us, ffp_server** out)
{
    if (!out || max_inflight < 1 || nstreams < 1 || nstreams > 16 || budget == 0) return FFP_EINVAL;
    Server* s = new Server(ffp::make_sim_device(ns_per_op, launch_us), budget, max_inflight, nstreams);
    int st = s->start();
    if (st != FFP_OK) {
        delete s;
        return st;
    }
    *out = new ffp_server{s};
    return FFP_OK;
}

int ffp_server_submit(ffp_server* s, const ffp_request* r, uint64_t* ticket)
{
    return s ? s->impl->submit(r, ticket) : FFP_EINVAL;
}

int ffp_server_status(ffp_server* s, uint64_t ticket, ffp_result* out)
{
    return s ? s->impl->status(ticket, out) : FFP_EINVAL;
}

int ffp_server_release(ffp_server* s, uint64_t ticket)
{
    return s ? s->impl->release(ticket) : FFP_EINVAL;
}

int ffp_server_drain(ffp_server* s, double timeout_s)
{
    return s ? s->impl->drain(timeout_s) : FFP_EINVAL;
}

int ffp_server_poll(ffp_server* s, uint64_t* tickets, int max, double timeout_s, int* count)
{
    return s ? s->impl->poll(tickets, max, timeout_s, count) : FFP_EINVAL;
}

int ffp_server_fetch(ffp_server* s, uint64_t ticket, uint32_t* dst, int64_t ldd, int64_t* info_dst,
                     void* stream)
{
    return s ? s->impl->fetch(ticket, dst, ldd, info_dst, stream) : FFP_EINVAL;
}

int ffp_server_cancel(ffp_server* s, uint64_t ticket)
{
    return s ? s->impl->cancel(ticket) : FFP_EINVAL;
}

int ffp_server_stats(ffp_server* s, ffp_serve_stats* out)
{
    return s ? s->impl->stats(out) : FFP_EINVAL;
}

int ffp_server_destroy(ffp_server* s)
{
    if (!s) return FFP_EINVAL;
    delete s->impl;
    delete s;
    return FFP_OK;
}

}  // extern "C"
