// Request loop with continuous (iteration-level) batching for A*A^T and
// LDL^T jobs.  The scheduler is written against a small device interface so
// that its admission and batching logic also runs against a simulated device
// (no computation) in host-only tests.
#pragma once
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <list>
#include <mutex>
#include <thread>
#include <vector>

#include "ffp.h"

namespace ffp {

// Requests per unit part (tuning knobs; at least 1).
extern int g_serve_batch;
extern int g_serve_ldlt_batch;

struct ServeReq {
    ffp_request rq;
    uint64_t ticket = 0;
    int state = FFP_STATE_QUEUED;
    size_t bytes = 0;        // arena bytes held for the result until release
    size_t off = 0;          // offset of the result in the arena
    size_t ws_bytes = 0;     // arena bytes of workspace, held while running
    size_t ws_off = 0;
    unsigned flags = 0;      // A*A^T: depth and placements fixed at submission
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = FFP_OK;
    bool released = false;
    double deadline = 0;     // steady-clock time after which a queued request times out (0: none)
    void* fetch_ev = nullptr; // real device: hipEvent_t recorded after the last fetch's copies
};

// One batch of a unit: its requests complete together.
struct UnitPart {
    std::vector<uint64_t> tickets;
    double sim_done = 0;     // simulated device: completion time
    void* event = nullptr;   // real device: hipEvent_t
    bool finished = false;
};

// One unit of work on a stream: the admitted A*A^T requests as one batched
// launch (part 0), then the admitted LDL^T requests as one
// multi-factorisation (part 1).  The stream's launch thread enqueues it;
// completions are only checked once it has been enqueued.
struct Unit {
    int stream = -1;
    double t_launch = 0;
    UnitPart part[2];
    std::vector<ServeReq*> batch[2];
    bool launched = false;
};

class DeviceIface {
public:
    virtual ~DeviceIface() = default;
    virtual int init(size_t arena_bytes, int nstreams) = 0;
    virtual void bind_thread() {}   // called first on the scheduler and launch threads
    virtual char* arena() = 0;
    // Enqueue a batch of SYRK (or of LDLT) requests, results at arena + off,
    // on stream s.
    virtual int launch_syrk(std::vector<ServeReq*>& batch, int s, UnitPart* u) = 0;
    virtual int launch_ldlt(std::vector<ServeReq*>& batch, int s, UnitPart* u) = 0;
    virtual bool done(UnitPart* u) = 0;
    virtual void sync_stream(int) {}
    virtual void release(UnitPart* u) = 0;
};

DeviceIface* make_hip_device();
DeviceIface* make_sim_device(double ns_per_op, double launch_us);

class Server {
public:
    Server(DeviceIface* dev, size_t budget, int max_inflight, int nstreams);
    ~Server();
    int start();
    int submit(const ffp_request* rq, uint64_t* ticket);
    int status(uint64_t ticket, ffp_result* out);
    int release(uint64_t ticket);
    int drain(double timeout_s);
    void finish_part(UnitPart& part, int status);
    int poll(uint64_t* tickets, int max, double timeout_s, int* count);
    int fetch(uint64_t ticket, uint32_t* dst, int64_t ldd, int64_t* info_dst, void* stream);
    int cancel(uint64_t ticket);
    int stats(ffp_serve_stats* out);

private:
    void loop();
    void launcher(int s);
    bool arena_alloc(size_t bytes, size_t* off);
    void arena_free(size_t off, size_t bytes);
    void expire_queued(double now);
    void reap_deferred();
    void fail_queued(ServeReq& q, int status, double now);

    DeviceIface* dev_;
    size_t budget_;
    int max_inflight_, nstreams_;
    std::mutex mu_;
    std::condition_variable cv_, cv_done_, cv_launch_;
    std::thread th_;
    std::vector<std::thread> launchers_;   // one per stream
    std::vector<Unit*> pending_;           // per stream: a unit to enqueue
    bool stop_ = false;
    bool sched_done_ = false;              // the scheduler has returned: launch threads end
    std::deque<uint64_t> queue_;           // submitted, not admitted (FIFO)
    std::deque<ServeReq> reqs_;            // by ticket - 1 (stable addresses)
    std::deque<uint64_t> done_q_;          // finished, not yet returned by poll
    std::list<Unit> running_;              // admitted units (stable addresses)
    std::vector<char> stream_busy_;
    std::vector<std::pair<size_t, size_t>> free_;   // (offset, size), sorted
    // released results whose memory a pending fetch copy still reads:
    // (offset, bytes, event recorded after the copy)
    struct Deferred {
        size_t off, bytes;
        void* ev;
    };
    std::vector<Deferred> deferred_;
    int64_t n_deadlines_ = 0;              // queued requests with a deadline
    double next_expiry_check_ = 0;
    size_t used_ = 0, peak_used_ = 0;
    int inflight_ = 0, peak_inflight_ = 0;
    int64_t units_ = 0, batched_jobs_ = 0, max_batch_ = 0, overlap_units_ = 0;
};

}  // namespace ffp
