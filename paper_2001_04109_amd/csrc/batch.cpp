// Batched form of fsyrk_modp: many independent jobs of uneven n, k and p.
//
// Every job gets its own schedule (Algorithm 2 at the depth of the tuning
// table, or of the built-in rule).  All
// jobs' operations go through the level scheduler as one program: an
// operation's level only depends on earlier operations of its own job, and
// the products of one class (and the packs) of all jobs on one level run
// as one grouped persistent launch, tiles longest first; other block
// operations run per job.  Each job only touches its own A, C and
// workspace slice, so results are bit-identical to the job run alone.
#include <vector>

#include "batch.h"
#include "ffp.h"
#include "runtime.h"

namespace ffp {

namespace {

int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

}  // namespace

int64_t job_workspace_bytes(const ffp_job& jb, unsigned flags)
{
    PlanRequest rq;
    if (make_syrk_request(jb.n, jb.k, jb.p, jb.A, jb.lda, jb.a_dtype, jb.alpha, jb.beta, jb.C, jb.ldc,
                          flags, &rq) != FFP_OK || jb.n == 0)
        return 0;
    Plan pl;
    if (build_syrk_plan(rq, &pl) != FFP_OK) return 0;
    return rup(pl.ws_bytes, 256);
}

int batched_run(int njobs, const ffp_job* jobs, unsigned flags, hipStream_t s, char* const* job_ws,
                const unsigned* job_flags)
{
    if (njobs < 0 || (njobs > 0 && jobs == nullptr)) return FFP_EINVAL;
    std::vector<Plan> plans(njobs);
    std::vector<int64_t> wsoff(njobs, 0);
    std::vector<char> live(njobs, 0);
    int64_t ws_total = 0;
    for (int j = 0; j < njobs; ++j) {
        const ffp_job& jb = jobs[j];
        PlanRequest rq;
        int st = make_syrk_request(jb.n, jb.k, jb.p, jb.A, jb.lda, jb.a_dtype, jb.alpha, jb.beta, jb.C,
                                   jb.ldc, job_flags ? job_flags[j] : flags, &rq);
        if (st != FFP_OK) return st;
        if (jb.n == 0) continue;
        st = build_syrk_plan(rq, &plans[j]);
        if (st != FFP_OK) return st;
        live[j] = 1;
        wsoff[j] = ws_total;
        ws_total += rup(plans[j].ws_bytes, 256);
    }
    std::vector<char*> jws(njobs, nullptr);
    if (job_ws) {
        for (int j = 0; j < njobs; ++j) jws[j] = job_ws[j];
    } else if (ws_total > 0) {
        Workspace* w = nullptr;
        const int st = acquire_workspace(s, (size_t)ws_total, 0, &w);
        if (st != FFP_OK) return st;
        for (int j = 0; j < njobs; ++j) jws[j] = (char*)w->ptr + wsoff[j];
    }
    // every job's operations, job after job; the level scheduler groups the
    // independent products (and packs) of all jobs level by level
    std::vector<SchedItem> items;
    for (int j = 0; j < njobs; ++j) {
        if (!live[j]) continue;
        for (const Op& o : plans[j].ops) items.push_back(SchedItem{&plans[j], &o, jobs[j].A, jobs[j].C, jws[j], j});
    }
    return run_leveled(items, s);
}

}  // namespace ffp
