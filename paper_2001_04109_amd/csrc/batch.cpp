// Batched form of fsyrk_modp: many independent jobs of uneven n, k and p.
//
// Every job gets its own schedule (Tables 3/4, depth from the tuned
// default).  Jobs whose schedules have the same sequence of operation kinds
// and classes form a group; a group is executed operation by operation, and
// the products and representation changes of all its jobs at one position
// run as one grouped launch (products of one class share one persistent
// launch of the product kernel, tasks ordered longest first).  Other block
// operations are launched per job.  Each job only touches its own A, C and
// workspace slice, so results are bit-identical to the job run alone.
#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "batch.h"
#include "ffp.h"
#include "runtime.h"

namespace ffp {

namespace {

int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

std::string signature(const Plan& pl)
{
    std::string s = std::to_string(pl.cls) + ":";
    for (const Op& o : pl.ops) {
        s += std::to_string((int)o.kind);
        s += ",";
        s += std::to_string(o.cls);
        s += ",";
        s += std::to_string(o.src_cls);
        s += ";";
    }
    return s;
}

// Work of one tile row: k (the products' tiles differ only by their k).
bool longer(const ProdTask& a, const ProdTask& b)
{
    if (a.k != b.k) return a.k > b.k;
    return (int64_t)a.m * a.n > (int64_t)b.m * b.n;
}

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

int batched_run(int njobs, const ffp_job* jobs, unsigned flags, hipStream_t s, char* const* job_ws)
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
                                   jb.ldc, flags, &rq);
        if (st != FFP_OK) return st;
        if (jb.n == 0) continue;
        st = build_syrk_plan(rq, &plans[j]);
        if (st != FFP_OK) return st;
        live[j] = 1;
        wsoff[j] = ws_total;
        ws_total += rup(plans[j].ws_bytes, 256);
    }
    // group jobs by schedule signature, in order of first appearance
    std::map<std::string, int> gidx;
    std::vector<std::vector<int>> groups;
    for (int j = 0; j < njobs; ++j) {
        if (!live[j]) continue;
        const std::string sig = signature(plans[j]);
        auto it = gidx.find(sig);
        if (it == gidx.end()) {
            gidx[sig] = (int)groups.size();
            groups.push_back({j});
        } else {
            groups[it->second].push_back(j);
        }
    }
    // metadata staging: one task or pack descriptor per job and grouped op
    size_t meta = 0;
    for (const auto& g : groups) {
        for (const Op& o : plans[g[0]].ops) {
            if (o.kind == OP_SYRK || o.kind == OP_GEMM) meta += rup(g.size() * sizeof(ProdTask), 256);
            else if (o.kind == OP_PACK) meta += rup(g.size() * sizeof(PackDesc), 256);
        }
    }
    std::vector<char*> jws(njobs, nullptr);
    int st = FFP_OK;
    if (job_ws) {
        for (int j = 0; j < njobs; ++j) jws[j] = job_ws[j];
    } else {
        Workspace* w = nullptr;
        st = acquire_workspace(s, (size_t)ws_total, 0, &w);
        if (st != FFP_OK) return st;
        for (int j = 0; j < njobs; ++j) jws[j] = (char*)w->ptr + wsoff[j];
    }
    char* host_meta = nullptr;
    char* dev_meta = nullptr;
    st = acquire_staging(s, meta, &host_meta, &dev_meta);
    if (st != FFP_OK) return st;
    size_t moff = 0;

    for (const auto& g : groups) {
        const size_t nops = plans[g[0]].ops.size();
        for (size_t i = 0; i < nops; ++i) {
            const Op& o0 = plans[g[0]].ops[i];
            if (o0.kind == OP_SYRK || o0.kind == OP_GEMM) {
                ProdTask* tasks = (ProdTask*)(host_meta + moff);
                ProdTask* dtasks = (ProdTask*)(dev_meta + moff);
                moff += rup(g.size() * sizeof(ProdTask), 256);
                int nt = 0;
                for (int j : g)
                    tasks[nt++] = make_task(plans[j], plans[j].ops[i], jobs[j].A, jobs[j].C, jws[j]);
                std::stable_sort(tasks, tasks + nt, longer);
                if (launch_products(o0.cls, tasks, nt, dtasks, s) != hipSuccess) return FFP_EDEVICE;
            } else if (o0.kind == OP_PACK) {
                PackDesc* d = (PackDesc*)(host_meta + moff);
                PackDesc* dd = (PackDesc*)(dev_meta + moff);
                moff += rup(g.size() * sizeof(PackDesc), 256);
                int nd = 0;
                for (int j : g)
                    d[nd++] = make_pack(plans[j], plans[j].ops[i], jobs[j].A, jobs[j].C, jws[j]);
                if (launch_pack_grouped(o0.src_cls, o0.cls, d, nd, dd, s) != hipSuccess) return FFP_EDEVICE;
            } else {
                for (int j : g) {
                    st = execute_op(plans[j], plans[j].ops[i], jobs[j].A, jobs[j].C, jws[j], s);
                    if (st != FFP_OK) return st;
                }
            }
        }
    }
    return release_staging(s);
}

}  // namespace ffp
