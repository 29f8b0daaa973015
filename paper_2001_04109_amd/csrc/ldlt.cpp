// Host driver of fldlt_modp: recursive LDL^T without pivoting whose
// Schur-complement updates S22 <- S22 - L21 D1 L21^T run as Algorithm 5
// (D1 = Delta Delta^T, Abar = L21 Delta) followed by the accumulate form of
// Algorithm 2 (Table 4 schedule) with alpha = p - 1, beta = 1.
#include "ldlt.h"

#include <algorithm>
#include <cstring>
#include <deque>

#include "ffp.h"
#include "field.h"
#include "plan.h"
#include "runtime.h"

namespace ffp {

int g_ldlt_fold = 1;

namespace {

int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

int64_t split_point(int64_t n) { return rup((n + 1) / 2, kLdltLeaf); }

struct NodeLayout {
    int64_t abar_ld, kpad;
    int64_t off_abar, off_flag, off_root, off_dinv, off_rank, off_desc, off_syrk;
    int64_t bytes_before_syrk;
};

NodeLayout layout(int64_t n1, int64_t n2)
{
    NodeLayout L;
    L.kpad = rup(n1 + 1, 128);
    L.abar_ld = L.kpad;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = rup(off, 256); off = o + bytes; return o; };
    L.off_abar = take(n2 * L.abar_ld * 4);
    L.off_flag = take(n1 * 4);
    L.off_root = take(n1 * 4);
    L.off_dinv = take(n1 * 4);
    L.off_rank = take(n1 * 4);
    L.off_desc = take((n1 + 1) * (int64_t)sizeof(ColOp));
    L.off_syrk = rup(off, 256);
    L.bytes_before_syrk = L.off_syrk;
    return L;
}

PlanRequest schur_request(int64_t n2, const NodeLayout& L, uint32_t p, int64_t lds, bool c_aligned)
{
    PlanRequest rq;
    rq.n = n2;
    rq.k = L.kpad;
    rq.p = p;
    rq.a_cls = CLS_F64;
    rq.lda = L.abar_ld;
    rq.ldc = lds;
    rq.alpha = p - 1;
    rq.beta = 1;
    rq.depth = -1;
    rq.no_tune = true;      // the workspace figure must not depend on the tuning table
    // above the one- and two-limb int8 range, three int8 limbs where they
    // hold the residues (several times the FP64 matrix-core rate, no
    // recursion needed)
    rq.force_limb3 = p > 65521u && p < (1u << 23);
    rq.a_aligned16 = true;
    rq.c_aligned16 = c_aligned;
    return rq;
}

// One step of a factorisation, at its level in the job's sequence.
enum StepKind { SK_DEV = 0, SK_PROD = 1, SK_OP = 2 };
struct Step {
    int level;
    int sk;
    int kind;          // SK_DEV: LK_*
    int cls;           // SK_PROD: base class of the product
    LdltDesc d;        // SK_DEV
    ProdTask t;        // SK_PROD
    const Plan* pl;    // SK_OP
    const Op* op;
    const void* a;
    void* c;
    void* ws;
};

// Flattens the recursion of one factorisation into steps.  Consecutive
// steps depend on each other, except the block operations of one Schur
// update, which take the levels of the level scheduler.
struct Builder {
    FieldPlan fpl;
    Fp f;
    int kb;
    uint32_t s_lqnr, c_lqnr;
    uint32_t* linv;     // inverses of the leaf blocks of L: column block c at linv + 64 c
    char* ws;
    int64_t* info;
    int64_t lds;
    std::deque<Plan>* plans;
    std::vector<Step>* out;
    int level = 0;
    int status = FFP_OK;

    LdltDesc base() const
    {
        LdltDesc d{};
        d.f = f;
        d.kb = kb;
        d.s_lqnr = s_lqnr;
        d.c_lqnr = c_lqnr;
        d.info = info;
        return d;
    }
    void dev(int kind, const LdltDesc& d)
    {
        Step s{};
        s.level = level++;
        s.sk = SK_DEV;
        s.kind = kind;
        s.d = d;
        out->push_back(s);
    }
    void prod(const ProdTask& t)
    {
        if (g_ldlt_fold) {
            // a step of the per-level launch, tile by tile
            LdltDesc d = base();
            d.t = t;
            if (prepare_f64_tile_task(&d.t)) {
                dev(LK_PRODF, d);
                return;
            }
        }
        Step s{};
        s.level = level++;
        s.sk = SK_PROD;
        s.cls = CLS_F64;
        s.t = t;
        out->push_back(s);
    }
    void plan_ops(const Plan& pl, const void* a, void* c, void* w)
    {
        // a three-limb update (pack, product) as two steps of the per-level
        // launches
        if (g_ldlt_fold && pl.cls == CLS_LIMB3 && pl.ops.size() == 2 && pl.ops[0].kind == OP_PACK &&
            pl.ops[1].kind == OP_SYRK) {
            ProdTask t = make_task(pl, pl.ops[1], a, c, w);
            if (prepare_limb3_tile_task(&t)) {
                const PackDesc pk = make_pack(pl, pl.ops[0], a, c, w);
                LdltDesc d = base();
                d.X = (uint32_t*)pk.src.p;
                d.ldx = pk.src.ld;
                d.rows = pk.n;
                d.ncols = (int32_t)pk.k;
                d.rows_pad = pk.n_pad;
                d.kpad = (int32_t)pk.k_pad;
                d.Ab = (uint32_t*)pk.dst.p;
                d.ldab = pk.dst.ld;
                d.pplane = pk.dst.plane;
                dev(LK_PACK3, d);
                LdltDesc e = base();
                e.t = t;
                dev(LK_PRODL3, e);
                return;
            }
        }
        std::vector<SchedItem> items;
        items.reserve(pl.ops.size());
        for (const Op& o : pl.ops) items.push_back(SchedItem{&pl, &o, a, c, w, 0});
        const std::vector<int> lv = schedule_levels(items);
        int mx = -1;
        for (size_t i = 0; i < items.size(); ++i) {
            const Op& o = pl.ops[i];
            Step s{};
            s.level = level + lv[i];
            if (o.kind == OP_SYRK || o.kind == OP_GEMM) {
                s.sk = SK_PROD;
                s.cls = o.cls;
                s.t = make_task(pl, o, a, c, w);
            } else {
                s.sk = SK_OP;
                s.pl = &pl;
                s.op = &o;
                s.a = a;
                s.c = c;
                s.ws = w;
            }
            out->push_back(s);
            mx = std::max(mx, lv[i]);
        }
        level += mx + 1;
    }

    // X <- X L^-T for the unit lower triangular m x m factor L whose first
    // column is column col0 of the whole factorisation.  The blocks split as
    // the factorisation does, so every leaf is a leaf block of rec() whose
    // inverse is in linv.
    void trsm(int64_t nrows, int64_t m, uint32_t* X, int64_t ldx, const uint32_t* L, int64_t ldl, int64_t col0)
    {
        if (nrows <= 0 || m <= 0) return;
        if (m <= kLdltLeaf) {
            LdltDesc d = base();
            d.rows = nrows;
            d.nb = (int32_t)m;
            d.X = X;
            d.ldx = ldx;
            d.linv = linv + col0 * kLdltLeaf;
            dev(LK_TRSM, d);
            return;
        }
        const int64_t m1 = rup((m + 1) / 2, kLdltLeaf);
        trsm(nrows, m1, X, ldx, L, ldl, col0);
        // X[:, m1:] <- X[:, m1:] - X[:, :m1] L[m1:, :m1]^T
        ProdTask t{};
        init_task(&t, fpl);
        t.A = DView{X, ldx, 0};
        t.B = DView{(void*)(L + m1 * ldl), ldl, 0};
        t.C = X + m1;
        t.ldc = ldx;
        t.m = (int32_t)nrows;
        t.n = (int32_t)(m - m1);
        t.k = (int32_t)m1;
        t.syrk = 0;
        t.alpha = f.p - 1;
        t.beta = 1;
        prod(t);
        trsm(nrows, m - m1, X + m1, ldx, L + m1 * ldl + m1, ldl, col0 + m1);
    }

    void rec(int64_t n, uint32_t* S, int64_t offset)
    {
        if (n <= 0 || status != FFP_OK) return;
        if (n <= kLdltLeaf) {
            LdltDesc d = base();
            d.nb = (int32_t)n;
            d.X = S;
            d.ldx = lds;
            d.offset = offset;
            d.linv = linv + offset * kLdltLeaf;
            dev(LK_LEAF, d);
            return;
        }
        const int64_t n1 = split_point(n), n2 = n - n1;
        uint32_t* S11 = S;
        uint32_t* S21 = S + n1 * lds;
        uint32_t* S22 = S + n1 * lds + n1;
        rec(n1, S11, offset);
        // W = S21 L11^-T, then L21 = W D1^-1
        trsm(n2, n1, S21, lds, S11, lds, offset);
        const NodeLayout L = layout(n1, n2);
        LdltDesc d = base();
        d.sc = Alg5Scratch{(int32_t*)(ws + L.off_flag), (uint32_t*)(ws + L.off_root),
                           (uint32_t*)(ws + L.off_dinv), (int32_t*)(ws + L.off_rank),
                           (ColOp*)(ws + L.off_desc)};
        d.nb = (int32_t)n1;
        d.X = S11;
        d.ldx = lds;
        dev(LK_CLASSIFY, d);
        dev(LK_PAIR, d);
        LdltDesc sd = d;
        sd.rows = n2;
        sd.X = S21;
        dev(LK_SCALE, sd);
        uint32_t* Ab = (uint32_t*)(ws + L.off_abar);
        LdltDesc ad = d;
        ad.rows = n2;
        ad.ncols = (int32_t)(n1 + 1);
        ad.kpad = (int32_t)L.kpad;
        ad.X = S21;
        ad.Ab = Ab;
        ad.ldab = L.abar_ld;
        dev(LK_ABAR, ad);
        // S22 <- S22 - Abar Abar^T  (alpha = p - 1, beta = 1: Table 4 schedule)
        plans->emplace_back();
        Plan& pl = plans->back();
        const int st = build_syrk_plan(schur_request(n2, L, f.p, lds, (((uintptr_t)S22) & 15) == 0), &pl);
        if (st != FFP_OK) {
            status = st;
            return;
        }
        plan_ops(pl, Ab, S22, ws + L.off_syrk);
        rec(n2, S22, offset + n1);
    }
};

int64_t rup256(int64_t x) { return (x + 255) / 256 * 256; }

// Runs the steps of independent jobs level by level: all device steps of a
// level (whatever their kinds) as one launch over their descriptors,
// products of one class as one grouped launch (on a paired stream when the
// level also has device steps, joined before the level ends), block
// operations one by one.
int execute_steps(const std::vector<Step>& steps, hipStream_t s)
{
    if (steps.empty()) return FFP_OK;
    int maxlev = 0;
    for (const Step& st : steps) maxlev = std::max(maxlev, st.level);
    std::vector<std::vector<int>> by(maxlev + 1);
    for (size_t i = 0; i < steps.size(); ++i) by[steps[i].level].push_back((int)i);

    // descriptor table: one slice per level (kinds in a fixed order, the
    // longest-running first); product tables for groups beyond the inline
    // capacity
    struct Slice { int first, count, blocks; };
    static const int kOrder[LK_KINDS] = {LK_LEAF, LK_PRODL3, LK_PRODF, LK_PAIR,  LK_BDIAG, LK_CLASSIFY,
                                         LK_TRSM, LK_PACK3,  LK_ABAR2, LK_ABAR, LK_SCALE, LK_ZERO};
    std::vector<Slice> slices(maxlev + 1, Slice{0, 0, 0});
    std::vector<LdltDesc> table;
    size_t prod_bytes = 0;
    for (int lv = 0; lv <= maxlev; ++lv) {
        Slice sl{(int)table.size(), 0, 0};
        for (int kind : kOrder) {
            for (int i : by[lv]) {
                const Step& st = steps[i];
                if (st.sk != SK_DEV || st.kind != kind) continue;
                LdltDesc d = st.d;
                d.kind = kind;
                const int nbk = ldlt_blocks(kind, &d);
                if (nbk <= 0) continue;
                d.block0 = sl.blocks;
                sl.blocks += nbk;
                table.push_back(d);
                ++sl.count;
            }
        }
        slices[lv] = sl;
        int np[kNumCls] = {0};
        for (int i : by[lv])
            if (steps[i].sk == SK_PROD) ++np[steps[i].cls];
        for (int q : np)
            if (q > kInlineTasks) prod_bytes += (size_t)rup256((int64_t)q * (int64_t)sizeof(ProdTask));
    }
    const size_t desc_bytes = (size_t)rup256((int64_t)(table.size() * sizeof(LdltDesc)));
    char* host = nullptr;
    char* dev = nullptr;
    if (desc_bytes + prod_bytes > 0) {
        const int st = acquire_staging(s, desc_bytes + prod_bytes, &host, &dev);
        if (st != FFP_OK) return st;
    }
    // levels with both device steps and products (of other jobs) run the
    // products on a paired stream, so that the two overlap
    bool overlap = false;
    for (int lv = 0; lv <= maxlev && !overlap; ++lv) {
        if (!slices[lv].count) continue;
        for (int i : by[lv])
            if (steps[i].sk == SK_PROD) { overlap = true; break; }
    }
    SideStream* ss = nullptr;
    if (overlap) {
        const int st = side_stream(s, &ss);
        if (st != FFP_OK) return st;
    }
    if (const int st = capture_point(s); st != FFP_OK) return st;
    if (!table.empty()) {
        memcpy(host, table.data(), table.size() * sizeof(LdltDesc));
        if (hipMemcpyAsync(dev, host, table.size() * sizeof(LdltDesc), hipMemcpyHostToDevice, s) != hipSuccess)
            return FFP_EDEVICE;
    }
    const LdltDesc* dtable = (const LdltDesc*)dev;
    size_t poff = desc_bytes;
    int status = FFP_OK;
    for (int lv = 0; lv <= maxlev && status == FFP_OK; ++lv) {
        const Slice& sl = slices[lv];
        bool has_prod = false;
        for (int i : by[lv]) has_prod = has_prod || steps[i].sk == SK_PROD;
        hipStream_t ps = s;
        if (ss && sl.count && has_prod) {
            if (hipEventRecord(ss->fork, s) != hipSuccess || hipStreamWaitEvent(ss->side, ss->fork, 0) != hipSuccess)
                status = FFP_EDEVICE;
            ps = ss->side;
        }
        if (status == FFP_OK && sl.count && launch_ldlt_steps(dtable + sl.first, sl.count, sl.blocks, s) != hipSuccess)
            status = FFP_EDEVICE;
        for (int cls = 0; cls < kNumCls && status == FFP_OK; ++cls) {
            std::vector<ProdTask> g;
            for (int i : by[lv])
                if (steps[i].sk == SK_PROD && steps[i].cls == cls) g.push_back(steps[i].t);
            if (g.empty()) continue;
            std::stable_sort(g.begin(), g.end(), [](const ProdTask& a, const ProdTask& b) {
                if (a.k != b.k) return a.k > b.k;
                return (int64_t)a.m * a.n > (int64_t)b.m * b.n;
            });
            ProdTask* tasks = g.data();
            ProdTask* dtasks = nullptr;
            if (g.size() > (size_t)kInlineTasks) {
                tasks = (ProdTask*)(host + poff);
                dtasks = (ProdTask*)(dev + poff);
                poff += (size_t)rup256((int64_t)(g.size() * sizeof(ProdTask)));
                memcpy(tasks, g.data(), g.size() * sizeof(ProdTask));
            }
            if (launch_products(cls, tasks, (int)g.size(), dtasks, ps) != hipSuccess) status = FFP_EDEVICE;
        }
        if (ps != s) {
            // join even after a failure, so that no work is left unordered
            if (hipEventRecord(ss->join, ps) != hipSuccess || hipStreamWaitEvent(s, ss->join, 0) != hipSuccess)
                status = FFP_EDEVICE;
        }
        for (int i : by[lv]) {
            if (status != FFP_OK) break;
            const Step& st = steps[i];
            if (st.sk == SK_OP) status = execute_op(*st.pl, *st.op, st.a, st.c, st.ws, s);
        }
    }
    if (desc_bytes + prod_bytes > 0) {
        const int st = release_staging(s);
        if (status == FFP_OK) status = st;
    }
    return status;
}

size_t ws_need(int64_t n, uint32_t p, int64_t lds)
{
    if (n <= kLdltLeaf) return 0;
    const int64_t n1 = split_point(n), n2 = n - n1;
    const NodeLayout L = layout(n1, n2);
    Plan pl;
    size_t syrk_ws = 0;
    if (build_syrk_plan(schur_request(n2, L, p, lds, false), &pl) == FFP_OK) syrk_ws = (size_t)pl.ws_bytes;
    size_t here = (size_t)L.off_syrk + syrk_ws;
    return std::max(here, std::max(ws_need(n1, p, lds), ws_need(n2, p, lds)));
}

size_t linv_bytes(int64_t n) { return (size_t)rup(n * kLdltLeaf * 4, 256); }

}  // namespace

size_t ldlt_workspace_bytes(int64_t n, uint32_t p, int64_t lds) { return linv_bytes(n) + ws_need(n, p, lds); }

int ldlt_run_multi(const std::vector<LdltJobSpec>& jobs, hipStream_t s)
{
    std::deque<Plan> plans;
    std::vector<Step> steps;
    for (const LdltJobSpec& j : jobs) {
        Builder b;
        if (!make_field_plan(j.p, &b.fpl)) return FFP_EPRIME;
        b.f = Fp{j.p, (j.p - 1) / 2, b.fpl.pinv, b.fpl.ya, b.fpl.yb};
        b.kb = ldlt_dot_block(j.p);
        uint32_t sq = 2;
        while (legendre(sq, j.p) == 1) ++sq;
        b.s_lqnr = sq;
        b.c_lqnr = (uint32_t)sqrt_mod(sq - 1, j.p);
        b.info = j.info;
        b.lds = j.lds;
        b.linv = (uint32_t*)j.ws;
        b.ws = (char*)j.ws + linv_bytes(j.n);
        b.plans = &plans;
        b.out = &steps;
        b.dev(LK_ZERO, b.base());
        b.rec(j.n, j.S, 0);
        if (b.status != FFP_OK) return b.status;
    }
    return execute_steps(steps, s);
}

namespace {

// Workspace of fsyrkbd_modp: Dbar and the Algorithm 5 scratch (n pivots),
// the Algorithm 6 column ops (n) and Algorithm 5's (n + 1), Abar, then the
// product's own workspace.
struct BdLayout {
    int64_t kpad;
    int64_t off_dbar, off_flag, off_root, off_dinv, off_rank, off_desc1, off_desc, off_abar, off_syrk;
};

BdLayout bd_layout(int64_t m, int64_t n)
{
    BdLayout L;
    L.kpad = syrkbd_kpad(n);
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = rup(off, 256); off = o + bytes; return o; };
    L.off_dbar = take(n * 4);
    L.off_flag = take(n * 4);
    L.off_root = take(n * 4);
    L.off_dinv = take(n * 4);
    L.off_rank = take(n * 4);
    L.off_desc1 = take(n * (int64_t)sizeof(ColOp));
    L.off_desc = take((n + 1) * (int64_t)sizeof(ColOp));
    L.off_abar = take(m * L.kpad * 4);
    L.off_syrk = rup(off, 256);
    return L;
}

}  // namespace

int64_t syrkbd_kpad(int64_t n) { return rup(n + 1, 128); }

size_t syrkbd_workspace_bytes(int64_t m, int64_t n, const PlanRequest& rq)
{
    const BdLayout L = bd_layout(m, n);
    Plan pl;
    if (build_syrk_plan(rq, &pl) != FFP_OK) return 0;
    return (size_t)(L.off_syrk + pl.ws_bytes);
}

int syrkbd_run(int64_t m, int64_t n, uint32_t p, const uint32_t* A, int64_t lda, const uint32_t* bd,
               const uint32_t* bo, const PlanRequest& rq, uint32_t* C, int64_t* info, void* ws, hipStream_t s)
{
    const BdLayout L = bd_layout(m, n);
    std::deque<Plan> plans;
    std::vector<Step> steps;
    Builder b;
    if (!make_field_plan(p, &b.fpl)) return FFP_EPRIME;
    b.f = Fp{p, (p - 1) / 2, b.fpl.pinv, b.fpl.ya, b.fpl.yb};
    b.kb = ldlt_dot_block(p);
    uint32_t sq = 2;
    while (legendre(sq, p) == 1) ++sq;
    b.s_lqnr = sq;
    b.c_lqnr = (uint32_t)sqrt_mod(sq - 1, p);
    b.info = info;
    b.lds = rq.ldc;
    b.linv = nullptr;
    b.ws = (char*)ws;
    b.plans = &plans;
    b.out = &steps;
    char* w = (char*)ws;
    ColOp* desc1 = (ColOp*)(w + L.off_desc1);
    uint32_t* dbar = (uint32_t*)(w + L.off_dbar);
    uint32_t* Ab = (uint32_t*)(w + L.off_abar);
    if (n > 0) {
        // Algorithm 6: Abar = A M, Dbar (column ops only; Abar is formed once below)
        LdltDesc d = b.base();
        d.nb = (int32_t)n;
        d.bd = bd;
        d.bo = bo;
        d.desc1 = desc1;
        d.dbar = dbar;
        b.dev(LK_BDIAG, d);
        // Algorithm 5 on Dbar: square roots of the residues, non-residues in
        // pairs through Algorithm 4 (the pivots are read with stride 1)
        LdltDesc c = b.base();
        c.sc = Alg5Scratch{(int32_t*)(w + L.off_flag), (uint32_t*)(w + L.off_root), (uint32_t*)(w + L.off_dinv),
                           (int32_t*)(w + L.off_rank), (ColOp*)(w + L.off_desc)};
        c.nb = (int32_t)n;
        c.X = dbar;
        c.ldx = 0;
        b.dev(LK_CLASSIFY, c);
        b.dev(LK_PAIR, c);
        LdltDesc a = c;
        a.rows = m;
        a.ncols = (int32_t)(n + 1);
        a.kpad = (int32_t)L.kpad;
        a.X = (uint32_t*)A;
        a.ldx = lda;
        a.desc1 = desc1;
        a.Ab = Ab;
        a.ldab = L.kpad;
        b.dev(LK_ABAR2, a);
    } else if (info != nullptr) {
        b.dev(LK_ZERO, b.base());
    }
    // lower(C) <- alpha Abar Abar^T + beta lower(C) through Algorithm 2
    plans.emplace_back();
    Plan& pl = plans.back();
    PlanRequest r = rq;
    r.k = n > 0 ? L.kpad : 0;
    r.lda = L.kpad;
    const int st = build_syrk_plan(r, &pl);
    if (st != FFP_OK) return st;
    b.plan_ops(pl, Ab, C, w + L.off_syrk);
    return execute_steps(steps, s);
}

int ldlt_run(int64_t n, uint32_t p, uint32_t* S, int64_t lds, int64_t* info, hipStream_t s, void* ws)
{
    if (!ws) {
        const size_t need = ldlt_workspace_bytes(n, p, lds);
        Workspace* w = nullptr;
        int st = acquire_workspace(s, need, 0, &w);
        if (st != FFP_OK) return st;
        ws = w->ptr;
    }
    return ldlt_run_multi({LdltJobSpec{n, p, S, lds, info, ws}}, s);
}

}  // namespace ffp
