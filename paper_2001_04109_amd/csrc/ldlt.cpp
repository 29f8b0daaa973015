// Host driver of fldlt_modp: recursive LDL^T without pivoting whose
// Schur-complement updates S22 <- S22 - L21 D1 L21^T run as Algorithm 5
// (D1 = Delta Delta^T, Abar = L21 Delta) followed by the accumulate form of
// Algorithm 2 (Table 4 schedule) with alpha = p - 1, beta = 1.
//
// The triangular solve W = S21 L11^-T is one product with the inverse of
// L11, which the recursion assembles from the inverses of its parts:
// [[La, 0], [Lb, Lc]]^-1 = [[La^-1, 0], [-Lc^-1 Lb La^-1, Lc^-1]], the leaves
// inverting their 64 x 64 unit factors; the product Lb La^-1 runs beside
// the Schur update, the one with Lc^-1 once Lc is factored.  A node needs
// its inverse unless it lies on the path from the root through right
// children, so a solve never waits for a chain of smaller solves.
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
    int64_t off_abar, off_syrk;
};

NodeLayout layout(int64_t n1, int64_t n2)
{
    NodeLayout L;
    L.kpad = rup(n1 + 1, 128);
    L.abar_ld = L.kpad;
    L.off_abar = 0;
    L.off_syrk = rup(n2 * L.abar_ld * 4, 256);
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
    rq.no_tune = true;      // the workspace figure must not depend on the tuning table
    // above the one- and two-limb int8 range, three int8 limbs where they
    // hold the residues (several times the FP64 matrix-core rate)
    rq.force_limb3 = p > 65521u && p < (1u << 23);
    // Algorithm 5 ends with the product of A-bar by its transpose through
    // Algorithm 2: updates of order 4096 and more keep one level of it on
    // three limbs (k about n, where the base product alone is some 0.07 ms
    // faster at order 4096); otherwise the class's default depth.
    rq.depth = (rq.force_limb3 && n2 >= 4096) ? 1 : -1;
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

// Flattens the recursion of one factorisation into steps.  Steps go one
// level after the step they wait for; the product Lb La^-1 of a node shares
// the level of its Schur update, and the block operations of a Schur update
// take the levels of the level scheduler.
struct Builder {
    FieldPlan fpl{};
    Fp f{};
    int kb = 0;
    uint32_t s_lqnr = 0, c_lqnr = 0, s_inv = 0;
    Alg5Scratch piv{};  // per pivot of the whole factorisation (LDL^T)
    uint32_t* invbuf = nullptr;   // inverse of the left child of a node on the right spine
    int64_t ldi = 0;
    std::vector<uint32_t*> t1;   // per depth: Lb La^-1 of the node being built
    std::vector<int64_t> t1ld;
    uint32_t* wbuf = nullptr;   // W = S21 L11^-T of the current node (dense, ld n1)
    char* ws = nullptr;         // node region: Abar, then the Schur update's workspace
    int64_t* info = nullptr;
    int64_t lds = 0;
    int64_t ntotal = 0;         // order of the whole factorisation
    std::deque<Plan>* plans = nullptr;
    std::vector<Step>* out = nullptr;
    int level = 0;
    int status = FFP_OK;

    LdltDesc base() const
    {
        LdltDesc d{};
        d.f = f;
        d.kb = kb;
        d.s_lqnr = s_lqnr;
        d.c_lqnr = c_lqnr;
        d.s_inv = s_inv;
        d.info = info;
        return d;
    }
    void dev_at(int kind, const LdltDesc& d, int lv)
    {
        Step s{};
        s.level = lv;
        s.sk = SK_DEV;
        s.kind = kind;
        s.d = d;
        out->push_back(s);
    }
    void dev(int kind, const LdltDesc& d) { dev_at(kind, d, level++); }
    // C (m x n, ldc) <- alpha A op(B) as 64 x 64 FP64 tiles of the level's launch
    void tile_prod(int form, int lv, const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb, uint32_t* C,
                   int64_t ldc, int64_t m, int64_t n, int64_t k, uint32_t alpha)
    {
        LdltDesc d = base();
        init_task(&d.t, fpl);
        d.t.A = DView{(void*)A, lda, 0};
        d.t.B = DView{(void*)B, ldb, 0};
        d.t.C = C;
        d.t.ldc = ldc;
        d.t.m = (int32_t)m;
        d.t.n = (int32_t)n;
        d.t.k = (int32_t)k;
        d.t.syrk = 0;
        d.t.alpha = alpha;
        d.t.beta = 0;
        prepare_f64_tile_task(&d.t);
        d.pform = form;
        dev_at(LK_PRODF, d, lv);
    }
    void plan_ops(const Plan& pl, const void* a, void* c, void* w)
    {
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

    // Factors the n x n block at S whose first pivot is pivot `offset` of the
    // whole factorisation; when inv is not null, also writes the inverse of
    // its unit lower factor there (ld ldi).
    void rec(int64_t n, uint32_t* S, int64_t offset, uint32_t* inv, int depth)
    {
        if (n <= 0 || status != FFP_OK) return;
        if (n <= kLdltLeaf) {
            LdltDesc d = base();
            d.nb = (int32_t)n;
            d.X = S;
            d.ldx = lds;
            d.offset = offset;
            d.sc = piv;
            d.linv = inv;
            d.ldi = ldi;
            dev(LK_LEAF, d);
            // its pivots' classes beside the next step (none after the last leaf)
            if (offset + n < ntotal) dev_at(LK_ROOTS, d, level);
            return;
        }
        const int64_t n1 = split_point(n), n2 = n - n1;
        uint32_t* S11 = S;
        uint32_t* S21 = S + n1 * lds;
        uint32_t* S22 = S + n1 * lds + n1;
        uint32_t* inv1 = inv ? inv : invbuf;
        uint32_t* inv2 = inv ? inv + n1 * (ldi + 1) : nullptr;
        rec(n1, S11, offset, inv1, depth + 1);
        // W = S21 L11^-T (L11^-1 lower triangular)
        tile_prod(TILE_NT_BLOW, level++, S21, lds, inv1, ldi, wbuf, n1, n2, n1, n1, 1u);
        // S22 <- S22 - Abar Abar^T (alpha = p - 1, beta = 1: Table 4 schedule)
        const NodeLayout L = layout(n1, n2);
        plans->emplace_back();
        Plan& pl = plans->back();
        const int st = build_syrk_plan(schur_request(n2, L, f.p, lds, (((uintptr_t)S22) & 15) == 0), &pl);
        if (st != FFP_OK) {
            status = st;
            return;
        }
        uint32_t* Ab = (uint32_t*)(ws + L.off_abar);
        void* w = ws + L.off_syrk;
        // Algorithm 5: L21 = W D1^-1 and Abar = L21 Delta; a three-limb
        // update takes Abar straight in limb planes
        LdltDesc ad = base();
        ad.nb = (int32_t)n1;
        ad.offset = offset;
        ad.sc = piv;
        ad.rows = n2;
        ad.ncols = (int32_t)(n1 + 1);
        ad.kpad = (int32_t)L.kpad;
        ad.X = wbuf;
        ad.ldx = n1;
        ad.Y = S21;
        ad.ldy = lds;
        ad.Ab = Ab;
        ad.ldab = L.abar_ld;
        bool folded = false;
        ProdTask lt{};
        if (g_ldlt_fold && pl.cls == CLS_LIMB3 && pl.ops.size() == 2 && pl.ops[0].kind == OP_PACK &&
            pl.ops[1].kind == OP_SYRK) {
            lt = make_task(pl, pl.ops[1], Ab, S22, w);
            const PackDesc pk = make_pack(pl, pl.ops[0], Ab, S22, w);
            if (prepare_limb3_tile_task(&lt) && pk.k_pad == L.kpad && pk.n == n2) {
                folded = true;
                ad.amode = 1;
                ad.Ab = (uint32_t*)pk.dst.p;
                ad.ldab = pk.dst.ld;
                ad.pplane = pk.dst.plane;
                ad.rows_pad = pk.n_pad;
            }
        }
        dev(LK_ABARX, ad);
        // Lb La^-1 (La^-1 lower triangular), beside the Schur update
        if (inv) tile_prod(TILE_NN_BLOW, level, S21, lds, inv1, ldi, t1[depth], t1ld[depth], n2, n1, n1, 1u);
        if (folded) {
            LdltDesc e = base();
            e.t = lt;
            dev(LK_PRODL3, e);
        } else {
            plan_ops(pl, Ab, S22, w);
        }
        rec(n2, S22, offset + n1, inv2, depth + 1);
        // -Lc^-1 (Lb La^-1) below the diagonal blocks of the inverse
        if (inv)
            tile_prod(TILE_NN_ALOW, level++, inv2, ldi, t1[depth], t1ld[depth], inv + n1 * ldi, ldi, n2, n1, n2,
                      f.p - 1);
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
    static const int kOrder[LK_KINDS] = {LK_LEAF,     LK_PRODL3, LK_PRODF, LK_PAIR,  LK_ROOTS,
                                         LK_BDIAG, LK_CLASSIFY, LK_ABARX, LK_ABAR2, LK_ZERO};
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
            hipEvent_t e0 = nullptr;
            const bool prof = prof_enabled();
            double flops = 0.0;
            if (prof) {
                for (const ProdTask& t : g)
                    flops += t.syrk ? (double)t.m * (double)(t.m + 1) * (double)t.k
                                    : 2.0 * (double)t.m * (double)t.n * (double)t.k;
                prof_begin(ps, &e0);
            }
            if (launch_products(cls, tasks, (int)g.size(), dtasks, ps) != hipSuccess) status = FFP_EDEVICE;
            if (prof) prof_end(ps, e0, flops, cls);
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

// Workspace of one factorisation: the pivot data of Algorithm 5, the
// inverse of the leading unit factor of a node on the right spine, one
// Lb La^-1 block per recursion depth, W, then the node region (Abar and the
// Schur update's workspace, reused node after node).
struct JobLayout {
    int64_t off_flag = 0, off_root = 0, off_dinv = 0, off_inv = 0, ldi = 0, off_w = 0, off_node = 0;
    std::vector<int64_t> off_t1, ld_t1;
    size_t bytes = 0;
};

void walk(int64_t n, int depth, bool spine, uint32_t p, int64_t lds, std::vector<int64_t>* m1,
          std::vector<int64_t>* m2, int64_t* wmax, size_t* node_max)
{
    if (n <= kLdltLeaf) return;
    const int64_t n1 = split_point(n), n2 = n - n1;
    if ((int)m1->size() <= depth) {
        m1->resize(depth + 1, 0);
        m2->resize(depth + 1, 0);
    }
    if (!spine) {
        (*m1)[depth] = std::max((*m1)[depth], n1);
        (*m2)[depth] = std::max((*m2)[depth], n2);
    }
    *wmax = std::max(*wmax, n1 * n2);
    const NodeLayout L = layout(n1, n2);
    Plan pl;
    size_t syrk_ws = 0;
    if (build_syrk_plan(schur_request(n2, L, p, lds, false), &pl) == FFP_OK) syrk_ws = (size_t)pl.ws_bytes;
    *node_max = std::max(*node_max, (size_t)L.off_syrk + syrk_ws);
    walk(n1, depth + 1, false, p, lds, m1, m2, wmax, node_max);
    walk(n2, depth + 1, spine, p, lds, m1, m2, wmax, node_max);
}

JobLayout job_layout(int64_t n, uint32_t p, int64_t lds)
{
    JobLayout J;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = rup(off, 256); off = o + bytes; return o; };
    J.off_flag = take(n * 4);
    J.off_root = take(n * 4);
    J.off_dinv = take(n * 4);
    if (n > kLdltLeaf) {
        const int64_t n1 = split_point(n);
        J.ldi = n1;
        J.off_inv = take(n1 * n1 * 4);
        std::vector<int64_t> m1, m2;
        int64_t wmax = 0;
        size_t node_max = 0;
        walk(n, 0, true, p, lds, &m1, &m2, &wmax, &node_max);
        for (size_t d = 0; d < m1.size(); ++d) {
            J.off_t1.push_back(take(m1[d] * m2[d] * 4));
            J.ld_t1.push_back(m1[d]);
        }
        J.off_w = take(wmax * 4);
        J.off_node = take((int64_t)node_max);
    }
    J.bytes = (size_t)rup(off, 256);
    return J;
}

}  // namespace

size_t ldlt_workspace_bytes(int64_t n, uint32_t p, int64_t lds) { return job_layout(n, p, lds).bytes; }

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
        b.s_inv = (uint32_t)inv_mod(sq, j.p);
        const JobLayout J = job_layout(j.n, j.p, j.lds);
        char* w = (char*)j.ws;
        b.piv = Alg5Scratch{(int32_t*)(w + J.off_flag), (uint32_t*)(w + J.off_root), (uint32_t*)(w + J.off_dinv),
                            nullptr, nullptr};
        b.invbuf = (uint32_t*)(w + J.off_inv);
        b.ldi = J.ldi;
        for (size_t d = 0; d < J.off_t1.size(); ++d) {
            b.t1.push_back((uint32_t*)(w + J.off_t1[d]));
            b.t1ld.push_back(J.ld_t1[d]);
        }
        b.wbuf = (uint32_t*)(w + J.off_w);
        b.ws = w + J.off_node;
        b.info = j.info;
        b.lds = j.lds;
        b.ntotal = j.n;
        b.plans = &plans;
        b.out = &steps;
        b.dev(LK_ZERO, b.base());
        b.rec(j.n, j.S, 0, nullptr, 0);
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
