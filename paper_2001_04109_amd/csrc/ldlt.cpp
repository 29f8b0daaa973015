// Host driver of fldlt_modp: recursive LDL^T without pivoting whose
// Schur-complement updates S22 <- S22 - L21 D1 L21^T run as Algorithm 5
// (D1 = Delta Delta^T, Abar = L21 Delta) followed by the accumulate form of
// Algorithm 2 (Table 4 schedule) with alpha = p - 1, beta = 1.
#include "ldlt.h"

#include <algorithm>

#include "ffp.h"
#include "field.h"
#include "plan.h"
#include "runtime.h"

namespace ffp {

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
    rq.a_aligned16 = true;
    rq.c_aligned16 = c_aligned;
    return rq;
}

struct Ctx {
    FieldPlan fpl;
    Fp f;
    uint32_t s_lqnr, c_lqnr;
    uint32_t* linv;     // inverses of the leaf blocks of L: column block c at linv + 64 c
    char* ws;
    int64_t* info;
    hipStream_t s;
};

// X <- X L^-T for the unit lower triangular m x m factor L whose first
// column is column col0 of the whole factorisation.  The blocks split as
// the factorisation did, so every leaf is a leaf block of ldlt_rec whose
// inverse is in c.linv.
int trsm_rec(Ctx& c, int64_t nrows, int64_t m, uint32_t* X, int64_t ldx, const uint32_t* L,
             int64_t ldl, int64_t col0)
{
    if (m <= kLdltLeaf)
        return launch_trsm_leaf(c.f, nrows, (int)m, X, ldx, c.linv + col0 * kLdltLeaf, c.s) == hipSuccess
                   ? FFP_OK
                   : FFP_EDEVICE;
    const int64_t m1 = rup((m + 1) / 2, kLdltLeaf);
    int st = trsm_rec(c, nrows, m1, X, ldx, L, ldl, col0);
    if (st != FFP_OK) return st;
    // X[:, m1:] <- X[:, m1:] - X[:, :m1] L[m1:, :m1]^T
    ProdTask t{};
    init_task(&t, c.fpl);
    t.A = DView{X, ldx, 0};
    t.B = DView{(void*)(L + m1 * ldl), ldl, 0};
    t.C = X + m1;
    t.ldc = ldx;
    t.m = (int32_t)nrows;
    t.n = (int32_t)(m - m1);
    t.k = (int32_t)m1;
    t.syrk = 0;
    t.alpha = c.f.p - 1;
    t.beta = 1;
    if (launch_products(CLS_F64, &t, 1, nullptr, c.s) != hipSuccess) return FFP_EDEVICE;
    return trsm_rec(c, nrows, m - m1, X + m1, ldx, L + m1 * ldl + m1, ldl, col0 + m1);
}

int ldlt_rec(Ctx& c, int64_t n, uint32_t* S, int64_t lds, int64_t offset)
{
    if (n <= 0) return FFP_OK;
    if (n <= kLdltLeaf)
        return launch_ldlt_leaf(c.f, (int)n, S, lds, c.info, offset, c.linv + offset * kLdltLeaf, c.s) ==
                       hipSuccess
                   ? FFP_OK
                   : FFP_EDEVICE;
    const int64_t n1 = split_point(n), n2 = n - n1;
    uint32_t* S11 = S;
    uint32_t* S21 = S + n1 * lds;
    uint32_t* S22 = S + n1 * lds + n1;
    int st = ldlt_rec(c, n1, S11, lds, offset);
    if (st != FFP_OK) return st;
    // W = S21 L11^-T, then L21 = W D1^-1
    st = trsm_rec(c, n2, n1, S21, lds, S11, lds, offset);
    if (st != FFP_OK) return st;
    const NodeLayout L = layout(n1, n2);
    Alg5Scratch sc{(int32_t*)(c.ws + L.off_flag), (uint32_t*)(c.ws + L.off_root),
                   (uint32_t*)(c.ws + L.off_dinv), (int32_t*)(c.ws + L.off_rank),
                   (ColOp*)(c.ws + L.off_desc)};
    if (launch_alg5(c.f, (int)n1, S11, lds, c.s_lqnr, c.c_lqnr, c.s_lqnr, sc, c.s) != hipSuccess)
        return FFP_EDEVICE;
    if (launch_scale_cols(c.f, n2, (int)n1, S21, lds, sc.dinv, c.s) != hipSuccess) return FFP_EDEVICE;
    uint32_t* Ab = (uint32_t*)(c.ws + L.off_abar);
    if (launch_build_abar(c.f, n2, (int)(n1 + 1), (int)L.kpad, S21, lds, sc.desc, Ab, L.abar_ld, c.s) !=
        hipSuccess)
        return FFP_EDEVICE;
    // S22 <- S22 - Abar Abar^T  (alpha = p - 1, beta = 1: Table 4 schedule)
    Plan pl;
    st = build_syrk_plan(schur_request(n2, L, c.f.p, lds, (((uintptr_t)S22) & 15) == 0), &pl);
    if (st != FFP_OK) return st;
    st = execute_plan(pl, Ab, S22, c.ws + L.off_syrk, c.s);
    if (st != FFP_OK) return st;
    return ldlt_rec(c, n2, S22, lds, offset + n1);
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

int ldlt_run(int64_t n, uint32_t p, uint32_t* S, int64_t lds, int64_t* info, hipStream_t s, void* ws)
{
    Ctx c;
    if (!make_field_plan(p, &c.fpl)) return FFP_EPRIME;
    c.f = Fp{p, (p - 1) / 2, c.fpl.pinv, c.fpl.ya, c.fpl.yb};
    uint32_t sq = 2;
    while (legendre(sq, p) == 1) ++sq;
    c.s_lqnr = sq;
    c.c_lqnr = (uint32_t)sqrt_mod(sq - 1, p);
    c.info = info;
    c.s = s;
    if (launch_zero_i64(info, s) != hipSuccess) return FFP_EDEVICE;
    if (!ws) {
        const size_t need = ldlt_workspace_bytes(n, p, lds);
        Workspace* w = nullptr;
        int st = acquire_workspace(s, need, 0, &w);
        if (st != FFP_OK) return st;
        ws = w->ptr;
    }
    c.linv = (uint32_t*)ws;
    c.ws = (char*)ws + linv_bytes(n);
    return ldlt_rec(c, n, S, lds, 0);
}

}  // namespace ffp
