// Schedule builder for fsyrk_modp (host only, no device calls).
#include "plan.h"
#include "tune.h"

#include <algorithm>
#include <cstdio>
#include <initializer_list>

#include "ffp.h"

namespace ffp {

int g_wide_schedule = 1;
int64_t g_winograd_min = 0;

namespace {

int64_t elem_size(int cls) { return cls == CLS_F64 ? 4 : 1; }

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

PView sub(const PView& v, int64_t r, int64_t c, int64_t es)
{
    PView o = v;
    o.off += (r * v.ld + c) * es;
    return o;
}

struct Builder {
    int cls;
    Fp fp;
    bool yb_nonzero;
    bool wide = false;
    int64_t ws_top = 0, ws_max = 0;
    std::vector<Op>* ops;

    int64_t es() const { return elem_size(cls); }

    int64_t alloc(int64_t bytes)
    {
        const int64_t off = round_up(ws_top, 256);
        ws_top = off + bytes;
        ws_max = std::max(ws_max, ws_top);
        return off;
    }

    // uint32 m x c matrix in the workspace
    PView ws_u32(int64_t rows, int64_t cols)
    {
        PView v;
        v.buf = BUF_WS;
        v.ld = std::max<int64_t>(cols, 1);
        v.off = alloc(rows * v.ld * 4);
        return v;
    }

    // operand-class rows x cols matrix in the workspace
    PView ws_opnd(int64_t rows, int64_t cols)
    {
        PView v;
        v.buf = BUF_WS;
        v.ld = round_up(std::max<int64_t>(cols, 1), 16);
        const int64_t planes = cls_planes(cls);
        v.off = alloc(rows * v.ld * es() * planes);
        v.plane = planes > 1 ? rows * v.ld : 0;
        return v;
    }

    // operand-class m x h matrix stored inside an m x m uint32 block (h <= m)
    PView in_block(const PView& blk, int64_t h) const
    {
        PView v = blk;
        v.ld = blk.ld * 4 / es();
        v.plane = (cls == CLS_LIMB2 || cls == CLS_LIMB3) ? h : 0;   // planes side by side in a row
        return v;
    }

    void emit(const Op& o) { ops->push_back(o); }

    Op op(OpKind kind, int level) const
    {
        Op o;
        o.kind = kind;
        o.cls = cls;
        o.level = level;
        return o;
    }

    void prod_syrk(int level, int64_t n, int64_t k, const PView& A, uint32_t alpha, uint32_t beta,
                   const PView& C)
    {
        Op o = op(OP_SYRK, level);
        o.m = o.n = n;
        o.k = k;
        o.alpha = alpha;
        o.beta = beta;
        o.v[0] = A;
        o.v[1] = C;
        emit(o);
    }

    void prod_gemm(int level, int64_t m, int64_t n, int64_t k, const PView& A, const PView& B,
                   uint32_t alpha, uint32_t beta, const PView& C)
    {
        Op o = op(OP_GEMM, level);
        o.m = m;
        o.n = n;
        o.k = k;
        o.alpha = alpha;
        o.beta = beta;
        o.v[0] = A;
        o.v[1] = B;
        o.v[2] = C;
        emit(o);
    }

    // v <- sum of +-in[i] mod p over m x k uint32 blocks (neg: bit i set = subtract)
    void lincomb(int level, int64_t m, int64_t k, std::initializer_list<PView> in, unsigned neg,
                 const PView& out)
    {
        Op o = op(OP_LINCOMB, level);
        o.m = m;
        o.k = k;
        o.mode = (int32_t)in.size() | (int32_t)(neg << 3);
        int i = 0;
        for (const PView& v : in) o.v[i++] = v;
        o.v[5] = out;
        emit(o);
    }

    // C <- alpha A B^T (m x n, inner k), with one level of Strassen-Winograd
    // (Algorithm 1) when the FP64 class runs with wide placements, beta = 0
    // and the product is large; X = A, Y = B^T split in 2 x 2 blocks:
    //   S1 = X21 + X22, S2 = S1 - X11, S3 = X11 - X21, S4 = X12 - S2,
    //   T1 = Y12 - Y11, T2 = Y22 - T1, T3 = Y22 - Y12, T4 = T2 - Y21,
    //   P1 = X11 Y11, P2 = X12 Y21, P3 = S4 Y22, P4 = X22 T4, P5 = S1 T1,
    //   P6 = S2 T2, P7 = S3 T3,
    //   C11 = P1 + P2, C12 = P1 + P6 + P5 + P3, C21 = P1 + P6 + P7 - P4,
    //   C22 = P1 + P6 + P7 + P5.
    // With Y = B^T the T blocks are transposes of combinations of B blocks
    // (T1^T = B21 - B11, ...), so all seven products stay of the A B^T form.
    void gemm(int level, int64_t m, int64_t n, int64_t k, const PView& A, const PView& B, uint32_t alpha,
              uint32_t beta, const PView& C)
    {
        const bool wino = g_winograd_min > 0 && cls == CLS_F64 && wide && beta == 0 && m >= g_winograd_min &&
                          n >= g_winograd_min && k >= g_winograd_min && m % 2 == 0 && n % 2 == 0 && k % 2 == 0;
        if (!wino) { prod_gemm(level, m, n, k, A, B, alpha, beta, C); return; }
        const int64_t mm = m / 2, nn = n / 2, h = k / 2, e = es();
        const PView X11 = sub(A, 0, 0, e), X12 = sub(A, 0, h, e), X21 = sub(A, mm, 0, e), X22 = sub(A, mm, h, e);
        const PView B11 = sub(B, 0, 0, e), B12 = sub(B, 0, h, e), B21 = sub(B, nn, 0, e), B22 = sub(B, nn, h, e);
        const PView S1 = ws_opnd(mm, h), S2 = ws_opnd(mm, h), S3 = ws_opnd(mm, h), S4 = ws_opnd(mm, h);
        const PView T1 = ws_opnd(nn, h), T2 = ws_opnd(nn, h), T3 = ws_opnd(nn, h), T4 = ws_opnd(nn, h);
        // each block from the quadrants directly (no chains between the
        // additions, so all eight share a level and the seven products the next)
        lincomb(level, mm, h, {X21, X22}, 0u, S1);
        lincomb(level, mm, h, {X21, X22, X11}, 4u, S2);
        lincomb(level, mm, h, {X11, X21}, 2u, S3);
        lincomb(level, mm, h, {X12, X21, X22, X11}, 6u, S4);                 // X12 - S2
        lincomb(level, nn, h, {B21, B11}, 2u, T1);                           // T1^T
        lincomb(level, nn, h, {B22, B21, B11}, 2u, T2);                      // T2^T = B22 - T1^T
        lincomb(level, nn, h, {B22, B21}, 2u, T3);                           // T3^T
        lincomb(level, nn, h, {B22, B21, B11, B12}, 10u, T4);                // T4^T = T2^T - B12
        PView P[7];
        for (PView& v : P) v = ws_u32(mm, round_up(nn, 4));
        prod_gemm(level, mm, nn, h, X11, B11, alpha, 0, P[0]);
        prod_gemm(level, mm, nn, h, X12, B12, alpha, 0, P[1]);
        prod_gemm(level, mm, nn, h, S4, B22, alpha, 0, P[2]);
        prod_gemm(level, mm, nn, h, X22, T4, alpha, 0, P[3]);
        prod_gemm(level, mm, nn, h, S1, T1, alpha, 0, P[4]);
        prod_gemm(level, mm, nn, h, S2, T2, alpha, 0, P[5]);
        prod_gemm(level, mm, nn, h, S3, T3, alpha, 0, P[6]);
        const PView C11 = sub(C, 0, 0, 4), C12 = sub(C, 0, nn, 4), C21 = sub(C, mm, 0, 4), C22 = sub(C, mm, nn, 4);
        lincomb(level, mm, nn, {P[0], P[1]}, 0u, C11);
        lincomb(level, mm, nn, {P[0], P[5], P[4], P[2]}, 0u, C12);
        lincomb(level, mm, nn, {P[0], P[5], P[6], P[3]}, 8u, C21);
        lincomb(level, mm, nn, {P[0], P[5], P[6], P[4]}, 0u, C22);
    }

    // Table 3: lower(C) <- alpha A A^T, with C's strict upper triangle as the
    // only temporary when k <= n; two m x h workspace blocks otherwise.
    void syrk3(int d, int level, int64_t n, int64_t k, const PView& A, uint32_t alpha, const PView& C)
    {
        if (d == 0) { prod_syrk(level, n, k, A, alpha, 0, C); return; }
        const int64_t m = n / 2, h = k / 2, e = es();
        const PView A11 = sub(A, 0, 0, e), A12 = sub(A, 0, h, e), A21 = sub(A, m, 0, e),
                    A22 = sub(A, m, h, e);
        const PView C11 = sub(C, 0, 0, 4), C12 = sub(C, 0, m, 4), C21 = sub(C, m, 0, 4),
                    C22 = sub(C, m, m, 4);
        const int64_t save = ws_top;
        PView S1, S2, S4;
        if (h <= m && !wide) {
            S1 = in_block(C21, h);    // S1, then S3 in place
            S2 = in_block(C12, h);
            S4 = in_block(C11, h);
        } else {
            S1 = ws_opnd(m, h);
            S2 = ws_opnd(m, h);
            S4 = S2;                  // S2 is dead once P4^T is formed
        }
        Op a = op(OP_S1S2, level);
        a.m = m; a.k = h;
        a.v[0] = A11; a.v[1] = A21; a.v[2] = A22; a.v[3] = S1; a.v[4] = S2;
        emit(a);
        gemm(level, m, m, h, S2, S1, alpha, 0, C22);                       // P4^T = S2 S1^T
        Op b = op(OP_S34, level);
        b.mode = 3; b.m = m; b.k = h;
        b.v[0] = S1; b.v[1] = A22; b.v[2] = A12; b.v[3] = S1; b.v[4] = S4;
        emit(b);                                                            // S3 = S1 - A22, S4 = S3 + A12
        syrk3(d - 1, level + 1, m, h, S1, alpha, C12);                     // P5 = S3 S3^T
        gemm(level, m, m, h, A22, S4, alpha, 0, C21);                      // P3 = A22 S4^T
        syrk3(d - 1, level + 1, m, h, A11, alpha, C11);                    // P1 = A11 A11^T
        Op c = op(OP_POSTADD, level);
        c.m = m;
        c.v[0] = C11; c.v[1] = C12; c.v[2] = C22; c.v[3] = C21;
        emit(c);                                                            // U1, U2, U4 -> C21, U5 -> C22
        // P2 = A12 A12^T: in place of P5 (C12), or in a block of its own
        const PView P2 = wide ? ws_u32(m, round_up(m, 4)) : C12;
        syrk3(d - 1, level + 1, m, h, A12, alpha, P2);
        Op u = op(OP_ADDLOW, level);
        u.m = m;
        u.v[0] = C11; u.v[1] = P2; u.v[2] = C11;
        emit(u);                                                            // U3 = P1 + P2
        if (!wide) ws_top = save;
    }

    // Table 4: lower(C) <- alpha A A^T + beta lower(C), with C12 and one
    // m x m block tmp as temporaries, plus an m-vector keeping diag(C22),
    // which Up(C11) cannot hold.
    void syrk4(int d, int level, int64_t n, int64_t k, const PView& A, uint32_t alpha,
               uint32_t beta, const PView& C)
    {
        if (d == 0) { prod_syrk(level, n, k, A, alpha, beta, C); return; }
        const int64_t m = n / 2, h = k / 2, e = es();
        const PView A11 = sub(A, 0, 0, e), A12 = sub(A, 0, h, e), A21 = sub(A, m, 0, e),
                    A22 = sub(A, m, h, e);
        const PView C11 = sub(C, 0, 0, 4), C12 = sub(C, 0, m, 4), C21 = sub(C, m, 0, 4),
                    C22 = sub(C, m, m, 4);
        const int64_t save = ws_top;
        const PView tmp = ws_u32(m, round_up(m, 4));
        const PView dvec = ws_u32(1, m);
        PView S1, S2;
        if (h <= m) {
            S1 = in_block(tmp, h);     // S1 -> S3 -> S4 in place
            S2 = in_block(C12, h);
        } else {
            S1 = ws_opnd(m, h);
            S2 = ws_opnd(m, h);
        }
        Op a = op(OP_S1S2, level);
        a.m = m; a.k = h;
        a.v[0] = A11; a.v[1] = A21; a.v[2] = A22; a.v[3] = S1; a.v[4] = S2;
        emit(a);
        Op sv = op(OP_SAVEC22, level);
        sv.m = m;
        sv.v[0] = C22; sv.v[1] = C11; sv.v[2] = dvec;
        emit(sv);                                                            // Up(C11) = Low(C22)^T, diag
        prod_gemm(level, m, m, h, S2, S1, alpha, 0, C22);                  // P4^T = alpha S2 S1^T
        Op b3 = op(OP_S34, level);
        b3.mode = 1; b3.m = m; b3.k = h;
        b3.v[0] = S1; b3.v[1] = A22; b3.v[2] = A12; b3.v[3] = S1; b3.v[4] = S1;
        emit(b3);                                                           // S3 = S1 - A22
        syrk3(d - 1, level + 1, m, h, S1, alpha, C12);                     // P5 = alpha S3 S3^T
        Op b4 = op(OP_S34, level);
        b4.mode = 2; b4.m = m; b4.k = h;
        b4.v[0] = S1; b4.v[1] = A22; b4.v[2] = A12; b4.v[3] = S1; b4.v[4] = S1;
        emit(b4);                                                           // S4 = S3 + A12
        prod_gemm(level, m, m, h, A22, S1, alpha, beta, C21);              // P3 = alpha A22 S4^T + beta C21
        syrk3(d - 1, level + 1, m, h, A11, alpha, tmp);                    // P1 = alpha A11 A11^T
        Op c = op(OP_POSTADD, level);
        c.m = m;
        c.beta = beta;
        c.v[0] = tmp; c.v[1] = C12; c.v[2] = C22; c.v[3] = C21; c.v[4] = C11; c.v[5] = dvec;
        emit(c);                                                            // U4, U5 (+ beta C22)
        syrk4(d - 1, level + 1, m, h, A12, alpha, beta, C11);              // P2 = alpha A12 A12^T + beta C11
        Op u = op(OP_ADDLOW, level);
        u.m = m;
        u.v[0] = tmp; u.v[1] = C11; u.v[2] = C11;
        emit(u);                                                            // U3 = P1 + P2
        ws_top = save;
    }
};

}  // namespace

namespace {
bool valid_dtype_(int d) { return d == FFP_U32 || d == FFP_I8_CENTERED || d == FFP_I8_LIMB2; }

int dtype_cls(int d)
{
    switch (d) {
    case FFP_I8_CENTERED: return CLS_I8;
    case FFP_I8_LIMB2: return CLS_LIMB2;
    default: return CLS_F64;
    }
}

bool aligned16(const void* p) { return (((uintptr_t)p) & 15) == 0; }

}  // namespace

int make_syrk_request(int64_t n, int64_t k, uint32_t p, const void* A, int64_t lda, int a_dtype,
                 uint32_t alpha, uint32_t beta, const uint32_t* C, int64_t ldc, unsigned flags,
                 PlanRequest* rq)
{
    if (n < 0 || k < 0) return FFP_EINVAL;
    if (!valid_dtype_(a_dtype)) return FFP_EDTYPE;
    if (!supported_prime(p)) return FFP_EPRIME;
    // the int8 storages hold odd-p residues (centred, or two limbs)
    if (a_dtype == FFP_I8_CENTERED && (p > 251 || p == 2)) return FFP_EDTYPE;
    if (a_dtype == FFP_I8_LIMB2 && (p > 65521 || p == 2)) return FFP_EDTYPE;
    if (alpha >= p || beta >= p) return FFP_EINVAL;
    if (n > 0 && (C == nullptr || ldc < n)) return FFP_EINVAL;
    if (n > 0 && k > 0 && (A == nullptr || lda < k)) return FFP_EINVAL;
    if (n > (int64_t)1 << 30 || k > (int64_t)1 << 30) return FFP_EINVAL;
    rq->n = n;
    rq->k = k;
    rq->p = p;
    rq->a_cls = dtype_cls(a_dtype);
    rq->lda = lda;
    rq->ldc = ldc;
    rq->a_plane = a_dtype == FFP_I8_LIMB2 ? n * lda : 0;
    rq->alpha = alpha;
    rq->beta = beta;
    const unsigned dfield = (flags >> 4) & 0xFu;
    rq->depth = dfield ? (int)dfield - 1 : -1;
    rq->fill_upper = (flags & FFP_FILL_UPPER) != 0;
    rq->force_f64 = (flags & FFP_BASE_F64) != 0;
    rq->force_limb3 = (flags & FFP_BASE_LIMB3) != 0;
    if (rq->force_f64 && rq->force_limb3) return FFP_EINVAL;
    if (rq->force_limb3 && (a_dtype != FFP_U32 || p >= (1u << 23))) return FFP_EDTYPE;
    rq->wide = g_wide_schedule != 0 && (flags & FFP_LOW_MEMORY) == 0;
    rq->a_aligned16 = aligned16(A);
    rq->c_aligned16 = aligned16(C);
    return FFP_OK;
}

int choose_class(uint32_t p, int a_cls, bool force_f64, bool force_limb3)
{
    if (a_cls == CLS_I8) return CLS_I8;
    if (a_cls == CLS_LIMB2) return CLS_LIMB2;
    if (force_f64) return CLS_F64;
    if (force_limb3) return CLS_LIMB3;
    if (p == 2) return CLS_F64;     // residues 0, 1 (centred: 0, -1) on FP64 matrix cores
    if (p <= 251) return CLS_I8;
    if (p <= 65521) return CLS_LIMB2;
    return CLS_F64;
}

int default_depth(int cls, int64_t n, int64_t k)
{
    // Each level trades one eighth of the multiply-adds (5 products instead
    // of 6 on half-size blocks, Table 1) for HBM-bound block additions.  On
    // FP64 matrix cores that trade pays while the leaves stay large enough
    // to fill the chip.  Three int8 limbs (nine products per block): one
    // level pays once n and k / 2 reach 4096 (p = 131071: 8192 x 8192 2.16
    // against 2.26 ms at depth 0, 8192 x 32768 7.32 against 8.56 ms,
    // 16384^2 14.1 against 16.0 ms; 4096^2 0.39 against 0.32 ms; depth 2
    // slower than depth 1 everywhere).  One int8
    // plane and two limbs: the additions cost as much as or more than the
    // saved products at every size measured (16384^2: int8 2.17 ms at depth
    // 0, 2.50 at depth 1; two limbs 7.50 and 7.52 ms), so no recursion.
    if (cls == CLS_LIMB3) return std::min(n, k / 2) >= 4096 ? 1 : 0;
    const int64_t nn = std::min(n, 2 * k);
    if (cls != CLS_F64) return 0;
    int d = 0;
    while (d < 4 && (nn >> (d + 1)) >= 1024) ++d;
    return d;
}

int build_syrk_plan(const PlanRequest& rq, Plan* out)
{
    if (rq.n < 0 || rq.k < 0) return FFP_EINVAL;
    Plan pl;
    if (!supported_prime(rq.p) || !make_field_plan(rq.p, &pl.field)) return FFP_EPRIME;
    pl.cls = choose_class(rq.p, rq.a_cls, rq.force_f64, rq.force_limb3);
    if (pl.cls == CLS_I8 && rq.p > 251) return FFP_EDTYPE;
    if (pl.cls == CLS_LIMB2 && rq.p > 65521) return FFP_EDTYPE;
    if (pl.cls == CLS_LIMB3 && rq.p >= (1u << 23)) return FFP_EDTYPE;
    const int64_t n = rq.n, k = rq.k;

    int d = rq.depth;
    bool wide = rq.wide;
    int tile = rq.tile;
    if (!rq.no_tune) {
        TuneChoice tc;
        if (tune_lookup(pl.cls, n, k, rq.alpha != 1u || rq.beta != 0u, !rq.wide, &tc)) {
            if (d < 0) {
                d = tc.depth;
                wide = rq.wide && tc.wide != 0;
                pl.tuned = true;
                // the table may move FP64-path shapes (uint32 operands, p < 2^23)
                // to the three-limb int8 products
                if (tc.base == CLS_LIMB3 && pl.cls == CLS_F64 && rq.a_cls == CLS_F64 && !rq.force_f64 &&
                    rq.p < (1u << 23))
                    pl.cls = CLS_LIMB3;
            }
            if (d == tc.depth && tile == 0) tile = tc.tile;
        }
    }
    if (d < 0) d = default_depth(pl.cls, n, k);
    while (d > 0 && (n >> d) < 8) --d;
    if (k == 0) d = 0;
    pl.depth = d;
    pl.wide = wide;
    pl.tile = tile;

    const int64_t es_op = elem_size(pl.cls);
    int64_t kunit = ((pl.cls == CLS_F64) ? 4 : 64) << (d + (pl.field.yb ? 1 : 0));
    // three-limb leaf products with k a multiple of 128 can take the
    // direct-to-LDS tile (whole 128-byte stages)
    if (pl.cls == CLS_LIMB3 && kunit < ((int64_t)128 << d)) kunit = (int64_t)128 << d;
    const int64_t nunit = d > 0 ? (int64_t)4 << d : 1;
    const int64_t n_pad = n == 0 ? 0 : round_up(n, nunit);
    const int64_t k_pad = k == 0 ? 0 : round_up(k, (pl.cls == CLS_F64 && d == 0) ? 1 : kunit);
    pl.n_pad = n_pad;
    pl.k_pad = k_pad;

    Builder B;
    B.cls = pl.cls;
    B.fp = Fp{rq.p, (rq.p - 1) / 2, pl.field.pinv, pl.field.ya, pl.field.yb};
    B.yb_nonzero = pl.field.yb != 0;
    B.wide = wide;
    B.ops = &pl.ops;

    // Operand: pack when the class, the shape or the alignment differ.
    PView A;
    A.buf = BUF_A;
    A.off = 0;
    A.ld = rq.lda;
    A.plane = rq.a_plane;
    bool a_ok = (pl.cls == rq.a_cls) && n_pad == n && k_pad == k;
    if (pl.cls == CLS_F64) a_ok = a_ok && (d == 0 || ((rq.lda % 4) == 0 && rq.a_aligned16));
    else a_ok = a_ok && (rq.lda % 16) == 0 && rq.a_aligned16 &&
                (pl.cls == CLS_I8 || (rq.a_plane % 16) == 0);
    if (!a_ok && n_pad > 0 && k_pad > 0) {
        PView Ap = B.ws_opnd(n_pad, k_pad);
        Op o = B.op(OP_PACK, 0);
        o.src_cls = rq.a_cls;
        o.m = n_pad; o.k = k_pad; o.m_src = n; o.k_src = k;
        o.v[0] = A; o.v[1] = Ap;
        B.emit(o);
        A = Ap;
    }
    (void)es_op;

    // Output: a padded copy when n is padded or C's layout breaks alignment.
    PView C;
    C.buf = BUF_C;
    C.ld = rq.ldc;
    bool c_copy = n_pad != n || (d > 0 && ((rq.ldc % 4) != 0 || !rq.c_aligned16));
    PView Cw = C;
    if (c_copy && n_pad > 0) {
        Cw = B.ws_u32(n_pad, round_up(n_pad, 4));
        Op o = B.op(OP_PACK, 0);
        o.cls = CLS_F64;
        o.src_cls = CLS_F64;
        o.m = n_pad; o.k = n_pad; o.m_src = rq.beta ? n : 0; o.k_src = rq.beta ? n : 0;
        o.v[0] = C; o.v[1] = Cw;
        B.emit(o);                 // zero-padded copy (copies C only when beta != 0)
    }

    if (n_pad > 0) {
        if (k_pad == 0) {
            // A A^T = 0: lower(C) <- beta lower(C), as a product with k = 0
            B.prod_syrk(0, n_pad, 0, A, rq.alpha, rq.beta, Cw);
        } else if (rq.beta == 0) {
            B.syrk3(d, 0, n_pad, k_pad, A, rq.alpha, Cw);
        } else {
            B.syrk4(d, 0, n_pad, k_pad, A, rq.alpha, rq.beta, Cw);
        }
    }

    if (c_copy && n > 0) {
        Op o = B.op(OP_COPY, 0);
        o.cls = CLS_F64;
        o.mode = 1;
        o.m = n; o.n = n;
        o.v[0] = Cw; o.v[1] = C;
        B.emit(o);
    }
    if (rq.fill_upper && n > 0) {
        Op o = B.op(OP_MIRROR, 0);
        o.cls = CLS_F64;
        o.m = n;
        o.v[0] = C;
        B.emit(o);
    }
    pl.ws_bytes = B.ws_max;
    *out = std::move(pl);
    return FFP_OK;
}

std::string describe_plan(const Plan& pl)
{
    std::string s;
    char buf[512];
    snprintf(buf, sizeof buf,
             "plan cls=%d depth=%d n_pad=%lld k_pad=%lld ws=%lld ya=%u yb=%u wide=%d tile=%d tuned=%d\n",
             pl.cls, pl.depth, (long long)pl.n_pad, (long long)pl.k_pad, (long long)pl.ws_bytes,
             pl.field.ya, pl.field.yb, pl.wide ? 1 : 0, pl.tile, pl.tuned ? 1 : 0);
    s += buf;
    for (const Op& o : pl.ops) {
        snprintf(buf, sizeof buf, "op %d %d %d %d %lld %lld %lld %lld %lld %u %u %d", (int)o.kind, o.cls,
                 o.src_cls, o.mode, (long long)o.m, (long long)o.n, (long long)o.k,
                 (long long)o.m_src, (long long)o.k_src, o.alpha, o.beta, o.level);
        s += buf;
        for (int i = 0; i < 6; ++i) {
            snprintf(buf, sizeof buf, " %d %lld %lld %lld", o.v[i].buf, (long long)o.v[i].off,
                     (long long)o.v[i].ld, (long long)o.v[i].plane);
            s += buf;
        }
        for (int i = 0; i < 5; ++i) {
            snprintf(buf, sizeof buf, " %u", o.coef[i]);
            s += buf;
        }
        s += "\n";
    }
    return s;
}

}  // namespace ffp
