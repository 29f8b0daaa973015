// Schedules of the symmetric products over F_p[i] = F_p[x]/(x^2 + 1) (the
// field F_(p^2) when p = 3 mod 4): C = A A^T (Section 3.1, complex field:
// Algorithm 2 with Y = i I) and C = A A^H with conj(a + ib) = a - ib
// (Section 3.3: Algorithm 2 with conjugate transposition and
// Y = (a + ib) I, a^2 + b^2 = -1 in F_p).  An element is a pair of residues
// (re, im) and a matrix two uint32 planes; every block operation of the
// complex recursion is written as operations on planes:
//   - the pre-additions S1..S4 and the post-additions as linear
//     combinations of planes with coefficients (OP_LCT), multiplication by
//     Y = a + ib included: (u + iv)(a + ib) = (au - bv) + i(bu + av);
//   - the general products P3, P4 as three real products each (the 3M
//     method of Section 4.1), e.g. for A B^T: T1 = Ar Br^T, T2 = Ai Bi^T,
//     T3 = (Ar + Ai)(Br + Bi)^T, re = T1 - T2, im = T3 - T1 - T2;
//   - the leaves as two real products (the 2M method of Section 4.1):
//     A A^T: H = X Y^T, G = (X + Y)(X - Y)^T, re = G - H^T + H,
//     im = H + H^T;  A A^H: H = X Y^T, G = (X + Y)(X + Y)^T (a real
//     symmetric product), re = G - H - H^T, im = H^T - H;
//     only the lower triangles are formed (G as lower-triangle tiles).
// The real products run on the FP64 matrix cores (uint32 operands).
#include "cplan.h"

#include <algorithm>
#include <initializer_list>

#include "ffp.h"

namespace ffp {

namespace {

int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

PView subv(const PView& v, int64_t r, int64_t c) { PView o = v; o.off += (r * v.ld + c) * 4; return o; }

struct CView {
    PView re, im;
    CView sub(int64_t r, int64_t c) const { return CView{subv(re, r, c), subv(im, r, c)}; }
};

struct Term {
    PView v;
    uint32_t c;
    bool t;
};

struct CBuilder {
    uint32_t p;
    bool herk;
    uint32_t ya, yb;        // Y = ya + i yb
    int64_t ws_top = 0, ws_max = 0;
    std::vector<Op>* ops;

    uint32_t neg(uint32_t x) const { return x == 0 ? 0 : p - x; }

    PView ws(int64_t rows, int64_t cols)
    {
        PView v;
        v.buf = BUF_WS;
        v.ld = rup(std::max<int64_t>(cols, 1), 4);
        const int64_t off = rup(ws_top, 256);
        ws_top = off + rows * v.ld * 4;
        ws_max = std::max(ws_max, ws_top);
        v.off = off;
        return v;
    }
    CView wsc(int64_t rows, int64_t cols) { return CView{ws(rows, cols), ws(rows, cols)}; }

    // out (m x k) <- sum of terms; lower: lower triangle only
    void lct(int level, int64_t m, int64_t k, std::initializer_list<Term> terms, const PView& out, bool lower = false)
    {
        Op o;
        o.kind = OP_LCT;
        o.cls = CLS_F64;
        o.level = level;
        o.m = m;
        o.k = k;
        int i = 0, mode = 0;
        for (const Term& t : terms) {
            o.v[i] = t.v;
            o.coef[i] = t.c % p;
            if (t.t) mode |= 1 << (3 + i);
            ++i;
        }
        o.mode = mode | i | (lower ? 256 : 0);
        o.v[5] = out;
        ops->push_back(o);
    }

    void gemm(int level, int64_t m, int64_t n, int64_t k, const PView& A, const PView& B, const PView& C,
              bool lower = false)
    {
        Op o;
        o.kind = OP_GEMM;
        o.cls = CLS_F64;
        o.level = level;
        o.mode = lower ? 1 : 0;
        o.m = m;
        o.n = n;
        o.k = k;
        o.v[0] = A;
        o.v[1] = B;
        o.v[2] = C;
        ops->push_back(o);
    }

    void syrk(int level, int64_t n, int64_t k, const PView& A, const PView& C)
    {
        Op o;
        o.kind = OP_SYRK;
        o.cls = CLS_F64;
        o.level = level;
        o.m = o.n = n;
        o.k = k;
        o.v[0] = A;
        o.v[1] = C;
        ops->push_back(o);
    }

    void mirror(int level, int64_t n, const PView& C, bool negate)
    {
        Op o;
        o.kind = OP_MIRROR;
        o.cls = CLS_F64;
        o.level = level;
        o.mode = negate ? 1 : 0;
        o.m = n;
        o.v[0] = C;
        ops->push_back(o);
    }

    // C (m x n) <- A B^T, or A B^H for herk, by the 3M method
    void cgemm(int level, int64_t m, int64_t n, int64_t k, const CView& A, const CView& B, const CView& C)
    {
        const PView SA = ws(m, k), SB = ws(n, k);
        lct(level, m, k, {{A.re, 1, false}, {A.im, 1, false}}, SA);
        lct(level, n, k, {{B.re, 1, false}, {B.im, herk ? p - 1 : 1, false}}, SB);   // Br -+ Bi
        const PView T1 = ws(m, n), T2 = ws(m, n), T3 = ws(m, n);
        gemm(level, m, n, k, A.re, B.re, T1);
        gemm(level, m, n, k, A.im, B.im, T2);
        gemm(level, m, n, k, SA, SB, T3);
        if (!herk) {
            lct(level, m, n, {{T1, 1, false}, {T2, p - 1, false}}, C.re);                    // T1 - T2
            lct(level, m, n, {{T3, 1, false}, {T1, p - 1, false}, {T2, p - 1, false}}, C.im); // T3 - T1 - T2
        } else {
            lct(level, m, n, {{T1, 1, false}, {T2, 1, false}}, C.re);                        // T1 + T2
            lct(level, m, n, {{T3, 1, false}, {T1, p - 1, false}, {T2, 1, false}}, C.im);     // T3 - T1 + T2
        }
    }

    // lower(C) <- A A^T (A A^H), A n x k, by the 2M method
    void leaf(int level, int64_t n, int64_t k, const CView& A, const CView& C)
    {
        const PView H = ws(n, n), G = ws(n, n), S = ws(n, k);
        gemm(level, n, n, k, A.re, A.im, H);                                            // H = X Y^T
        if (!herk) {
            const PView D = ws(n, k);
            lct(level, n, k, {{A.re, 1, false}, {A.im, 1, false}}, S);                  // X + Y
            lct(level, n, k, {{A.re, 1, false}, {A.im, p - 1, false}}, D);              // X - Y
            gemm(level, n, n, k, S, D, G, true);                                        // lower of (X+Y)(X-Y)^T
            lct(level, n, n, {{G, 1, false}, {H, 1, false}, {H, p - 1, true}}, C.re, true);   // G + H - H^T
            lct(level, n, n, {{H, 1, false}, {H, 1, true}}, C.im, true);                      // H + H^T
        } else {
            lct(level, n, k, {{A.re, 1, false}, {A.im, 1, false}}, S);                  // X + Y
            syrk(level, n, k, S, G);                                                    // lower of (X+Y)(X+Y)^T
            lct(level, n, n, {{G, 1, false}, {H, p - 1, false}, {H, p - 1, true}}, C.re, true);  // G - H - H^T
            lct(level, n, n, {{H, 1, true}, {H, p - 1, false}}, C.im, true);                     // H^T - H
        }
    }

    // lower(C) <- A A^T (A A^H): Algorithm 2 over F_p[i] to depth d, its
    // blocks S1..S4, P1..P5 and U's in the workspace (n, k divisible by 2^d)
    void csyrk(int d, int level, int64_t n, int64_t k, const CView& A, const CView& C)
    {
        if (d == 0) { leaf(level, n, k, A, C); return; }
        const int64_t m = n / 2, h = k / 2;
        const CView A11 = A.sub(0, 0), A12 = A.sub(0, h), A21 = A.sub(m, 0), A22 = A.sub(m, h);
        const uint32_t a = ya, b = yb;
        // S1 = (A21 - A11) Y
        const CView S1 = wsc(m, h), S2 = wsc(m, h), S3 = wsc(m, h), S4 = wsc(m, h);
        lct(level, m, h, {{A21.re, a, false}, {A11.re, neg(a), false}, {A21.im, neg(b), false}, {A11.im, b, false}},
            S1.re);
        lct(level, m, h, {{A21.re, b, false}, {A11.re, neg(b), false}, {A21.im, a, false}, {A11.im, neg(a), false}},
            S1.im);
        // S2 = A22 - A21 Y
        lct(level, m, h, {{A22.re, 1, false}, {A21.re, neg(a), false}, {A21.im, b, false}}, S2.re);
        lct(level, m, h, {{A22.im, 1, false}, {A21.re, neg(b), false}, {A21.im, neg(a), false}}, S2.im);
        // S3 = S1 - A22, S4 = S3 + A12
        lct(level, m, h, {{S1.re, 1, false}, {A22.re, p - 1, false}}, S3.re);
        lct(level, m, h, {{S1.im, 1, false}, {A22.im, p - 1, false}}, S3.im);
        lct(level, m, h, {{S3.re, 1, false}, {A12.re, 1, false}}, S4.re);
        lct(level, m, h, {{S3.im, 1, false}, {A12.im, 1, false}}, S4.im);
        // P4^T = S2 S1^T (P4^H = S2 S1^H), P3 = A22 S4^T (A22 S4^H)
        const CView P4t = wsc(m, m), P3 = wsc(m, m), P1 = wsc(m, m), P2 = wsc(m, m), P5 = wsc(m, m);
        cgemm(level, m, m, h, S2, S1, P4t);
        cgemm(level, m, m, h, A22, S4, P3);
        // P5 = S3 S3^T, P1 = A11 A11^T, P2 = A12 A12^T (recursive); P1, P5 in full
        csyrk(d - 1, level + 1, m, h, S3, P5);
        csyrk(d - 1, level + 1, m, h, A11, P1);
        csyrk(d - 1, level + 1, m, h, A12, P2);
        mirror(level, m, P5.re, false);
        mirror(level, m, P5.im, herk);
        mirror(level, m, P1.re, false);
        mirror(level, m, P1.im, herk);
        // P4 = (P4^T)^T, or (P4^H)^H: the imaginary plane transposed and negated
        const uint32_t s4 = herk ? p - 1 : 1;
        const CView C11 = C.sub(0, 0), C21 = C.sub(m, 0), C22 = C.sub(m, m);
        // U4 = P1 + P5 + P4 + P3 -> C21;  U5 = P1 + P5 + P4 + P4^T -> Low(C22);  U3 = P1 + P2 -> Low(C11)
        lct(level, m, m, {{P1.re, 1, false}, {P5.re, 1, false}, {P4t.re, 1, true}, {P3.re, 1, false}}, C21.re);
        lct(level, m, m, {{P1.im, 1, false}, {P5.im, 1, false}, {P4t.im, s4, true}, {P3.im, 1, false}}, C21.im);
        lct(level, m, m, {{P1.re, 1, false}, {P5.re, 1, false}, {P4t.re, 1, true}, {P4t.re, 1, false}}, C22.re, true);
        lct(level, m, m, {{P1.im, 1, false}, {P5.im, 1, false}, {P4t.im, s4, true}, {P4t.im, 1, false}}, C22.im,
            true);
        lct(level, m, m, {{P1.re, 1, false}, {P2.re, 1, false}}, C11.re, true);
        lct(level, m, m, {{P1.im, 1, false}, {P2.im, 1, false}}, C11.im, true);
    }
};

}  // namespace

int default_complex_depth(int64_t n, int64_t k)
{
    // Each level saves an eighth of the real products for a dozen
    // plane-wise block additions; measured on the FP64 matrix cores the
    // trade pays from n = 8192 (n = k = 8192, p = 131071: 24.6 ms at depth
    // 0, 23.0 ms at depth 1; n = 4096: 3.63 ms at depth 0, 3.70 at depth 1).
    int d = 0;
    const int64_t nn = std::min(n, 2 * k);
    while (d < 4 && (nn >> (d + 1)) >= 4096) ++d;
    return d;
}

int build_complex_plan(const ComplexRequest& rq, Plan* out)
{
    if (rq.n < 0 || rq.k < 0) return FFP_EINVAL;
    Plan pl;
    if (rq.p < 3 || !supported_prime(rq.p) || !make_field_plan(rq.p, &pl.field)) return FFP_EPRIME;
    pl.cls = CLS_F64;
    int d = rq.depth >= 0 ? rq.depth : default_complex_depth(rq.n, rq.k);
    while (d > 0 && (rq.n >> d) < 8) --d;
    if (rq.k == 0) d = 0;
    pl.depth = d;
    const int64_t unit = (int64_t)1 << d;
    const int64_t n = rq.n, k = rq.k;
    const int64_t n_pad = rup(n, unit), k_pad = rup(k, unit);
    pl.n_pad = n_pad;
    pl.k_pad = k_pad;

    CBuilder B;
    B.p = rq.p;
    B.herk = rq.herk;
    // Y = i I for the symmetric product; Y = (a + ib) I with a^2 + b^2 = -1
    // in F_p (the field plan's pair) for the Hermitian one
    B.ya = rq.herk ? pl.field.ya : 0u;
    B.yb = rq.herk ? pl.field.yb : 1u;
    B.ops = &pl.ops;

    CView A{PView{BUF_A, 0, rq.lda, 0}, PView{BUF_A, rq.a_plane * 4, rq.lda, 0}};
    CView C{PView{BUF_C, 0, rq.ldc, 0}, PView{BUF_C, rq.c_plane * 4, rq.ldc, 0}};
    if (n > 0 && k > 0 && (n_pad != n || k_pad != k)) {
        // zero-padded copy of both planes
        const CView Ap = B.wsc(n_pad, k_pad);
        const PView src[2] = {A.re, A.im}, dst[2] = {Ap.re, Ap.im};
        for (int q = 0; q < 2; ++q) {
            Op o;
            o.kind = OP_PACK;
            o.cls = CLS_F64;
            o.src_cls = CLS_F64;
            o.m = n_pad; o.k = k_pad; o.m_src = n; o.k_src = k;
            o.v[0] = src[q];
            o.v[1] = dst[q];
            pl.ops.push_back(o);
        }
        A = Ap;
    }
    const bool c_copy = n_pad != n;
    CView Cw = c_copy && n > 0 ? B.wsc(n_pad, n_pad) : C;
    if (n > 0) {
        if (k == 0) {
            B.lct(0, n_pad, n_pad, {{Cw.re, 0, false}}, Cw.re, true);
            B.lct(0, n_pad, n_pad, {{Cw.im, 0, false}}, Cw.im, true);
        } else {
            B.csyrk(d, 0, n_pad, k_pad, A, Cw);
        }
    }
    if (c_copy && n > 0) {
        const PView src[2] = {Cw.re, Cw.im}, dst[2] = {C.re, C.im};
        for (int q = 0; q < 2; ++q) {
            Op o;
            o.kind = OP_COPY;
            o.cls = CLS_F64;
            o.mode = 1;
            o.m = n; o.n = n;
            o.v[0] = src[q];
            o.v[1] = dst[q];
            pl.ops.push_back(o);
        }
    }
    if (rq.fill_upper && n > 0) {
        B.mirror(0, n, C.re, false);
        B.mirror(0, n, C.im, rq.herk);
    }
    pl.ws_bytes = B.ws_max;
    *out = std::move(pl);
    return FFP_OK;
}

}  // namespace ffp
