// Host-side schedule of one fsyrk_modp call: a list of block operations on
// views of three buffers (the operand A, the output C and the library's
// workspace), built without touching the device.  The schedule follows
// Algorithm 2 with the placements of Table 3 (beta = 0) and Table 4
// (beta != 0), recursing depth-first.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "field.h"
#include "kernels.h"

namespace ffp {

enum BufId : int32_t { BUF_A = 0, BUF_C = 1, BUF_WS = 2, BUF_A_LO = 3 };

// View of a matrix inside one buffer.  `off` is in bytes from the buffer
// start; `ld` and `plane` are in elements of the view's storage type.
struct PView {
    int32_t buf = BUF_WS;
    int64_t off = 0;
    int64_t ld = 0;
    int64_t plane = 0;
};

enum OpKind : int32_t {
    OP_S1S2 = 0,     // v0=A11 v1=A21 v2=A22 -> v3=S1 v4=S2      (m x k blocks)
    OP_S34 = 1,      // mode bit0: v3=S3 <- v0=S1 - v1=A22; bit1: v4=S4 <- S3 + v2=A12
    OP_GEMM = 2,     // v2 <- alpha v0 v1^T + beta v2   (m x n, inner k)
    OP_SYRK = 3,     // lower(v1) <- alpha v0 v0^T + beta lower(v1)   (n = m)
    OP_POSTADD = 4,  // v0=P1 v1=P5 v2=C22(P4^T) v3=C21(P3) [beta: v4=Up(C11) v5=dvec]
    OP_ADDLOW = 5,   // lower(v2) <- lower(v0) + lower(v1)
    OP_SAVEC22 = 6,  // Up(v1) <- Low(v0)^T strictly, v2 <- diag(v0)
    OP_MIRROR = 7,   // Up(v0) <- Low(v0)^T
    OP_PACK = 8,     // v1 (class cls, m x k padded from n x k... see pack_*) <- v0 (class src_cls)
    OP_COPY = 9,     // v1 <- v0 (m x n uint32), mode 1: lower triangle only
    OP_LINCOMB = 10, // v5 <- sum of +-v_i, i < (mode & 7), mod p; bit 3 + i of mode: subtract v_i
                     // (m x k uint32 blocks; the Strassen-Winograd additions)
    OP_LCT = 11,     // v5 <- sum of coef[i] * op_i(v_i), i < (mode & 7), mod p, over m x k uint32;
                     // bit 3 + i of mode: op_i is the transpose (v_i is k x m); bit 8: lower
                     // triangle only (m = k)
};
// OP_GEMM mode bit 0: lower-triangle tiles of C only (m = n; the product
// A B^T need not be symmetric).  OP_MIRROR mode bit 0: Up(v0) <- -Low(v0)^T.

struct Op {
    OpKind kind;
    int32_t cls = CLS_F64;      // storage class of operand views (S, A)
    int32_t src_cls = CLS_F64;  // OP_PACK source class
    int32_t mode = 0;
    int64_t m = 0, n = 0, k = 0;
    int64_t m_src = 0, k_src = 0;  // OP_PACK: valid source extent
    uint32_t alpha = 1, beta = 0;
    int32_t level = 0;          // recursion level that emitted the op
    PView v[6];
    uint32_t coef[5] = {1, 1, 1, 1, 1};   // OP_LCT
};

struct PlanRequest {
    int64_t n = 0, k = 0;
    uint32_t p = 0;
    int32_t a_cls = CLS_F64;     // storage class of the caller's A
    int64_t lda = 0, ldc = 0;
    int64_t a_plane = 0;         // LIMB2: element offset of the lo plane
    uint32_t alpha = 1, beta = 0;
    int32_t depth = -1;          // -1: tuned default
    bool fill_upper = false;
    bool force_f64 = false;
    bool force_limb3 = false;    // base products on three int8 limbs (p < 2^23, depth 0)
    bool a_aligned16 = true;     // caller's A pointer is 16-byte aligned
    bool c_aligned16 = true;
    // Table 3 with independent siblings: S1, S2 always in the workspace,
    // P2 into a workspace block, no workspace reuse between siblings, so
    // that P2 and the recursive calls P5, P1 with P3 have no memory in common
    // and the level scheduler runs them together (more workspace).
    bool wide = false;
    int32_t tile = 0;            // product tile edge (0: launch rule)
    bool no_tune = false;        // ignore the tuning table
};

struct Plan {
    FieldPlan field;
    int32_t cls = CLS_F64;       // base path class
    int32_t depth = 0;
    bool wide = false;           // placements used (see PlanRequest::wide)
    int32_t tile = 0;            // product tile edge for its launches (0: rule)
    bool tuned = false;          // depth and placements came from the tuning table
    int64_t n_pad = 0, k_pad = 0;
    int64_t ws_bytes = 0;
    std::vector<Op> ops;
};

// Validates fsyrk_modp arguments and fills a request (FFP_* status).
int make_syrk_request(int64_t n, int64_t k, uint32_t p, const void* A, int64_t lda, int a_dtype,
                      uint32_t alpha, uint32_t beta, const uint32_t* C, int64_t ldc, unsigned flags,
                      PlanRequest* rq);

// Returns FFP_* status (0 on success).
int build_syrk_plan(const PlanRequest& rq, Plan* out);
// Process-wide default of PlanRequest::wide for fsyrk_modp (tuning knob;
// 1 by default).
extern int g_wide_schedule;
// General products (P3, P4) of the FP64 class with wide placements and
// beta = 0 whose m, n and k are all at least this run one level of
// Strassen-Winograd (Algorithm 1): 7 half-size products instead of 8
// (0, the default: never; on the depth-3 8192 workload the additions and
// the smaller launches cost more than the eighth of the products saved).
extern int64_t g_winograd_min;
int choose_class(uint32_t p, int a_cls, bool force_f64, bool force_limb3 = false);
int default_depth(int cls, int64_t n, int64_t k);
std::string describe_plan(const Plan& pl);

}  // namespace ffp
