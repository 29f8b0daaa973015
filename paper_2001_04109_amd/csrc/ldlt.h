// LDL^T factorisation without pivoting (Section 5 of the paper): recursive
// split, unit-lower triangular solve through inverses of the leading unit
// factors, Algorithm 5 applied to the pivots and the Schur-complement update
// S22 <- S22 - Abar Abar^T through the Table 4 schedule of fsyrk.
//
// The host flattens the recursion of every factorisation into a sequence of
// steps; the steps of several factorisations run together, level by level,
// each level as one launch over an array of descriptors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "kernels.h"

namespace ffp {

constexpr int kLdltLeaf = 64;

// One column of Abar as a combination of at most two columns of L21.
struct ColOp {
    int32_t j1;
    uint32_t s1;
    int32_t j2;
    uint32_t s2;
};

struct Alg5Scratch {
    int32_t* flag;      // per pivot: quadratic non-residue
    uint32_t* root;     // per pivot: square root (LDL^T: of D / s for a non-residue)
    uint32_t* dinv;     // per pivot: inverse
    int32_t* rank_idx;  // indices of the non-residues in order (fsyrkbd_modp)
    ColOp* desc;        // n1 + 1 column operations (fsyrkbd_modp)
};

// Device step kinds.
enum LdltKind : int32_t {
    LK_ZERO = 0,     // *info = 0
    LK_LEAF,         // leaf factorisation of the nb x nb block at X; inverse of its unit factor
    LK_ROOTS,        // Algorithm 5 per pivot of a factored leaf: flag, root, inverse
    LK_CLASSIFY,     // Algorithm 5, per pivot of X (nb pivots, stride ldx + 1): flag, root, inverse
    LK_PAIR,         // Algorithm 5: rank the non-residues, Algorithm 4 per pair, column ops
    LK_ABARX,        // Algorithm 5 on a node's pivots: L21 = W D1^-1 and Abar from W in one pass
    LK_PRODF,        // product task t, 64 x 64 FP64 tiles (operand form pform)
    LK_PRODL3,       // product task t, 64 x 64 three-limb int8 tiles
    LK_BDIAG,        // Algorithm 6 (odd p): column ops desc1 and diagonal dbar of a block diagonal B
    LK_ABAR2,        // Abar (rows x kpad) from the column ops desc (on A desc1) on A = X
    LK_KINDS
};

// Descriptor of one device step (read by the kernels from device memory).
struct LdltDesc {
    int32_t kind;      // LK_*
    Fp f;
    int32_t kb;        // residue products per FP64 partial sum
    int32_t nb;        // leaf order; Algorithm 5: number of pivots n1
    int64_t rows;      // LK_ABARX, LK_ABAR2: rows of W / A
    int32_t ncols, kpad;
    int32_t block0;    // first workgroup of this descriptor in its launch
    int32_t gx;        // column blocks (LK_ABARX, LK_ABAR2)
    uint32_t* X;
    int64_t ldx;
    int64_t* info;
    int64_t offset;    // leaf, LK_ABARX: index of its first pivot in the whole factorisation
    uint32_t* linv;    // leaf: inverse of its unit factor (ld ldi), or null
    int64_t ldi;
    Alg5Scratch sc;
    uint32_t s_lqnr, c_lqnr, s_inv;   // smallest non-residue s, sqrt(s - 1), 1/s
    uint32_t* Ab;
    int64_t ldab;
    uint32_t* Y;       // LK_ABARX: L21 (ldy)
    int64_t ldy;
    int32_t amode;     // LK_ABARX: 0 Abar as uint32, 1 as three int8 limb planes
    int32_t pform;     // LK_PRODF: operand form (TILE_* of prod_f64_tile.h)
    ProdTask t;        // LK_PRODF, LK_PRODL3
    // LK_ABARX with amode 1: limb planes of rows_pad x kpad at Ab, plane offset pplane
    int64_t rows_pad, pplane;
    // LK_BDIAG: B's diagonal bd (nb entries) and off-diagonal bo (nb - 1);
    // out: desc1 (nb column ops on A), dbar (nb pivots).  LK_ABAR2 reads desc1.
    const uint32_t* bd;
    const uint32_t* bo;
    ColOp* desc1;
    uint32_t* dbar;
};

// Workgroups a descriptor of the kind needs (sets d->gx where used).
int ldlt_blocks(int kind, LdltDesc* d);
// One launch over n descriptors of any kinds in device memory (block0 set,
// ascending): each workgroup runs the step of its descriptor's kind.
hipError_t launch_ldlt_steps(const LdltDesc* dev, int n, int total_blocks, hipStream_t s);
// Residue products whose sum stays below 2^53, at most 64.
int ldlt_dot_block(uint32_t p);
// 1 (default): three-limb Schur updates run as steps of the per-level
// launch (Abar written straight into limb planes); 0: through the product
// schedule's own launches.
extern int g_ldlt_fold;

struct LdltJobSpec {
    int64_t n;
    uint32_t p;
    uint32_t* S;
    int64_t lds;
    int64_t* info;
    void* ws;          // ldlt_workspace_bytes(n, p, lds) bytes, 256-byte aligned
};

// Host driver.  Returns an FFP_* status; enqueues everything on s.
// ws: optional device workspace of ldlt_workspace_bytes(n, p, lds) bytes,
// 256-byte aligned; when null the library's per-stream workspace is used.
int ldlt_run(int64_t n, uint32_t p, uint32_t* S, int64_t lds, int64_t* info, hipStream_t s,
             void* ws = nullptr);
// Several independent factorisations (disjoint S, info and workspaces)
// enqueued together on s.
int ldlt_run_multi(const std::vector<LdltJobSpec>& jobs, hipStream_t s);
size_t ldlt_workspace_bytes(int64_t n, uint32_t p, int64_t lds);

// fsyrkbd_modp (Algorithm 6, odd p): lower(C) <- alpha A B A^T + beta lower(C)
// for A m x n and B block diagonal (diagonal bd, off-diagonal bo, both device
// arrays).  rq: the product request for Abar (m x kpad) with Abar in the
// workspace; validated by the caller.  ws: syrkbd_workspace_bytes bytes.
struct PlanRequest;
int syrkbd_run(int64_t m, int64_t n, uint32_t p, const uint32_t* A, int64_t lda, const uint32_t* bd,
               const uint32_t* bo, const PlanRequest& rq, uint32_t* C, int64_t* info, void* ws,
               hipStream_t s);
// Columns of Abar (n + 1 rounded up to 128) and workspace of syrkbd_run.
int64_t syrkbd_kpad(int64_t n);
size_t syrkbd_workspace_bytes(int64_t m, int64_t n, const PlanRequest& rq);

}  // namespace ffp
