// LDL^T factorisation without pivoting (Section 5 of the paper): recursive
// split, unit-lower triangular solve, Algorithm 5 applied to the pivots and
// the Schur-complement update S22 <- S22 - Abar Abar^T through the Table 4
// schedule of fsyrk.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

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
    int32_t* flag;      // n1: pivot is a quadratic non-residue
    uint32_t* root;     // n1: square root of residue pivots
    uint32_t* dinv;     // n1: inverse pivots
    int32_t* rank_idx;  // n1: indices of the non-residues in order
    ColOp* desc;        // n1 + 1 column operations
};

// Leaf factorisation; also writes the inverse of the leaf's unit lower
// factor to linv (nb rows of stride kLdltLeaf), used by launch_trsm_leaf.
hipError_t launch_ldlt_leaf(const Fp& f, int nb, uint32_t* S, int64_t lds, int64_t* info,
                            int64_t offset, uint32_t* linv, hipStream_t s);
// X <- X L^-T for an nrows x nb block X, given linv = L^-1 of the unit lower
// nb x nb factor as written by launch_ldlt_leaf.
hipError_t launch_trsm_leaf(const Fp& f, int64_t nrows, int nb, uint32_t* X, int64_t ldx,
                            const uint32_t* linv, hipStream_t s);
hipError_t launch_alg5(const Fp& f, int n1, const uint32_t* S11, int64_t lds, uint32_t s_lqnr,
                       uint32_t c_lqnr, uint32_t z, Alg5Scratch sc, hipStream_t s);
hipError_t launch_scale_cols(const Fp& f, int64_t rows, int n1, uint32_t* W, int64_t ldw,
                             const uint32_t* dinv, hipStream_t s);
hipError_t launch_build_abar(const Fp& f, int64_t rows, int ncols, int kpad, const uint32_t* L,
                             int64_t ldl, const ColOp* desc, uint32_t* Ab, int64_t ldab,
                             hipStream_t s);
hipError_t launch_zero_i64(int64_t* p, hipStream_t s);

// Host driver.  Returns an FFP_* status; enqueues everything on s.
// ws: optional device workspace of ldlt_workspace_bytes(n, p, lds) bytes,
// 256-byte aligned; when null the library's per-stream workspace is used.
int ldlt_run(int64_t n, uint32_t p, uint32_t* S, int64_t lds, int64_t* info, hipStream_t s,
             void* ws = nullptr);
size_t ldlt_workspace_bytes(int64_t n, uint32_t p, int64_t lds);

}  // namespace ffp
