// Device kernels of the product library and their host launchers.
//
// Operand classes (storage of A and of the pre-added blocks S1..S4):
//   CLS_F64   uint32 residues in [0,p); products run on FP64 matrix cores
//             (v_mfma_f64_16x16x4f64) on centered values, delayed reduction.
//   CLS_I8    int8 centered residues, p <= 251; int8 matrix cores with int32
//             accumulation (v_mfma_i32_32x32x32_i8).
//   CLS_LIMB2 two int8 planes, value 256*hi + lo in [-32896, 32639],
//             p <= 65521; four limb products per tile, int32 accumulation.
// Products and every block of C are uint32 residues in [0,p).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffp {

// Storage classes of product operands: FP64 path (uint32 residues,
// converted in the kernel), centred int8, two int8 limbs (256 hi + lo),
// three int8 limbs (lo + 256 mid + 65536 hi; p < 2^23, depth 0 only).
enum Cls : int32_t { CLS_F64 = 0, CLS_I8 = 1, CLS_LIMB2 = 2, CLS_LIMB3 = 3 };
constexpr int kNumCls = 4;
// int8 planes of a class's storage
constexpr int cls_planes(int cls) { return cls == CLS_LIMB2 ? 2 : (cls == CLS_LIMB3 ? 3 : 1); }

// Field constants passed to every kernel.
struct Fp {
    uint32_t p;
    uint32_t half;   // (p-1)/2
    double pinv;     // 1/p
    uint32_t ya, yb; // skew-orthogonal Y = [[ya I, yb I], [-yb I, ya I]]
};

// A strided matrix view: element (i, j) is at base + i*ld + j; for limb
// classes plane q is at base + q*plane + i*ld + j (CLS_LIMB2: hi, lo;
// CLS_LIMB3: lo, mid, hi).  Units are elements of the view's storage type.
struct DView {
    void* p;
    int64_t ld;
    int64_t plane;
};

// ---- products --------------------------------------------------------
// One product C <- alpha * A * B^T + beta * C (kind GEMM) or
// lower(C) <- alpha * A * A^T + beta * lower(C) (kind SYRK), A m x k, B n x k.
struct ProdTask {
    DView A, B;
    uint32_t* C;
    int64_t ldc;
    int32_t m, n, k;
    int32_t syrk;
    uint32_t p, alpha, beta, half;
    double pinv;
    int32_t kblk;     // delayed-reduction block length (FP64 class)
    int32_t tm, tn;   // tile grid (rows, cols)
    int32_t tile0;    // first global tile index
};

// Operand forms of the 64 x 64 FP64 tile body (prod_f64_tile.h).
// C = alpha A B^T + beta C (A m x k, B n x k, row-major) in the plain form; the triangular forms skip the k-range where
// a triangular operand is zero (its zero entries inside the diagonal 64 x 64
// blocks must be stored; blocks above them are never read):
//   TILE_NT_BLOW  B lower triangular (B[c][t] = 0 for t > c)
//   TILE_NN_BLOW  C = alpha A B + beta C with B k x n row-major, lower
//                 triangular (B[t][c] = 0 for t < c)
//   TILE_NN_ALOW  C = alpha A B + beta C with A lower triangular
//                 (A[r][t] = 0 for t > r), B k x n row-major
enum TileForm : int { TILE_NT = 0, TILE_NT_BLOW = 1, TILE_NN_BLOW = 2, TILE_NN_ALOW = 3 };

constexpr int kInlineTasks = 6;
struct ProdArgs {
    int32_t ntasks;
    int32_t total_tiles;
    const ProdTask* dev_tasks;       // used when ntasks > kInlineTasks
    ProdTask inl[kInlineTasks];
};

// Tile shapes of the product kernels (output rows x cols per workgroup).
constexpr int kF64TileM = 64, kF64TileN = 64;
constexpr int kI8TileM = 256, kI8TileN = 256;
constexpr int kL2TileM = 128, kL2TileN = 128;

int64_t f64_kblk(uint32_t p);   // largest safe delayed-reduction block (multiple of 16)

// Fill the tile grid and k-block of a task run tile by tile by another
// kernel (the LDL^T step kernel): 64 x 64 FP64 tiles with operands from
// global memory, or 64 x 64 three-limb int8 tiles.  false: the task needs
// the regular launch (operand layout, or k beyond one exact block).
bool prepare_f64_tile_task(ProdTask* t);
bool prepare_limb3_tile_task(ProdTask* t);

// Test cap on the delayed-reduction block (0: none).
extern int64_t g_kblk_cap;
// Tile-variant overrides for tests and tuning (0: automatic).
extern int g_f64_tile_override;
extern int g_i8_tile_override;
extern int g_i8_bk_override;
extern int g_f64_pipe;         // FP64 128x128, 8 waves: operands as doubles in LDS (when k fits one exact block)
// Tile edge chosen for the product launches of the current call on this
// thread (0: the launch rule or the override above); set from the tuned
// choice of the call's plan.
extern thread_local int g_tile_hint;
extern int g_i8_dma;           // CLS_I8 256x256 / CLS_LIMB2 128x128, k a multiple of 128: operands
                               // straight to LDS (1, default)
// Scratch the int8 launcher may use for the k-chunks of a split tile round
// (set for one call by the executor; null: no split).
struct TailScratch {
    void* ptr;
    size_t bytes;
};
extern thread_local TailScratch g_tail_scratch;
extern int g_l3_dma;           // CLS_LIMB3 128 x 64 tiles straight to LDS: 1 (default) for large
                               // products, 2 whenever k is a multiple of 128, 0 never
struct TailScratchScope {
    TailScratch saved;
    TailScratchScope(void* p, size_t b) : saved(g_tail_scratch) { g_tail_scratch = TailScratch{p, b}; }
    ~TailScratchScope() { g_tail_scratch = saved; }
};
// 1 (default): a single-task int8 launch whose last round of tiles would
// leave most workgroups idle splits that round's tiles along k.
extern int g_split_tail;
extern int g_i8_pipe;          // CLS_I8 256x256x128: LDS writes spread over the MFMAs, loads two stages ahead
// Multi-task product launches run persistent workgroups (1, default) or one
// workgroup per tile (0).
extern int g_persistent;
// Product-kernel variant chosen by the most recent launch on this thread
// (for the timing hooks): 0 FP64 64x64, 1 unused, 2 int8
// 128x128, 3 int8 256x256 (k stage 64), 4 int8 256x256 (k stage 128), 5 int8
// limbs, 6 int8 256x256 straight to LDS, 7 limbs 128x128 straight to LDS, 8 FP64
// 128x128 LDS (8 waves), 9 int8
// three limbs, 10 int8 256x256 register-staged, 11 FP64 doubles in LDS, 12 limbs
// register-staged, 13 int8 256x256 straight to LDS with the last round's tiles
// split along k, 14 three limbs 128x64 straight to LDS.
extern thread_local int g_last_variant;
// Called by a launcher after the kernel whose time the current timing bracket
// measures when a small follow-up kernel of the same launch comes next: the
// bracket then ends there (no effect when timing is off).
void prof_mark_end(hipStream_t s);
// Workgroups of `kernel` (256 threads) resident at once on the device.
int resident_blocks(const void* kernel, int threads = 256);
inline int32_t cap_kblk(int64_t kb, int64_t unit)
{
    if (g_kblk_cap > 0 && g_kblk_cap < kb) kb = g_kblk_cap - g_kblk_cap % unit;
    if (kb < unit) kb = unit;
    return (int32_t)kb;
}


// ---- block additions (Algorithm 2, Tables 3 and 4) ---------------------
// S1 = (A21 - A11) Y, S2 = A22 - A21 Y on m x h blocks.
hipError_t launch_preadd_s1s2(int cls, const Fp& f, int64_t m, int64_t h, DView A11, DView A21,
                              DView A22, DView S1, DView S2, hipStream_t s);
// mode 1: S3 = S1 - A22 written to S3;  mode 2: S4 = S3 + A12 written to S4;
// mode 3: both (S3 from S1, then S4 from that S3).  In-place aliasing of the
// destination with the source block is allowed.
hipError_t launch_preadd_s34(int cls, const Fp& f, int mode, int64_t m, int64_t h, DView S1,
                             DView A22, DView A12, DView S3, DView S4, hipStream_t s);
// Fused U1 = P1 + P5, U2 = U1 + P4, U4 = U2 + P3 -> C21 (all of it) and
// U5 = U2 + P4^T (+ beta * C22_in) -> lower(C22).  P1, P5 lower triangles;
// P4T = P4^T full (stored in C22, overwritten); P3 full (stored in C21,
// overwritten).  When beta != 0, the strictly lower part of the input C22
// is read transposed from the upper triangle of `up_c11` and its diagonal
// from `dvec`.
hipError_t launch_postadd(const Fp& f, int64_t m, const uint32_t* P1, int64_t ld1,
                          const uint32_t* P5, int64_t ld5, uint32_t* C22, int64_t ld22,
                          uint32_t* C21, int64_t ld21, uint32_t beta, const uint32_t* up_c11,
                          int64_t ldu, const uint32_t* dvec, hipStream_t s);
// lower(Z) = lower(X) + lower(Y) (Z may alias X or Y).
hipError_t launch_add_lower(const Fp& f, int64_t m, const uint32_t* X, int64_t ldx,
                            const uint32_t* Y, int64_t ldy, uint32_t* Z, int64_t ldz,
                            hipStream_t s);
// Up(C11) = Low(C22)^T strictly, dvec = diag(C22) (Table 4, with the
// diagonal kept in its own vector).
hipError_t launch_save_c22(int64_t m, const uint32_t* C22, int64_t ld22, uint32_t* C11,
                           int64_t ld11, uint32_t* dvec, hipStream_t s);
// Up(C) = Low(C)^T.
hipError_t launch_mirror_lower(int64_t n, uint32_t* C, int64_t ldc, hipStream_t s);
// Up(C) <- -Low(C)^T mod p (the imaginary part of a Hermitian matrix).
hipError_t launch_mirror_lower_neg(uint32_t p, int64_t n, uint32_t* C, int64_t ldc, hipStream_t s);
// out (m x k) <- sum_i coef[i] * op_i(in[i]) mod p, op_i the transpose when
// bit i of trans is set (in[i] then k x m); lower: only entries j <= i (m = k).
hipError_t launch_lct(const Fp& f, int64_t m, int64_t k, int nin, const DView* in, const uint32_t* coef,
                      unsigned trans, int lower, DView out, hipStream_t s);

// ---- representation changes ----------------------------------------
// Copy an n x k block of uint32 residues (or int8 / limb storage of class
// src_cls) into the storage of class dst_cls, zero-padding to n_pad x
// k_pad.  Source values must be valid residues of their storage.
hipError_t launch_pack(const Fp& f, int src_cls, DView src, int64_t n, int64_t k, int dst_cls,
                       DView dst, int64_t n_pad, int64_t k_pad, hipStream_t s);
// Grouped pack of many matrices in one launch (batched jobs).  Descriptors
// are staged in host memory that stays valid until the copy to dev_descs
// has executed; block0 is filled in by the launcher.
struct PackDesc {
    DView src, dst;
    int64_t n, k, n_pad, k_pad;
    uint32_t p;
    double pinv;
    int32_t block0;
};
// 1 (default): representation changes from uint32 run 4 columns per thread
// when the destination allows aligned 4-column stores; 0: one per thread.
extern int g_pack_vec;
hipError_t launch_pack_grouped(int src_cls, int dst_cls, PackDesc* descs, int nd,
                               PackDesc* dev_descs, hipStream_t s);
// out <- sum of +-in[i] (i < nin <= 5; bit i of neg: subtract) mod p over
// m x k uint32 blocks of residues in [0, p).
hipError_t launch_lincomb(const Fp& f, int64_t m, int64_t k, int nin, const DView* in, unsigned neg, DView out,
                          hipStream_t s);
// Copy the lower triangle (or all, if full) of an n x n uint32 block.
hipError_t launch_copy_u32(int64_t rows, int64_t cols, const uint32_t* src, int64_t lds,
                           uint32_t* dst, int64_t ldd, int lower_only, hipStream_t s);
// rows x cols pseudo-random residues mod p in operand storage dtype
// (FFP_U32, FFP_I8_CENTERED, FFP_I8_LIMB2 with the lo plane `plane` bytes
// after the hi plane).
hipError_t launch_fill_residues(int64_t rows, int64_t cols, void* dst, int64_t ld, int64_t plane, int dtype,
                                uint32_t p, uint64_t seed, hipStream_t s);

}  // namespace ffp
