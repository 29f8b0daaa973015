/*
 * ffp_debug.h -- host-only introspection entry points of the ffp library.
 * None of these touches a device; they exist so that the host logic (the
 * field routines of Section 3.1 and the schedules of Tables 3 and 4) can be
 * checked without a GPU.
 */
#ifndef FFP_DEBUG_H
#define FFP_DEBUG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Skew-orthogonal Y = [[ya I, yb I], [-yb I, ya I]] chosen for p (Proposition
 * 3.3 when p = 1 mod 4; a = 1, b = sqrt(-2) when p = 3 mod 8; Algorithm 3
 * otherwise) and its cost y of Theorem 4.1.  FFP_EPRIME if p is not an odd
 * prime. */
int ffp_field_info(uint32_t p, uint32_t* ya, uint32_t* yb, int* ycost);

/* Canonical square root min(r, p-r) of a mod p; FFP_EINVAL if a is not a
 * square, FFP_EPRIME if p is not an odd prime. */
int ffp_host_sqrt(uint32_t a, uint32_t p, uint32_t* r);

/* Algorithm 3 (SoS): a^2 + b^2 = k mod p. */
int ffp_host_sos(uint32_t p, uint32_t k, uint32_t* a, uint32_t* b);

/* Algorithm 4 (nrsyf): Y (row-major 2x2) with Y Y^T = diag(alpha, beta) for
 * two quadratic non-residues; FFP_EINVAL if either is a residue. */
int ffp_host_nrsyf(uint32_t p, uint32_t alpha, uint32_t beta, uint32_t Y[4]);

/* Text description of the schedule fsyrk_modp would run for these
 * arguments (device pointers are taken as 16-byte aligned).  Writes at most
 * len bytes (NUL-terminated) to buf and returns the full length, or a
 * negative FFP_* status.  Format: a header line
 *   "plan cls=<c> depth=<d> n_pad=<n> k_pad=<k> ws=<bytes> ya=<a> yb=<b>"
 * then one line per operation:
 *   "op kind cls src_cls mode m n k m_src k_src alpha beta level" followed
 *   by six views "buf off ld plane" (buf 0 = A, 1 = C, 2 = workspace; off in
 *   bytes, ld and plane in elements of the view's storage) and the five
 *   coefficients of a linear combination (1 for other operations). */
int ffp_plan_describe(int64_t n, int64_t k, uint32_t p, int a_dtype, int64_t lda, int64_t ldc,
                      uint32_t alpha, uint32_t beta, unsigned flags, char* buf, size_t len);
/* Same for the schedule of fzsyrk_modp (herk = 0) or fherk_modp (herk = 1);
 * the op lines end with the five coefficients of the linear combinations. */
int ffp_complex_plan_describe(int64_t n, int64_t k, uint32_t p, int herk, int64_t lda, int64_t a_plane,
                              int64_t ldc, int64_t c_plane, unsigned flags, char* buf, size_t len);
/* Scheduler levels of that complex schedule's operations (as
 * ffp_plan_levels). */
int ffp_complex_plan_levels(int64_t n, int64_t k, uint32_t p, int herk, int64_t lda, int64_t a_plane,
                            int64_t ldc, int64_t c_plane, unsigned flags, int32_t* levels, size_t cap);

/* Level of every operation of the same plan (as ffp_plan_describe lists
 * them) under the library's level scheduler: an operation's level is one
 * more than the highest level of the earlier operations it depends on.
 * Writes min(count, cap) levels; returns the number of operations or a
 * negative FFP_* status.  Host only. */
int ffp_plan_levels(int64_t n, int64_t k, uint32_t p, int a_dtype, int64_t lda, int64_t ldc,
                    uint32_t alpha, uint32_t beta, unsigned flags, int32_t* levels, size_t cap);

/* Test hook: cap the delayed-reduction block of the product kernels at kblk
 * columns of k (rounded down to the kernel's k granularity; 0 restores the
 * largest exact block).  Process-wide; affects launches made after the
 * call.  Results stay exact for any cap: it only adds reductions. */
void ffp_debug_set_kblk(int64_t kblk);

/* Tuning and test knobs (process-wide): "kblk" (as ffp_debug_set_kblk),
 * "f64_tile" (64 or 128: force the FP64 product tile; 0 = automatic),
 * "serve_batch" and "serve_ldlt_batch" (1 to
 * 4096: A*A^T and LDL^T requests per unit of the request loop; 128 and 32
 * by default), "ldlt_fold" (1, the default: the LDL^T products run as steps
 * of the per-level launch; 0: as separate product launches),
 * "i8_tile" (128 or 256: force the int8 product tile; 0 = automatic),
 * "i8_bk" (64 or 128: k bytes per LDS stage of the 256 x 256 int8 tile),
 * "i8_dma" (1, the default: the 256 x 256 int8 tile and the 128 x 128
 * two-limb tile with 128-byte k stages load their operands straight into
 * LDS, no staging registers; 0: through registers as "i8_pipe" says),
 * "i8_split_tail" (1, the default: an fsyrk_modp int8 product launch whose
 * last round of 256 x 256 tiles would leave most workgroups idle runs that
 * round's tiles as k-chunks and adds them in a second small kernel; 0: no
 * split), "l3_dma" (1, the default: three-limb products of at least four
 * rounds of 128 x 64 tiles with k >= 1024 a multiple of 128 run those tiles
 * with operands straight to LDS; 2: whenever k is a multiple of 128; 0:
 * always the 64 x 64 tile), "i8_pipe" (1, the default: with "i8_dma" 0,
 * the 256 x 256 int8 tile with 128-byte k stages writes each stage's
 * operands to LDS between the MFMAs of the previous stage and loads them up
 * to two stages ahead; 0: the stage's LDS writes after its MFMAs), "f64_pipe" (1, the default: the
 * 128 x 128 FP64 tile of 8 waves keeps its operands as doubles in LDS,
 * converted once per workgroup, when k fits one exact block; 0: centred
 * int32 in LDS, converted by every wave that reads them),
 * "persistent" (2, the default: grouped product launches run persistent
 * workgroups; the register-staged int8 and limb tiles are dealt to the 8
 * XCDs in chunks of 8 neighbouring tiles; 1: persistent workgroups striding
 * over the tiles; 0: one workgroup per tile), "winograd_min" (n:
 * general products P3, P4 of the FP64 class with wide placements, beta = 0
 * and m, n, k >= n run one level of Strassen-Winograd, Algorithm 1, with its
 * additions as separate operations; 0, the default: never), "merge_tiles"
 * (size in 128 x 128 tiles under which a level's product launch counts as
 * small for "merge_products"; 512 by default), "pack_vec" (1, the
 * default: representation changes from uint32 residues convert 4 columns
 * per thread, 16 x 256 per workgroup, when the destination keeps those
 * stores aligned, and the FP64-class pre-additions run 4 columns per thread
 * when their rows are 16-byte aligned; 0: one element per thread),
 * "merge_products" (1,
 * the default: after the as-soon-as-possible levels are set, a product whose
 * grouped launch would be small moves to a later level with a larger
 * launch of its class when its dependents allow; 0: off), "leveled" (1, the
 * default: a call's block operations run level by level, independent
 * products of a level as one grouped launch; 0: one by one in schedule
 * order), "wide" (1, the default: Algorithm 2 keeps S1, S2 and P2 in
 * workspace blocks of their own, so that P2, P5, P1 and P3 are independent
 * and share levels; more workspace; 0: the placements of Table 3).
 * FFP_EINVAL for an unknown key. */
int ffp_debug_set(const char* key, int64_t value);

/* Timing hook for benchmarks: while enabled, every product-kernel launch is
 * bracketed by two HIP events on its stream.  ffp_debug_profile_read waits
 * for the recorded launches of base-path class cls (0 = FP64, 1 = int8,
 * 2 = two int8 limbs, 3 = three int8 limbs, -1 = all), returns the sum of their durations (ms), of
 * their algorithmic flops (2 m n k for a general product, n (n+1) k for a
 * lower-triangle product) and their count, and forgets them. */
void ffp_debug_profile(int enable);
int ffp_debug_profile_read(int cls, double* ms, double* flops, int64_t* launches);
/* Same, restricted to one product-kernel variant (0 FP64 64x64 tiles,
 * 1 unused, 2 int8 128x128, 3 int8 256x256 with 64-byte k stages, 4 int8
 * 256x256 with 128-byte k stages, 5 int8 limbs 128x128, 6 int8 256x256
 * with operands straight to LDS, 7 int8 limbs 128x128 straight to LDS,
 * 8 FP64 128x128 with centred int32 in LDS, 9 int8 three limbs 64x64,
 * 10 int8 256x256 with the LDS writes between the MFMAs, 11 FP64 128x128
 * with doubles in LDS, 12 int8 limbs 128x128 register-staged, 13 int8
 * 256x256 straight to LDS with the last round of tiles split along k; its
 * time excludes the small kernel that adds the split tiles' chunks, 14 int8
 * three limbs 128x64 straight to LDS);
 * ffp_debug_variant_name gives the kernel's demangled name. */
int ffp_debug_profile_read_variant(int variant, double* ms, double* flops, int64_t* launches);
const char* ffp_debug_variant_name(int variant);

/* A server whose device is simulated on the host: units of work complete
 * after launch_us + ns_per_op * (n^2 k, or n^3 / 3 for LDL^T) nanoseconds and
 * compute nothing; it exercises the scheduler (admission, batching,
 * overlap) without a GPU.  Results are not produced (C is NULL). */
int ffp_server_create_simulated(size_t budget, int max_inflight, int nstreams, double ns_per_op,
                                double launch_us, ffp_server** out);

#ifdef __cplusplus
}
#endif

#endif /* FFP_DEBUG_H */
