/*
 * ffp.h -- exact symmetric products and LDL^T over a prime field on AMD
 * Instinct MI355X (gfx950).
 *
 * Implements the method of Dumas, Pernet and Sedoglavic, "On Fast
 * Multiplication of a Matrix by its Transpose" (ISSAC 2020,
 * arXiv:2001.04109): the 2x2-block recursion of Algorithm 2 with three
 * recursive symmetric products and two general products, through a
 * skew-orthogonal Y with Y*Y^T = -I (Section 3.1), scheduled with the
 * low-memory placements of Table 3 and Table 4 (Section 4.2), and its use
 * for the Schur-complement updates of an LDL^T factorisation with diagonal
 * scaling (Section 5, Algorithms 4 and 5).
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major; a leading dimension counts elements of the
 *     operand's storage type and is at least the number of columns.
 *   - Matrix pointers are device pointers owned by the caller.  The library
 *     never frees or retains them beyond the call's stream order.
 *   - Residues are uint32 values in [0, p) unless the storage type says
 *     otherwise.  p must be prime; which p each base path accepts is stated
 *     at FFP_U32 below.
 *   - Every call validates its arguments synchronously (negative status on
 *     error, nothing enqueued), then enqueues its kernels on `stream` (a
 *     hipStream_t; NULL is the null stream) and returns without waiting.
 *     Device-detected conditions are reported through device memory (the
 *     `info` argument of fldlt_modp).
 *   - The library owns its device workspace (grown on demand, one per
 *     device and stream) and is safe to call from several host threads on
 *     different streams.
 *
 * Results are exact: every entry equals the plain definition reduced mod p.
 */
#ifndef FFP_H
#define FFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define FFP_OK            0
#define FFP_EINVAL       (-1) /* negative size, leading dimension too small, NULL pointer */
#define FFP_EPRIME       (-2) /* p not prime, or outside the range of the chosen path */
#define FFP_EDTYPE       (-3) /* unknown operand storage, or storage not valid for p */
#define FFP_ENOMEM       (-4) /* device workspace could not be allocated */
#define FFP_EDEVICE      (-5) /* a HIP runtime call failed */
#define FFP_EUNSUPPORTED (-6) /* a valid request this library does not implement */
#define FFP_ECANCELED    (-7) /* a served request was cancelled before it ran */
#define FFP_ETIMEDOUT    (-8) /* a served request was still queued at its deadline */

/* ---- operand storage of A ------------------------------------------- */
/* uint32 residues in [0,p).  Any prime 2 <= p <= 94906249 is accepted (the
 * largest prime with p (p-1) < 2^53).  The base path is chosen from p:
 * 3 <= p <= 251 packs to centered int8 (int8 matrix cores, int32
 * accumulation); p <= 65521 packs to two int8 limbs; p = 2 and larger p run
 * on FP64 matrix cores with delayed reduction, exact while every partial sum
 * stays below 2^53 (for p >= 2^25 the accumulators are reduced after every
 * 4-column matrix-core step). */
#define FFP_U32          0
/* int8 residues in [-(p-1)/2, (p-1)/2]; requires 3 <= p <= 251. */
#define FFP_I8_CENTERED  1
/* Two int8 planes of the same shape and leading dimension: the value of an
 * entry is 256*hi + lo, and must lie in [-32896, 32639] and be congruent to
 * the residue.  `A` points to the hi plane; the lo plane starts at
 * (const int8_t*)A + n*lda.  Requires 3 <= p <= 65521. */
#define FFP_I8_LIMB2     2

/* ---- flags ----------------------------------------------------------- */
/* Mirror the lower triangle into the upper one after the product, so C
 * holds the full symmetric result.  Without it the strict upper triangle
 * of C is scratch space on return (Algorithm 2 only defines the lower
 * triangle, and Tables 3 and 4 use the upper triangle as temporary). */
#define FFP_FILL_UPPER    0x1u
/* Force d levels of Algorithm 2 (0 <= d <= 7) instead of the tuned depth. */
#define FFP_DEPTH(d)      (((((unsigned)(d)) & 0x7u) + 1u) << 4)
/* Run the base products on FP64 matrix cores even where an int8 path
 * exists for p (only for FFP_U32 operands). */
#define FFP_BASE_F64      0x100u
/* Keep the placements of Table 3 (beta = 0): the strict upper triangle of C
 * is the only temporary when k <= n, and sibling sub-products reuse one
 * workspace region.  Without this flag the products P2, P5, P1 and P3 of
 * every level get memory of their own (S1, S2 and P2 in workspace blocks),
 * so that they run together; that needs more workspace (see
 * ffp_workspace_bytes).  Results are identical. */
#define FFP_LOW_MEMORY    0x200u
/* Run the base products on three int8 limbs (value = l + 256 m + 65536 h of
 * the centred residue, nine int8 matrix-core products per block, exact
 * int32 sums) instead of FP64 matrix cores; FFP_U32 operands, p < 2^23.
 * Algorithm 2's blocks S1..S4 are then formed in the three limb planes.
 * The autotuner chooses it (at depth 0) where it is faster.
 * Not with FFP_BASE_F64 (FFP_EINVAL); other storage or p: FFP_EDTYPE. */
#define FFP_BASE_LIMB3    0x400u

/* lower(C) <- (alpha * A * A^T + beta * lower(C)) mod p.
 * Algorithm 2 (Ensure: the lower triangle of A*A^T) in the accumulate form
 * of Table 4.  alpha = 1, beta = 0 runs the Table 3 schedule; any other
 * pair runs the Table 4 schedule.
 *   n, k     A is n x k, C is n x n; n, k >= 0.
 *   p        prime modulus (see FFP_U32 / FFP_I8_* for the accepted range).
 *   A, lda   device pointer and leading dimension (elements of a_dtype).
 *   a_dtype  FFP_U32, FFP_I8_CENTERED or FFP_I8_LIMB2.
 *   alpha, beta  residues in [0,p).
 *   C, ldc   device pointer, ldc >= n.  Entries of lower(C) must be in
 *            [0,p) when beta != 0.
 *   flags    FFP_FILL_UPPER, FFP_DEPTH(d), FFP_BASE_F64, FFP_BASE_LIMB3,
 *            FFP_LOW_MEMORY.
 * Errors: FFP_EINVAL, FFP_EPRIME, FFP_EDTYPE, FFP_ENOMEM, FFP_EDEVICE. */
int fsyrk_modp(int64_t n, int64_t k, uint32_t p, const void* A, int64_t lda, int a_dtype,
               uint32_t alpha, uint32_t beta, uint32_t* C, int64_t ldc, unsigned flags,
               void* stream);

/* fsyrk_modp for callers that cannot allocate device memory: code under HIP
 * stream capture, serving loops and harnesses that forbid hipMalloc.  Same
 * arguments, result and errors as fsyrk_modp; it allocates no device or
 * pinned host memory.  Its workspace is a static device buffer of
 * ffp_noalloc_scratch_bytes() (64 MiB) that every device the library runs
 * on holds until the process ends; a shape whose workspace
 * (ffp_workspace_bytes) exceeds it is rejected with FFP_ENOMEM before
 * anything is enqueued.  Grouped product launches carry their task tables
 * in the kernel arguments (several launches where fsyrk_modp would make
 * one).  All calls on one device share that device's buffer, which keeps
 * the last call's contents: calls that may overlap on one device (other
 * streams, other threads) race and must be serialised by the caller. */
int fsyrk_modp_noalloc(int64_t n, int64_t k, uint32_t p, const void* A, int64_t lda, int a_dtype,
                       uint32_t alpha, uint32_t beta, uint32_t* C, int64_t ldc, unsigned flags,
                       void* stream);
size_t ffp_noalloc_scratch_bytes(void);

/* C <- (alpha * A * B^T + beta * C) mod p, the general products P3 and P4
 * of Algorithm 2 as a stand-alone call.  A is m x k, B is n x k, C is
 * m x n, all uint32 residues; p a prime with 2 <= p <= 94906249.  FP64
 * matrix cores with delayed reduction.  Errors: FFP_EINVAL, FFP_EPRIME,
 * FFP_EDEVICE. */
int fgemm_modp(int64_t m, int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda,
               const uint32_t* B, int64_t ldb, uint32_t alpha, uint32_t beta, uint32_t* C,
               int64_t ldc, void* stream);

/* In-place LDL^T factorisation without pivoting, S = L * D * L^T mod p
 * (the symmetric factorisation of Section 5, whose Schur-complement
 * updates C <- C - A*D*A^T run as Algorithm 5 followed by fsyrk_modp with
 * alpha = p-1, beta = 1).
 *   n        order of S, n >= 0;  p an odd prime <= 94906249.
 *   S, lds   device pointer; on entry the lower triangle holds the
 *            symmetric matrix (residues in [0,p)); on exit the strict lower
 *            triangle holds the unit lower triangular L and the diagonal
 *            holds D.  The strict upper triangle is scratch space.
 *   info     device pointer to one int64: 0 on success, or j >= 1 when the
 *            j-th pivot is zero (S has no generic rank profile); the
 *            contents of S are then unspecified.
 * Errors: FFP_EINVAL, FFP_EPRIME, FFP_ENOMEM, FFP_EDEVICE. */
int fldlt_modp(int64_t n, uint32_t p, uint32_t* S, int64_t lds, int64_t* info, void* stream);

/* Device workspace fldlt_modp needs for order n (bytes), for admission
 * control; 0 if p is not an odd prime <= 94906249. */
size_t ffp_ldlt_workspace_bytes(int64_t n, uint32_t p);

/* lower(C) <- (alpha * A * B * A^T + beta * lower(C)) mod p for B block
 * diagonal with scalar blocks and 2 x 2 blocks [[0, b], [b, 0]], b != 0:
 * the symmetric product with block diagonal scaling of Algorithm 6
 * (Section 5.2, odd characteristic).  Each 2 x 2 block is factored by
 * eq. (antidiagonal) into two scalar pivots b/2 and -b/2 on the columns
 * A_j + A_(j+1) and A_j - A_(j+1); the resulting diagonal scaling runs as
 * Algorithm 5 (square roots of residues, Algorithm 4 on pairs of
 * non-residues, one appended zero column when their count is odd) and the
 * product of the scaled matrix as fsyrk_modp (Algorithm 2).
 *   m, n     A is m x n, B is n x n, C is m x m; m, n >= 0.
 *   p        odd prime <= 94906249 (characteristic 2 is not built).
 *   A, lda   device uint32 residues, lda >= n.
 *   bdiag    device array of n residues: B_jj.
 *   boff     device array of n - 1 residues: B_(j,j+1) = B_(j+1,j); a
 *            nonzero entry makes (j, j+1) a 2 x 2 block, whose diagonal
 *            entries must then be zero.  May be NULL when n <= 1.
 *   alpha, beta  residues in [0,p); C, ldc as in fsyrk_modp.
 *   info     device pointer to one int64, or NULL: 0, or j >= 1 when
 *            column j - 1 starts a malformed block (blocks overlap, a 2 x 2
 *            block has a nonzero diagonal entry, an entry of B is not below
 *            p); C is then unspecified.
 *   flags    FFP_FILL_UPPER, FFP_DEPTH(d), FFP_BASE_F64, FFP_LOW_MEMORY.
 * Errors: FFP_EINVAL, FFP_EPRIME (also p = 2), FFP_ENOMEM, FFP_EDEVICE. */
int fsyrkbd_modp(int64_t m, int64_t n, uint32_t p, const uint32_t* A, int64_t lda, const uint32_t* bdiag,
                 const uint32_t* boff, uint32_t alpha, uint32_t beta, uint32_t* C, int64_t ldc, int64_t* info,
                 unsigned flags, void* stream);

/* lower(C) <- A * A^T over F_p[i] = F_p[x]/(x^2 + 1) (the field F_(p^2)
 * when p = 3 mod 4): the symmetric product of Section 3.1 ("over the
 * complex field"), Algorithm 2 with Y = i I, whose multiplication only
 * exchanges the two planes with one sign change.  Its general products run
 * as three real products each (the 3M method) and its leaves as two (the
 * 2M method of Section 4.1), on FP64 matrix cores.
 *   n, k     A is n x k, C is n x n; n, k >= 0.
 *   p        odd prime <= 94906249.
 *   A, lda   device uint32 residues: real parts at A, imaginary parts at
 *            A + a_plane (elements, same lda); the planes must not overlap.
 *   C, ldc   likewise with c_plane.  The strict upper triangle of both
 *            planes is scratch unless FFP_FILL_UPPER mirrors it.
 *   flags    FFP_FILL_UPPER, FFP_DEPTH(d).
 * Errors: FFP_EINVAL, FFP_EPRIME (also p = 2), FFP_ENOMEM, FFP_EDEVICE. */
int fzsyrk_modp(int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda, int64_t a_plane, uint32_t* C,
                int64_t ldc, int64_t c_plane, unsigned flags, void* stream);

/* lower(C) <- A * A^H over F_p[i], conj(a + ib) = a - ib (Section 3.3):
 * Algorithm 2 with conjugate transposition and Y = (a + ib) I, where
 * a^2 + b^2 = -1 in F_p (Algorithm 3 for p = 3 mod 4; a = sqrt(-1), b = 0
 * for p = 1 mod 4), so that Y Y^H = -I.  The diagonal of C is real.  Same
 * arguments, flags and errors as fzsyrk_modp; FFP_FILL_UPPER writes the
 * conjugate of the lower triangle into the upper one. */
int fherk_modp(int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda, int64_t a_plane, uint32_t* C,
               int64_t ldc, int64_t c_plane, unsigned flags, void* stream);

/* One factorisation of fldlt_modp_batched (host struct; device pointers). */
typedef struct ffp_ldlt_job {
    int64_t n;
    uint32_t p;
    uint32_t* S;
    int64_t lds;
    int64_t* info;
} ffp_ldlt_job;

/* Runs njobs independent fldlt_modp factorisations together: the steps of
 * all recursions run level by level, each kind of step (leaf
 * factorisations, triangular solves, Algorithm 5, products) of all jobs as
 * one launch.  Each job must use its own S and info; results are
 * bit-identical to the jobs run one by one.  jobs is a host array.
 * Errors: as fldlt_modp, checked for every job before anything is
 * enqueued. */
int fldlt_modp_batched(int njobs, const ffp_ldlt_job* jobs, void* stream);

/* Device workspace fsyrk_modp needs for this shape (bytes), for admission
 * control; flags as for fsyrk_modp (beta != 0 is signalled by
 * FFP_WS_BETA). */
#define FFP_WS_BETA 0x80000000u
size_t ffp_workspace_bytes(int64_t n, int64_t k, uint32_t p, int a_dtype, unsigned flags);

/* ---- batched form ----------------------------------------------------- */
/* One independent fsyrk_modp job of a batch. */
typedef struct ffp_job {
    int64_t n, k;       /* A is n x k, C is n x n */
    uint32_t p;         /* prime, 2 <= p <= 94906249 */
    uint32_t alpha, beta;
    int32_t a_dtype;    /* FFP_U32 only, in this version */
    const void* A;      /* device pointer */
    int64_t lda;
    uint32_t* C;        /* device pointer */
    int64_t ldc;
} ffp_job;

/* Runs njobs independent products lower(C_j) <- alpha_j A_j A_j^T +
 * beta_j lower(C_j) mod p_j as grouped launches: jobs of the same base
 * path share one launch of the product kernel, with work ordered longest
 * first.  Each result is bit-identical to the job run alone by fsyrk_modp.
 * jobs is a host array; flags as for fsyrk_modp (applied to every job).
 * Errors: as fsyrk_modp, checked for every job before anything is
 * enqueued. */
int fsyrk_modp_batched(int njobs, const ffp_job* jobs, unsigned flags, void* stream);

/* ---- autotuner ------------------------------------------------------------ */
/* fsyrk_modp picks, for every call that does not force a depth, the
 * recursion depth of Algorithm 2 (its cut-off to the base products), the
 * placements (those of Tables 3 and 4, or the wide ones that give sibling
 * products memory of their own) and the product tile edge from a
 * process-wide tuning table, and falls back to a built-in rule for shapes
 * the table does not hold.  Entries cover a shape class: the base path
 * (FP64, int8, int8 limbs, from p and a_dtype), ceil(log2 n), ceil(log2 k),
 * the form ((alpha, beta) = (1, 0) or not) and FFP_LOW_MEMORY.  Batched
 * jobs consult the same table.  The LDL^T driver's Schur updates use the
 * built-in rule. */
typedef struct ffp_tune_result {
    int32_t depth;       /* levels of Algorithm 2 */
    int32_t tile;        /* product tile edge (0: the launch rule) */
    int32_t wide;        /* 1: wide placements, 0: those of Tables 3 and 4 */
    int32_t base;        /* 0: the base path of p; 3: three int8 limbs (FFP_BASE_LIMB3) */
    int32_t candidates;  /* configurations timed */
    double ms;           /* time of one call with the choice (at tuning) */
    double rule_ms;      /* time of one call with the built-in rule */
} ffp_tune_result;

/* Times fsyrk_modp on synthetic operands of shape n x k (storage a_dtype,
 * form alpha/beta, flags without FFP_DEPTH) for each candidate depth, tile
 * edge and placement (and, for FP64-path shapes with p < 2^23, the
 * three-limb base path), stores the fastest in the table for the shape
 * class and returns it.  Allocates its operands, runs on `stream` and waits for
 * it (a tuning call, not for the hot path).
 * Errors: FFP_EINVAL (n or k <= 0, FFP_DEPTH given), as fsyrk_modp
 * otherwise. */
int ffp_autotune(int64_t n, int64_t k, uint32_t p, int a_dtype, uint32_t alpha, uint32_t beta, unsigned flags,
                 void* stream, ffp_tune_result* out);
/* The depth, tile and placement a call of this shape would use now (host
 * only).  Returns 1 if they come from the table, 0 for the built-in rule,
 * or a negative FFP_* status. */
int ffp_tune_lookup(int64_t n, int64_t k, uint32_t p, int a_dtype, uint32_t alpha, uint32_t beta, unsigned flags,
                    ffp_tune_result* out);
/* Text form of the table (one shape class per line).  ffp_tune_load adds
 * the entries of a file written by ffp_tune_save and returns their number;
 * a malformed file changes nothing and gives FFP_EINVAL. */
int ffp_tune_save(const char* path);
int ffp_tune_load(const char* path);
void ffp_tune_clear(void);
int ffp_tune_entries(void);

/* ---- batched calls as HIP graphs ----------------------------------------- */
/* A batch recorded once and replayed: the host work of a batched call
 * (schedules of Algorithm 2 or of the LDL^T recursion, level grouping, task
 * tables) is done once, and each replay is one hipGraphLaunch of the
 * recorded kernels and table copies.  The graph owns the workspace and the
 * table buffers of the batch (ffp_graph_device_bytes), allocated before the
 * capture begins; nothing is allocated during the capture or a replay.
 *
 * Recording enqueues nothing: `stream` (not the null stream) is captured
 * and only serves to record.  A replay reads the jobs' operands at the
 * recorded addresses and writes the recorded outputs, so the caller keeps
 * those buffers alive and fills the inputs before each replay (an LDL^T
 * replay factors S in place again).  Replays of one graph share its
 * workspace and must not overlap: enqueue them on one stream, or order them
 * with events.  Results of every replay are bit-identical to the eager
 * batched call on the same inputs.
 * Errors: as fsyrk_modp_batched / fldlt_modp_batched; FFP_EINVAL for a null
 * stream or out pointer; FFP_EDEVICE if the capture or instantiation fails. */
typedef struct ffp_graph_s* ffp_graph;
int ffp_graph_syrk_batched(int njobs, const ffp_job* jobs, unsigned flags, void* stream, ffp_graph* out);
int ffp_graph_ldlt_batched(int njobs, const ffp_ldlt_job* jobs, void* stream, ffp_graph* out);
/* Enqueues one replay on stream (any stream of the recording device). */
int ffp_graph_launch(ffp_graph g, void* stream);
/* Device memory the graph owns (workspace and tables). */
size_t ffp_graph_device_bytes(ffp_graph g);
/* Nodes of the recorded graph (kernels and copies); 0 for an empty batch. */
size_t ffp_graph_nodes(ffp_graph g);
/* Frees the graph and its buffers; no replay may still be pending. */
void ffp_graph_destroy(ffp_graph g);

/* ---- request loop: continuous batching ---------------------------------- */
/* A server owns a pool of HIP streams (default priority) and one device
 * arena of hbm_budget bytes that holds every result and every running job's
 * workspace.  A scheduler thread admits queued requests in arrival order
 * while their footprint (result buffer plus workspace) fits in the arena and
 * fewer than max_inflight requests are running; a job's workspace returns to
 * the arena when the job is done, its result when the caller releases it.
 * Every scheduler iteration turns the requests admitted for a free stream
 * into one unit: its A*A^T requests as one fsyrk_modp_batched launch, then
 * its LDL^T requests as one fldlt_modp_batched run; requests that arrive
 * while units run join the next unit, so their work overlaps on the device.
 * Each result is bit-identical to the same job run alone.  Operands are
 * caller-owned device memory that must stay valid and unchanged until the
 * request is done. */
#define FFP_REQ_SYRK 0      /* C = alpha * A * A^T mod p (lower triangle) */
#define FFP_REQ_LDLT 1      /* L D L^T of the symmetric matrix whose lower triangle is A */
#define FFP_STATE_QUEUED  0
#define FFP_STATE_RUNNING 1
#define FFP_STATE_DONE    2

typedef struct ffp_request {
    int32_t kind;          /* FFP_REQ_SYRK or FFP_REQ_LDLT */
    int64_t n, k;          /* SYRK: A is n x k; LDLT: A is n x n and k is ignored */
    uint32_t p;            /* prime, 2 <= p <= 94906249 (LDLT: odd) */
    uint32_t alpha;        /* SYRK scale, residue in [0,p) */
    const void* A;         /* device pointer, uint32 residues (FFP_U32 storage) */
    int64_t lda;
    double timeout_s;      /* > 0: the request fails with FFP_ETIMEDOUT if it has not
                              been admitted this many seconds after submission; 0: none */
} ffp_request;

typedef struct ffp_result {
    int32_t state;         /* FFP_STATE_* or a negative FFP_* status */
    uint32_t* C;           /* device result, valid from FFP_STATE_DONE until released:
                              SYRK: lower triangle of C; LDLT: strict lower L, diagonal D */
    int64_t ldc;
    int64_t* info;         /* LDLT: device pointer to the first zero pivot (0: none) */
    double t_submit, t_admit, t_done;   /* seconds on a steady clock */
} ffp_result;

typedef struct ffp_serve_stats {
    int64_t submitted, completed, units, batched_jobs, max_batch;
    int64_t peak_inflight, overlapped_units;   /* units launched while others ran */
    size_t peak_bytes;
} ffp_serve_stats;

typedef struct ffp_server ffp_server;

/* nstreams in [1, 16]; max_inflight >= 1.  FFP_ENOMEM if the arena cannot be
 * allocated. */
int ffp_server_create(size_t hbm_budget, int max_inflight, int nstreams, ffp_server** out);
/* Queues a request (thread-safe, does not block on the device).  FFP_EINVAL
 * or FFP_EPRIME for a malformed request, FFP_ENOMEM if its footprint alone
 * exceeds the budget. */
int ffp_server_submit(ffp_server* s, const ffp_request* r, uint64_t* ticket);
int ffp_server_status(ffp_server* s, uint64_t ticket, ffp_result* out);
/* Returns a done request's result memory to the budget.  Copies that
 * ffp_server_fetch enqueued from it may still be pending on the caller's
 * stream: the memory then returns to the arena only once they have executed
 * (the fetch records an event after them), so a release never lets a later
 * request overwrite a result that is still being copied. */
int ffp_server_release(ffp_server* s, uint64_t ticket);
/* Cancels a request that is still queued: it becomes done with state
 * FFP_ECANCELED and holds no memory.  FFP_EINVAL if it has already been
 * admitted (running work is not interrupted) or is done. */
int ffp_server_cancel(ffp_server* s, uint64_t ticket);
/* Waits until every submitted request is done (FFP_EDEVICE on timeout). */
int ffp_server_drain(ffp_server* s, double timeout_s);
/* Completion queue: waits up to timeout_s seconds (0: no wait) until some
 * request has finished, then returns in tickets up to max finished requests
 * (failed ones included) not returned before, oldest first; *count is the
 * number returned (0 on timeout). */
int ffp_server_poll(ffp_server* s, uint64_t* tickets, int max, double timeout_s, int* count);
/* Enqueues on stream a copy of a done request's result into the caller's
 * device buffer dst (n x n, row stride ldd >= n; only the lower triangle is
 * meaningful) and, for LDLT when info_dst is not null, of its info word.
 * FFP_EINVAL if the request is not done, failed or was released. */
int ffp_server_fetch(ffp_server* s, uint64_t ticket, uint32_t* dst, int64_t ldd, int64_t* info_dst,
                     void* stream);
int ffp_server_stats(ffp_server* s, ffp_serve_stats* out);
int ffp_server_destroy(ffp_server* s);

/* Human-readable name of a status code. */
const char* ffp_strerror(int status);

/* Library version string. */
const char* ffp_version(void);

/* The HIP call behind the calling thread's most recent FFP_ENOMEM or
 * FFP_EDEVICE from the library, with its HIP error name ("" if none). */
const char* ffp_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* FFP_H */
