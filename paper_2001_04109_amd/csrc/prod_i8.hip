// Base-case products on int8 matrix cores (CDNA4 v_mfma_i32_32x32x32_i8).
//
// CLS_I8: centred int8 residues (|x| <= 125 for p <= 251); each product is
// at most 125^2 in magnitude, so an int32 accumulator is exact for more than
// 137 000 columns of k; longer products run as several launches over k
// chunks, each reducing mod p into C.
//
// CLS_LIMB2: value = 256*hi + lo with int8 limbs; the tile accumulates
// hh = Ahi Bhi^T, ll = Alo Blo^T and x = Ahi Blo^T + Alo Bhi^T in three
// int32 accumulators and combines 2^16 hh + 2^8 x + ll mod p in the
// epilogue.
//
// CLS_LIMB3: value = l + 256 m + 65536 h with int8 limbs (centred residues
// of p < 2^23: |h| <= 65); the nine limb products go to five int32
// accumulators by weight 2^0 (ll), 2^8 (lm + ml), 2^16 (lh + mm + hl),
// 2^24 (mh + hm), 2^32 (hh), each exact for 32768 columns of k (three
// products of at most 128^2 per column), and the epilogue combines them
// mod p.
//
// A 256-thread workgroup computes a BM x BN tile; each of its 4 waves a
// (BM/2) x (BN/2) sub-tile of 32 x 32 MFMA blocks.  Per stage of BK (64 or
// 128) columns of k the workgroup copies the A and B row panels (BM and BN
// rows of BK bytes) into one of two LDS buffers: every thread issues its global
// loads for stage t+1 into registers before the MFMAs of stage t and writes
// them to the other buffer afterwards, so HBM/L2 latency overlaps matrix
// work.  The LDS row pitch is padded by 16 bytes so that the 16-byte reads
// of 8 consecutive rows fall in distinct banks.
//
// Every lane feeds one MFMA with 16 consecutive k-bytes of one row; A and B
// use the same lane-to-k assignment, so the sum is exact whatever the
// instruction's internal k order.
//
// Tile order: tiles are enumerated in bands of G tile rows (column by column
// inside a band) so that the tiles in flight on one XCD share a few A and B
// panels in its L2; for single-task launches each XCD gets a contiguous range
// of that order (blocks are dispatched round-robin over the 8 XCDs).
#include "prod_i8_tile.h"

#include <type_traits>
#include <vector>

namespace ffp {

// Wrapper of i8_tile_task over a launch's task list.
template <int BM, int BN, int BK, int PLANES>
__device__ __forceinline__ void i8_tile(const ProdArgs& args, int b)
{
    __shared__ __attribute__((aligned(16))) int8_t smem[I8Tile<BM, BN, BK, PLANES>::LDS];
    ProdTask t;
    select_task(args, b, &t);
    // three limbs: short products (batches, served requests) wait on their
    // loads; a second register set issues them two stages ahead
    i8_tile_task<BM, BN, BK, PLANES, PLANES == 3>(t, b - t.tile0, smem);
}

// ---- CLS_I8 with the LDS writes spread over the MFMAs -------------------
//
// Same tile, wave decomposition, LDS layout and epilogue as
// i8_tile_task<BM, BN, BK, 1>, in a different order per stage of BK = 128
// bytes (four k-steps of 32): two register sets hold the operand panels of
// the next two stages, so the global loads issued at the start of stage t
// (for stage t + 2) have more than a stage to land; the set loaded one stage
// earlier is written to the free LDS buffer during k-steps 0 and 1 (A panel,
// half in each) and 2 (B panel) of stage t, between the MFMAs; the workgroup
// barrier sits before
// k-step 3, whose MFMAs cover the reads of the first fragments of stage t + 1.
// Stages are processed in pairs; the loads of stages past the end of k return
// zeros (see bload), so an odd count gets one stage of zero products.
// Panel loads through a buffer resource whose base is the panel's first row
// (raw buffer, size = the valid rows' bytes, below 2^31).  For a full panel
// the row offset of each pass is uniform and goes in the scalar offset, so a
// lane keeps one vector offset for all its loads; for a partial panel (EDGE)
// every load carries its own row offset and rows past the end fall outside
// the resource.  Buffer loads outside the resource return zero, and the
// outputs of rows past the end are never stored.  A stage past the end of k
// (`live` false) adds 2^31 to the vector offsets, so all its loads return
// zero and it adds nothing.
template <int ROWS, int BK, bool EDGE>
__device__ __forceinline__ void bload(Prefetch<ROWS, BK>& pf, __amdgpu_buffer_rsrc_t rs, int ld, int k0,
                                      bool live)
{
    constexpr int CHUNKS = Prefetch<ROWS, BK>::CHUNKS;
    constexpr int RPP = 256 / CHUNKS;                      // rows per pass
    const uint32_t off = live ? 0u : 0x80000000u;
    const int r0 = threadIdx.x / CHUNKS, c = threadIdx.x % CHUNKS;
    const uint32_t vbase = (uint32_t)(r0 * ld + c * 16) + off;
#pragma unroll
    for (int ps = 0; ps < Prefetch<ROWS, BK>::PASSES; ++ps) {
        if constexpr (EDGE) {
            pf.v[ps] = __builtin_amdgcn_raw_buffer_load_b128(rs, vbase + (uint32_t)(ps * RPP * ld),
                                                             __builtin_amdgcn_readfirstlane(k0), 0);
        } else {
            pf.v[ps] = __builtin_amdgcn_raw_buffer_load_b128(rs, vbase,
                                                             __builtin_amdgcn_readfirstlane(k0 + ps * RPP * ld), 0);
        }
    }
}

// The panel's values are the same in every lane; readfirstlane lets the
// compiler keep the resource in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(const int8_t* p, int64_t bytes)
{
    const uint64_t a = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const int nb = __builtin_amdgcn_readfirstlane((int)(bytes < 0x7FFFFFFF ? bytes : 0x7FFFFFFF));
    void* base = (void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
    // raw buffer (stride 0), 32-bit dword format word for CDNA
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nb, 0x00020000);
}

// Passes [P0, P1) of a staged panel to LDS (lstore's layout).
template <int ROWS, int BK, int P0, int P1>
__device__ __forceinline__ void lstore_part(int8_t* __restrict__ lds, const Prefetch<ROWS, BK>& pf)
{
    constexpr int CHUNKS = Prefetch<ROWS, BK>::CHUNKS;
#pragma unroll
    for (int ps = P0; ps < P1; ++ps) {
        const int idx = ps * 256 + threadIdx.x;
        const int r = idx / CHUNKS, c = idx % CHUNKS;
        *reinterpret_cast<v4i*>(lds + r * Prefetch<ROWS, BK>::PITCH + c * 16) = pf.v[ps];
    }
}

// PLANES = 1: centred int8 (one accumulator); 2: two int8 limbs (hh, ll and
// hl + lh accumulators, as in i8_tile_task).
template <int BM, int BN, int BK, int PLANES, bool EDGE>
__device__ __forceinline__ void i8_pipe_body(const ProdTask& t, int ti, int tj, int8_t* smem)
{
    constexpr int PITCH = BK + 16;
    constexpr int WTM = BM / 2, WTN = BN / 2;
    constexpr int FM = WTM / 32, FN = WTN / 32;
    constexpr int KS = BK / 32;
    constexpr int NACC = PLANES == 1 ? 1 : 3;
    static_assert(KS == 4, "four k-steps per stage");
    static_assert(PLANES == 1 || PLANES == 2, "one plane or two limbs");
    auto sa = reinterpret_cast<int8_t(*)[PLANES][BM * PITCH]>(smem);
    auto sb = reinterpret_cast<int8_t(*)[PLANES][BN * PITCH]>(smem + 2 * PLANES * BM * PITCH);
    const int tile_r = ti * BM, tile_c = tj * BN;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lrow = lane & 31, lk = lane >> 5;

    v16i acc[NACC][FM][FN];
#pragma unroll
    for (int q = 0; q < NACC; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[q][i][j][e] = 0;
    const bool wave_live = !(t.syrk && (tile_c + wc * WTN) > (tile_r + wr * WTM + WTM - 1));

    const int nk = t.k / BK;
    if (nk > 0) {
        auto read_frags = [&](v4i (&xa)[PLANES][FM], v4i (&xb)[PLANES][FN], int buf, int ks) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    xa[pl][i] = *reinterpret_cast<const v4i*>(
                        &sa[buf][pl][(wr * WTM + i * 32 + lrow) * PITCH + ks * 32 + lk * 16]);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    xb[pl][j] = *reinterpret_cast<const v4i*>(
                        &sb[buf][pl][(wc * WTN + j * 32 + lrow) * PITCH + ks * 32 + lk * 16]);
            }
        };
        auto mfmas = [&](const v4i (&xa)[PLANES][FM], const v4i (&xb)[PLANES][FN]) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if constexpr (PLANES == 1) {
                        acc[0][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[0][i], xb[0][j], acc[0][i][j], 0, 0, 0);
                    } else {
                        acc[0][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[0][i], xb[0][j], acc[0][i][j], 0, 0, 0);
                        acc[1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[1][i], xb[1][j], acc[1][i][j], 0, 0, 0);
                        acc[2][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[0][i], xb[1][j], acc[2][i][j], 0, 0, 0);
                        acc[2][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[1][i], xb[0][j], acc[2][i][j], 0, 0, 0);
                    }
                }
        };
        constexpr int NREAD = PLANES * (FM + FN), NMFMA = FM * FN * PLANES * PLANES;
        constexpr int WA = PLANES * Prefetch<BM, BK>::PASSES, WB = PLANES * Prefetch<BN, BK>::PASSES;
        const int va = t.m - tile_r < BM ? t.m - tile_r : BM;    // valid rows of the panels
        const int vb = t.n - tile_c < BN ? t.n - tile_c : BN;
        const int lda = __builtin_amdgcn_readfirstlane((int)t.A.ld);
        const int ldb = __builtin_amdgcn_readfirstlane((int)t.B.ld);
        __amdgpu_buffer_rsrc_t ra[PLANES], rb[PLANES];
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            ra[pl] = panel_rsrc((const int8_t*)t.A.p + pl * t.A.plane + (int64_t)tile_r * t.A.ld, (int64_t)va * t.A.ld);
            rb[pl] = panel_rsrc((const int8_t*)t.B.p + pl * t.B.plane + (int64_t)tile_c * t.B.ld, (int64_t)vb * t.B.ld);
        }
        auto load_a = [&](Prefetch<BM, BK> (&x)[PLANES], int k0, bool live) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) bload<BM, BK, EDGE>(x[pl], ra[pl], lda, k0, live);
        };
        auto load_b = [&](Prefetch<BN, BK> (&x)[PLANES], int k0, bool live) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) bload<BN, BK, EDGE>(x[pl], rb[pl], ldb, k0, live);
        };
        Prefetch<BM, BK> pa0[PLANES], pa1[PLANES];
        Prefetch<BN, BK> pb[PLANES];
        load_a(pa0, 0, true);
        load_b(pb, 0, true);
        load_a(pa1, BK, nk > 1);
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            lstore<BM, BK>(sa[0][pl], pa0[pl]);
            lstore<BN, BK>(sb[0][pl], pb[pl]);
        }
        load_b(pb, BK, nk > 1);
        __syncthreads();
        v4i fa[PLANES][FM], fb[PLANES][FN];
        read_frags(fa, fb, 0, 0);

        auto stage = [&](auto par, int kt) {
            constexpr int cur = decltype(par)::value;
            Prefetch<BM, BK> (&la)[PLANES] = cur ? pa1 : pa0;   // reloaded now (its stage is in LDS)
            Prefetch<BM, BK> (&wa)[PLANES] = cur ? pa0 : pa1;   // stage kt + 1, written now
            __builtin_amdgcn_sched_barrier(0);
            load_a(la, (kt + 2) * BK, kt + 2 < nk);
            __builtin_amdgcn_sched_barrier(0);
            v4i na[PLANES][FM], nb[PLANES][FN];
            constexpr int PA = Prefetch<BM, BK>::PASSES, HA = PA / 2;
            // k-step 0, first half of the A panel of stage kt + 1 to LDS
            read_frags(na, nb, cur, 1);
            mfmas(fa, fb);
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) lstore_part<BM, BK, 0, HA>(sa[cur ^ 1][pl], wa[pl]);
#pragma unroll
            for (int q = 0; q < NREAD; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / (NREAD + WA / 2), 0);
                __builtin_amdgcn_sched_group_barrier(0x200, (WA / 2) / NREAD > 0 ? (WA / 2) / NREAD : 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / (NREAD + WA / 2), 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            // k-step 1, second half of the A panel
            read_frags(fa, fb, cur, 2);
            mfmas(na, nb);
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) lstore_part<BM, BK, HA, PA>(sa[cur ^ 1][pl], wa[pl]);
#pragma unroll
            for (int q = 0; q < NREAD; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / (NREAD + WA / 2), 0);
                __builtin_amdgcn_sched_group_barrier(0x200, (WA / 2) / NREAD > 0 ? (WA / 2) / NREAD : 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / (NREAD + WA / 2), 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            // k-step 2, B panel of stage kt + 1 to LDS, then the loads of
            // stage kt + 2's B panel into the same registers
            read_frags(na, nb, cur, 3);
            mfmas(fa, fb);
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) lstore<BN, BK>(sb[cur ^ 1][pl], pb[pl]);
#pragma unroll
            for (int q = 0; q < NREAD; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / (NREAD + WB), 0);
                __builtin_amdgcn_sched_group_barrier(0x200, WB / NREAD, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / (NREAD + WB), 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            load_b(pb, (kt + 2) * BK, kt + 2 < nk);
            __syncthreads();
            // k-step 3 with the first fragments of stage kt + 1
            read_frags(fa, fb, cur ^ 1, 0);
            mfmas(na, nb);
#pragma unroll
            for (int q = 0; q < NREAD; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / NREAD, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        // stages in pairs (static register sets and buffers, no branch
        // between them); for odd nk the last stage of the last pair has
        // all-zero operands
        for (int kt = 0; kt < nk; kt += 2) {
            stage(std::integral_constant<int, 0>{}, kt);
            stage(std::integral_constant<int, 1>{}, kt + 1);
        }
    }
    if constexpr (PLANES == 1) {
        store_tile_i8_reg<WTM, WTN, FM, FN>(acc[0], t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
    } else {
        if (!wave_live) return;
        const double pd = (double)t.p;
        const double alpha = (double)t.alpha, beta = (double)t.beta;
        const double r16 = (double)((65536u) % t.p), r8 = (double)(256u % t.p);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int col = tile_c + wc * WTN + j * 32 + lrow;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int row = tile_r + wr * WTM + i * 32 + 8 * (e >> 2) + 4 * lk + (e & 3);
                    if (row >= t.m || col >= t.n) continue;
                    if (t.syrk && col > row) continue;
                    const double hh = mod_f64((double)acc[0][i][j][e], pd, t.pinv);
                    const double ll = mod_f64((double)acc[1][i][j][e], pd, t.pinv);
                    const double xx = mod_f64((double)acc[2][i][j][e], pd, t.pinv);
                    const double v = mod_f64(hh * r16 + xx * r8 + ll, pd, t.pinv);
                    uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                    double x = alpha * v;
                    if (t.beta != 0u) x += beta * (double)(*dst);
                    *dst = (uint32_t)mod_f64(x, pd, t.pinv);
                }
            }
    }
}

// ---- CLS_I8 with operands straight to LDS -------------------------------
//
// 256 x 256 tiles, 4 waves of 128 x 128, 128-byte k stages in two LDS
// buffers of 64 KB (the A panel's 256 rows of 128 bytes, then the B
// panel's).  The operands go from global memory to LDS with buffer loads
// that write LDS themselves: no staging registers and no LDS write
// instructions between the MFMAs.  One load instruction fills 1 KB, 8 rows
// of a panel: lane L writes slot L % 8 of row L / 8 with that row's 16-byte
// chunk (L % 8) ^ s(row), s(r) = (r & 7) ^ ((r >> 3) & 1), so that the
// fragment reads (one chunk of 8 or 16 consecutive rows) meet distinct
// banks.  The loads of stage t + 2 go into the buffer of stage t once the
// barrier of k-step 3 of stage t has ended every read of it: half during
// k-step 3 of stage t, half during k-step 0 of stage t + 1; each wave waits
// for its own loads (vmcnt) before the barrier of k-step 3 of stage t + 1,
// which publishes stage t + 2.  Each k-step issues its 16 MFMAs with the
// other instructions between them in a fixed order (a scheduling barrier
// after each): the LDS reads of the next k-step's fragments in the order the
// MFMAs consume them, and the loads.  Without the fixed order the compiler
// grouped the LDS traffic between MFMAs that then waited for it.
//
// Panels are read through buffer resources: stages past the end of k add
// 2^31 to the vector offsets, so their loads return zeros; a partial panel
// (EDGE) keeps the row of every load in its vector offset, and rows past the
// valid ones fall outside the resource (zeros).  Outputs of rows or columns
// past the end are never stored.

template <int N> using IC = std::integral_constant<int, N>;
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(IC<B>{});
        static_for<B + 1, E>(f);
    }
}

typedef __attribute__((address_space(3))) void LdsVoid;

__device__ __forceinline__ int dma_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// Epilogue of a two-limb wave tile (hh, ll and hl + lh accumulators):
// 2^16 hh + 2^8 x + ll mod p, then alpha and beta.
template <int WTM, int WTN, int FM, int FN>
__device__ __forceinline__ void store_tile_limb2(const v16i (&acc)[3][FM][FN], const ProdTask& t, int row0,
                                                 int col0, bool live)
{
    if (!live) return;
    const int lane = threadIdx.x & 63, lrow = lane & 31, lk = lane >> 5;
    const double pd = (double)t.p;
    const double alpha = (double)t.alpha, beta = (double)t.beta;
    const double r16 = (double)((65536u) % t.p), r8 = (double)(256u % t.p);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = col0 + j * 32 + lrow;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = row0 + i * 32 + 8 * (e >> 2) + 4 * lk + (e & 3);
                if (row >= t.m || col >= t.n) continue;
                if (t.syrk && col > row) continue;
                // |acc| < 2^31, r16 < p <= 65521, r8 <= 256: the sum is below 2^49, exact
                const double v = mod_f64(fma((double)acc[0][i][j][e], r16,
                                             fma((double)acc[2][i][j][e], r8, (double)acc[1][i][j][e])),
                                         pd, t.pinv);
                uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                double x = alpha * v;
                if (t.beta != 0u) x += beta * (double)(*dst);
                *dst = (uint32_t)mod_f64(x, pd, t.pinv);
            }
        }
}

// PLANES = 1: centred int8 on 256 x 256 tiles (one accumulator);
// PLANES = 2: two int8 limbs on 128 x 128 tiles (hh, ll and hl + lh
// accumulators).  Either way a wave issues 16 MFMAs and reads 8 fragments
// per k-step, and a stage is 64 blocks of 1 KB: the A and B panels (and
// their planes) one after the other.
template <int PLANES, bool EDGE>
__device__ __forceinline__ void i8_dma_body(const ProdTask& t, int ti, int tj, int8_t* smem, int kst0 = 0,
                                            int kst1 = -1, int32_t* part = nullptr)
{
    constexpr int BM = PLANES == 1 ? 256 : 128, BN = BM, BK = 128;
    constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 32, FN = WTN / 32;
    constexpr int NACC = PLANES == 1 ? 1 : 3;
    constexpr int NFRAG = PLANES * (FM + FN);
    static_assert(NFRAG == 8 && FM * FN * PLANES * PLANES == 16, "16 MFMAs and 8 fragment reads per k-step");
    constexpr int REGION = BM * BK;                 // bytes of one plane of one panel per stage
    constexpr int BUF = 2 * PLANES * REGION;        // A planes then B planes
    static_assert(BUF == 64 * 1024, "64 blocks of 1 KB per stage");
    constexpr int RBLK = BM / 8;                    // 1 KB blocks per region
    const int tile_r = ti * BM, tile_c = tj * BN;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lrow = lane & 31, lk = lane >> 5;

    v16i acc[NACC][FM][FN];
#pragma unroll
    for (int q = 0; q < NACC; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[q][i][j][e] = 0;
    const bool wave_live = !(t.syrk && (tile_c + wc * WTN) > (tile_r + wr * WTM + WTM - 1));

    // stages [kst0, kst1) of the task's k (a k-chunk of a split tile), or all
    const int kend = kst1 < 0 ? t.k / BK : kst1;
    const int nk = kend - kst0;
    if (nk > 0) {
        const int va = t.m - tile_r < BM ? t.m - tile_r : BM;    // valid rows of the panels
        const int vb = t.n - tile_c < BN ? t.n - tile_c : BN;
        const int lda = __builtin_amdgcn_readfirstlane((int)t.A.ld);
        const int ldb = __builtin_amdgcn_readfirstlane((int)t.B.ld);
        const int kbyte0 = kst0 * BK;
        // this wave loads blocks 16 wave .. 16 wave + 15 of a stage, all in
        // one region (panel and plane): region = 16 wave / RBLK
        const int region = (16 * wave) / RBLK, blk0 = (16 * wave) % RBLK;
        const bool isB = region >= PLANES;
        const int pl = region % PLANES;
        const int ld = isB ? ldb : lda;
        const __amdgpu_buffer_rsrc_t rs = isB
            ? panel_rsrc((const int8_t*)t.B.p + pl * t.B.plane + (int64_t)tile_c * t.B.ld, (int64_t)vb * t.B.ld)
            : panel_rsrc((const int8_t*)t.A.p + pl * t.A.plane + (int64_t)tile_r * t.A.ld, (int64_t)va * t.A.ld);
        const int lr8 = lane >> 3, slot = lane & 7;
        const int v0 = lr8 * ld + 16 * (slot ^ lr8), v1 = lr8 * ld + 16 * (slot ^ lr8 ^ 1);
        auto dload = [&](int q, int stg, bool live) {
            const uint32_t dead = live ? 0u : 0x80000000u;
            const int blk = blk0 + q;
            int8_t* dst = smem + (stg & 1) * BUF + region * REGION + blk * 1024;
            const int v = (blk & 1) ? v1 : v0;
            if constexpr (EDGE) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LdsVoid*)dst, 16, (uint32_t)(v + 8 * blk * ld) + dead,
                                                         __builtin_amdgcn_readfirstlane(kbyte0 + stg * BK), 0, 0);
            } else {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (LdsVoid*)dst, 16, (uint32_t)v + dead,
                    __builtin_amdgcn_readfirstlane(kbyte0 + stg * BK + 8 * blk * ld), 0, 0);
            }
        };
        const int sw = dma_swz(lrow);
        int coff[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) coff[ks] = 16 * ((2 * ks + lk) ^ sw);
        const int rowA = (wr * WTM + lrow) * BK, rowB = PLANES * REGION + (wc * WTN + lrow) * BK;
        v4i fa[PLANES][FM], fb[PLANES][FN], na[PLANES][FM], nb[PLANES][FN];
        // fragment o of a k-step, in the order the MFMAs first use them
        auto rd = [&](v4i (&xa)[PLANES][FM], v4i (&xb)[PLANES][FN], int buf, int ks, int o) {
            const int8_t* base = smem + buf * BUF + coff[ks];
            if constexpr (PLANES == 1) {
                // a0 b0 b1 b2 b3 a1 a2 a3
                if (o == 0 || o >= 5) {
                    const int i = o == 0 ? 0 : o - 4;
                    xa[0][i] = *reinterpret_cast<const v4i*>(base + rowA + i * 32 * BK);
                } else {
                    xb[0][o - 1] = *reinterpret_cast<const v4i*>(base + rowB + (o - 1) * 32 * BK);
                }
            } else {
                // ah0 bh0 al0 bl0 bh1 bl1 ah1 al1 (planes: 0 = hi, 1 = lo)
                constexpr int kA = 0, kB = 1;
                const int who[8] = {kA, kB, kA, kB, kB, kB, kA, kA};
                const int pli[8] = {0, 0, 1, 1, 0, 1, 0, 1};
                const int idx[8] = {0, 0, 0, 0, 1, 1, 1, 1};
                if (who[o] == kA)
                    xa[pli[o]][idx[o]] = *reinterpret_cast<const v4i*>(base + pli[o] * REGION + rowA + idx[o] * 32 * BK);
                else
                    xb[pli[o]][idx[o]] = *reinterpret_cast<const v4i*>(base + pli[o] * REGION + rowB + idx[o] * 32 * BK);
            }
        };
        // the previous tile of a persistent workgroup may still read LDS
        __syncthreads();
        for (int q = 0; q < 16; ++q) dload(q, 0, true);
        for (int q = 0; q < 16; ++q) dload(q, 1, nk > 1);
        asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
        __syncthreads();
        for (int o = 0; o < 8; ++o) rd(fa, fb, 0, 0, o);
        // one k-step: 16 MFMAs on (xa, xb), the NOPS other operations spread
        // between them in order
        auto kstep = [&](const v4i (&xa)[PLANES][FM], const v4i (&xb)[PLANES][FN], auto nops, auto&& op) {
            constexpr int NOPS = decltype(nops)::value;
            static_for<0, 16>([&](auto q) {
                constexpr int Q = decltype(q)::value;
                if constexpr (PLANES == 1) {
                    acc[0][Q / 4][Q % 4] =
                        __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[0][Q / 4], xb[0][Q % 4], acc[0][Q / 4][Q % 4], 0, 0, 0);
                } else {
                    // block (i, j) = (Q / 8, (Q / 4) % 2); products hh, ll, hl, lh
                    constexpr int I = Q / 8, J = (Q / 4) % 2, W = Q % 4;
                    constexpr int PA = (W == 0 || W == 2) ? 0 : 1, PB = (W == 0 || W == 3) ? 0 : 1;
                    constexpr int ACC = W == 0 ? 0 : (W == 1 ? 1 : 2);
                    acc[ACC][I][J] =
                        __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[PA][I], xb[PB][J], acc[ACC][I][J], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
                static_for<Q * NOPS / 16, (Q + 1) * NOPS / 16>([&](auto o) {
                    op(o);
                    __builtin_amdgcn_sched_barrier(0);
                });
            });
        };
        auto stage = [&](auto par, int kt) {
            constexpr int cur = decltype(par)::value;
            // k0: fragments of k-step 1; second half of stage kt + 1's loads
            kstep(fa, fb, IC<16>{}, [&](auto o) {
                constexpr int O = decltype(o)::value;
                if constexpr (O % 2 == 0) rd(na, nb, cur, 1, O / 2);
                else dload(8 + O / 2, kt + 1, kt + 1 < nk);
            });
            kstep(na, nb, IC<8>{}, [&](auto o) { rd(fa, fb, cur, 2, decltype(o)::value); });
            kstep(fa, fb, IC<8>{}, [&](auto o) { rd(na, nb, cur, 3, decltype(o)::value); });
            // stage kt + 1 in LDS: this wave's loads, then every wave's
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            // k3: first fragments of stage kt + 1; first half of stage kt + 2's loads
            kstep(na, nb, IC<16>{}, [&](auto o) {
                constexpr int O = decltype(o)::value;
                if constexpr (O % 2 == 0) rd(fa, fb, cur ^ 1, 0, O / 2);
                else dload(IC<O / 2>{}, kt + 2, kt + 2 < nk);
            });
        };
        // stages in pairs (static buffer indices); for odd nk the last stage of
        // the last pair reads loads past the end of k, i.e. zeros.  The first
        // k-step 0 re-issues the second half of stage 1 (same data).
        for (int kt = 0; kt < nk; kt += 2) {
            stage(IC<0>{}, kt);
            stage(IC<1>{}, kt + 1);
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    if (part != nullptr) {
        // a k-chunk of a split tile: the raw int32 sums, row-major BM x BN
        if constexpr (PLANES == 1) {
            const int lane2 = threadIdx.x & 63;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int r = wr * WTM + i * 32 + 8 * (e >> 2) + 4 * (lane2 >> 5) + (e & 3);
#pragma unroll
                    for (int j = 0; j < FN; ++j) part[r * BN + wc * WTN + j * 32 + (lane2 & 31)] = acc[0][i][j][e];
                }
        }
        return;
    }
    if constexpr (PLANES == 1)
        store_tile_i8_reg<WTM, WTN, FM, FN>(acc[0], t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
    else
        store_tile_limb2<WTM, WTN, FM, FN>(acc, t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
}

// Tile-rounds tail of a single-task int8 launch: workgroups b < args.total_tiles
// run whole tiles; the next ntail * nsplit run the k-chunk (b - total) % nsplit
// of tile total + (b - total) / nsplit, writing its int32 sums to
// part + (b - total) * 65536.  tail_reduce_kernel then adds the chunks.
__device__ __forceinline__ void i8_dma_split_item(const ProdArgs& args, int item, int nsplit, int32_t* part,
                                                  int8_t* smem)
{
    const ProdTask& t = args.inl[0];
    const int tile = args.total_tiles + item / nsplit, chunk = item % nsplit;
    int ti, tj;
    if (t.syrk) band_tri(tile, t.tm, &ti, &tj);
    else band_rect(tile, t.tm, t.tn, &ti, &tj);
    const int nst = t.k / 128;
    const int k0 = (int)((int64_t)nst * chunk / nsplit), k1 = (int)((int64_t)nst * (chunk + 1) / nsplit);
    int32_t* dst = part + (int64_t)item * 65536;
    if ((ti + 1) * 256 <= t.m && (tj + 1) * 256 <= t.n) i8_dma_body<1, false>(t, ti, tj, smem, k0, k1, dst);
    else i8_dma_body<1, true>(t, ti, tj, smem, k0, k1, dst);
}

template <int PLANES>
__device__ __forceinline__ void i8_dma_tile(const ProdArgs& args, int b)
{
    constexpr int BM = PLANES == 1 ? 256 : 128;
    __shared__ __attribute__((aligned(1024))) int8_t smem[2 * 64 * 1024];
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) band_tri(r, t.tm, &ti, &tj);
    else band_rect(r, t.tm, t.tn, &ti, &tj);
    if ((ti + 1) * BM <= t.m && (tj + 1) * BM <= t.n) i8_dma_body<PLANES, false>(t, ti, tj, smem);
    else i8_dma_body<PLANES, true>(t, ti, tj, smem);
}

template <int PLANES>
__global__ __launch_bounds__(256) void prod_i8_dma_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) i8_dma_tile<PLANES>(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) i8_dma_tile<PLANES>(args, b);
}

// Single task, int8: the whole tiles [0, args.total_tiles) first (one per
// workgroup, XCD-aware over the first nfull_grid blocks), then the k-chunks
// of the remaining ntail tiles.
__global__ __launch_bounds__(256) void prod_i8_dma_split_kernel(ProdArgs args, int nfull_grid, int nsplit,
                                                                int32_t* part)
{
    __shared__ __attribute__((aligned(1024))) int8_t smem[2 * 64 * 1024];
    const int bid = blockIdx.x;
    if (bid < nfull_grid) {
        const int b = xcd_remap(bid, nfull_grid);
        if (b < args.total_tiles) {
            const ProdTask& t = args.inl[0];
            int ti, tj;
            if (t.syrk) band_tri(b, t.tm, &ti, &tj);
            else band_rect(b, t.tm, t.tn, &ti, &tj);
            if ((ti + 1) * 256 <= t.m && (tj + 1) * 256 <= t.n) i8_dma_body<1, false>(t, ti, tj, smem);
            else i8_dma_body<1, true>(t, ti, tj, smem);
        }
        return;
    }
    i8_dma_split_item(args, bid - nfull_grid, nsplit, part, smem);
}

// C of the ntail split tiles: the sum of their nsplit int32 chunks, reduced
// mod p with alpha and beta; 16 elements per thread, 16 workgroups per tile.
__global__ __launch_bounds__(256) void tail_reduce_kernel(ProdTask t, int tile0, int nsplit, const int32_t* part)
{
    const int ltile = blockIdx.x / 16, piece = blockIdx.x % 16;
    int ti, tj;
    if (t.syrk) band_tri(tile0 + ltile, t.tm, &ti, &tj);
    else band_rect(tile0 + ltile, t.tm, t.tn, &ti, &tj);
    const int e0 = (piece * 256 + (int)threadIdx.x) * 16;           // element of the 256 x 256 tile
    const int r = e0 / 256, c0 = e0 % 256;
    const int row = ti * 256 + r;
    if (row >= t.m) return;
    int32_t sum[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) sum[u] = 0;
    for (int q = 0; q < nsplit; ++q) {
        const int32_t* src = part + ((int64_t)ltile * nsplit + q) * 65536 + e0;
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
            const v4i x = *reinterpret_cast<const v4i*>(src + u);
            sum[u] += x[0];
            sum[u + 1] += x[1];
            sum[u + 2] += x[2];
            sum[u + 3] += x[3];
        }
    }
    const SmallMod md(t.p);
    const bool plain = t.alpha == 1u && t.beta == 0u;
    uint32_t* rp = t.C + (int64_t)row * t.ldc;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int col = tj * 256 + c0 + u;
        if (col >= t.n || (t.syrk && col > row)) continue;
        uint32_t v = md.red_i(sum[u]);
        if (!plain) {
            uint32_t w = t.alpha * v;
            if (t.beta != 0u) w += t.beta * rp[col];
            v = md.red_u(w);
        }
        rp[col] = v;
    }
}

template <int BM, int BN, int BK, int PLANES>
__device__ __forceinline__ void i8_pipe_tile(const ProdArgs& args, int b)
{
    __shared__ __attribute__((aligned(16))) int8_t smem[I8Tile<BM, BN, BK, PLANES>::LDS];
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) band_tri(r, t.tm, &ti, &tj);
    else band_rect(r, t.tm, t.tn, &ti, &tj);
    if ((ti + 1) * BM <= t.m && (tj + 1) * BN <= t.n) i8_pipe_body<BM, BN, BK, PLANES, false>(t, ti, tj, smem);
    else i8_pipe_body<BM, BN, BK, PLANES, true>(t, ti, tj, smem);
}

template <int BM, int BN, int BK, int PLANES>
__global__ __launch_bounds__(256) void prod_i8_pipe_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) i8_pipe_tile<BM, BN, BK, PLANES>(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) i8_pipe_tile<BM, BN, BK, PLANES>(args, b);
}

// mode 0: one workgroup per tile; 1: same, XCD-aware order; 2: persistent.
// mode 0: one workgroup per tile; 1: one task, tiles dealt to the XCDs in
// contiguous ranges; 2: persistent workgroups striding over the tiles; 3:
// persistent, tiles dealt to the XCDs in chunks of neighbours.
// Three limbs: registers capped for two workgroups per CU (the second
// prefetch set of the tile fits beside the accumulators).
template <int BM, int BN, int BK, int PLANES>
__global__ __launch_bounds__(256, PLANES == 3 ? 2 : 1) void prod_i8_kernel(ProdArgs args, int mode)
{
    if (mode >= 2) {
        for (int i = 0;; ++i) {
            const int b = mode == 3 ? persistent_tile(blockIdx.x, gridDim.x, i) : blockIdx.x + i * gridDim.x;
            if (b >= args.total_tiles) break;
            i8_tile<BM, BN, BK, PLANES>(args, b);
        }
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) i8_tile<BM, BN, BK, PLANES>(args, b);
}

namespace {

// ---- CLS_LIMB3 with operands straight to LDS -------------------------------
// Three int8 limbs on 128 x 64 tiles: 4 waves of 64 x 32 with five weight
// accumulators (160 registers); per k-step a wave issues 18 MFMAs (nine limb
// products on two row blocks) and reads 9 fragments.  A stage (128 bytes of
// k) is 72 blocks of 1 KB, the A panel's three planes (16 blocks each) then
// the B panel's (8 blocks each); each wave loads 18 of them, in two halves
// placed like the int8 tile's.

template <bool EDGE>
__device__ __forceinline__ void l3_dma_body(const ProdTask& t, int ti, int tj, int8_t* smem)
{
    constexpr int BM = 128, BN = 64, BK = 128, WTM = 64, WTN = 32, FM = 2, FN = 1;
    constexpr int RA = BM * BK, RB = BN * BK;        // bytes of one plane of a panel per stage
    constexpr int BUF = 3 * (RA + RB);               // 72 blocks of 1 KB
    constexpr int PER = BUF / 1024 / 4;              // blocks per wave and stage
    static_assert(PER == 18, "18 blocks per wave");
    const int tile_r = ti * BM, tile_c = tj * BN;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lrow = lane & 31, lk = lane >> 5;

    v16i acc[5][FM][FN];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[q][i][j][e] = 0;
    const bool wave_live = !(t.syrk && (tile_c + wc * WTN) > (tile_r + wr * WTM + WTM - 1));

    const int nk = t.k / BK;
    if (nk > 0) {
        const int va = t.m - tile_r < BM ? t.m - tile_r : BM;    // valid rows of the panels
        const int vb = t.n - tile_c < BN ? t.n - tile_c : BN;
        const int lda = __builtin_amdgcn_readfirstlane((int)t.A.ld);
        const int ldb = __builtin_amdgcn_readfirstlane((int)t.B.ld);
        const int lr8 = lane >> 3, slot = lane & 7;
        // Load q of a stage is block gb = 4 q + wave, so that at a given q
        // every wave loads from the same plane of the same panel, known at
        // compile time: q < 12: A plane q / 4, block 4 (q % 4) + wave; else B
        // plane (q - 12) / 2, block 4 ((q - 12) % 2) + wave.  Row 8 blk + lr8
        // of the panel, 16-byte chunk slot ^ lr8 ^ (blk & 1) of its 128 bytes
        // (the swizzle the fragment reads undo; blk & 1 = wave & 1).  One
        // resource per panel covers its three planes (offset pl * plane);
        // rows past the panel's valid ones fall in the next plane or, in the
        // last plane, past the range, i.e. zeros; either only feeds output
        // rows or columns that are not stored.
        const __amdgpu_buffer_rsrc_t rsa = panel_rsrc((const int8_t*)t.A.p + (int64_t)tile_r * t.A.ld,
                                                      2 * t.A.plane + (int64_t)va * t.A.ld);
        const __amdgpu_buffer_rsrc_t rsb = panel_rsrc((const int8_t*)t.B.p + (int64_t)tile_c * t.B.ld,
                                                      2 * t.B.plane + (int64_t)vb * t.B.ld);
        const int pla = __builtin_amdgcn_readfirstlane((int)t.A.plane);
        const int plb = __builtin_amdgcn_readfirstlane((int)t.B.plane);
        const int chunk = 16 * (slot ^ lr8 ^ (wave & 1));
        const int va0 = (8 * wave + lr8) * lda + chunk, vb0 = (8 * wave + lr8) * ldb + chunk;
        auto dload = [&](auto qc, int stg, bool live) {
            constexpr int Q = decltype(qc)::value;
            constexpr bool ISB = Q >= 12;
            constexpr int PL = ISB ? (Q - 12) / 2 : Q / 4;
            constexpr int BQ = ISB ? 4 * ((Q - 12) % 2) : 4 * (Q % 4);   // block - wave
            const uint32_t dead = live ? 0u : 0x80000000u;
            int8_t* dst = smem + (stg & 1) * BUF + (4 * Q + wave) * 1024;
            const int pofs = ISB ? PL * plb + 8 * BQ * ldb : PL * pla + 8 * BQ * lda;
            const int v0 = ISB ? vb0 : va0;
            if constexpr (EDGE) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ISB ? rsb : rsa, (LdsVoid*)dst, 16,
                                                         (uint32_t)(v0 + pofs) + dead,
                                                         __builtin_amdgcn_readfirstlane(stg * BK), 0, 0);
            } else {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ISB ? rsb : rsa, (LdsVoid*)dst, 16, (uint32_t)v0 + dead,
                                                         __builtin_amdgcn_readfirstlane(stg * BK + pofs), 0, 0);
            }
        };
        const int sw = dma_swz(lrow);
        int coff[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) coff[ks] = 16 * ((2 * ks + lk) ^ sw);
        const int rowA = (wr * WTM + lrow) * BK, rowB = 3 * RA + (wc * WTN + lrow) * BK;
        v4i fa[3][FM], fb[3][FN], na[3][FM], nb[3][FN];
        // fragment o of a k-step, in the order the MFMAs first use them:
        // a0[0] b0 a0[1] b1 b2 a1[0] a1[1] a2[0] a2[1]
        auto rd = [&](v4i (&xa)[3][FM], v4i (&xb)[3][FN], int buf, int ks, int o) {
            const int8_t* base = smem + buf * BUF + coff[ks];
            const int isA[9] = {1, 0, 1, 0, 0, 1, 1, 1, 1};
            const int pli[9] = {0, 0, 0, 1, 2, 1, 1, 2, 2};
            const int idx[9] = {0, 0, 1, 0, 0, 0, 1, 0, 1};
            if (isA[o])
                xa[pli[o]][idx[o]] = *reinterpret_cast<const v4i*>(base + pli[o] * RA + rowA + idx[o] * 32 * BK);
            else
                xb[pli[o]][idx[o]] = *reinterpret_cast<const v4i*>(base + pli[o] * RB + rowB);
        };
        // the previous tile of a persistent workgroup may still read LDS
        __syncthreads();
        static_for<0, PER>([&](auto q) { dload(q, 0, true); });
        static_for<0, PER>([&](auto q) { dload(q, 1, nk > 1); });
        asm volatile("s_waitcnt vmcnt(18)" ::: "memory");
        __syncthreads();
        for (int o = 0; o < 9; ++o) rd(fa, fb, 0, 0, o);
        // one k-step: 18 MFMAs on (xa, xb) (limb products u x v into the
        // accumulator of weight u + v), the NOPS other operations spread
        // between them in order
        auto kstep = [&](const v4i (&xa)[3][FM], const v4i (&xb)[3][FN], auto nops, auto&& op) {
            constexpr int NOPS = decltype(nops)::value;
            static_for<0, 18>([&](auto q) {
                constexpr int Q = decltype(q)::value;
                constexpr int U = Q / 6, V = (Q % 6) / 2, I = Q % 2;
                acc[U + V][I][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[U][I], xb[V][0], acc[U + V][I][0], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                static_for<Q * NOPS / 18, (Q + 1) * NOPS / 18>([&](auto o) {
                    op(o);
                    __builtin_amdgcn_sched_barrier(0);
                });
            });
        };
        auto stage = [&](auto par, int kt) {
            constexpr int cur = decltype(par)::value;
            // k0: fragments of k-step 1; second half of stage kt + 1's loads
            kstep(fa, fb, IC<18>{}, [&](auto o) {
                constexpr int O = decltype(o)::value;
                if constexpr (O % 2 == 0) rd(na, nb, cur, 1, O / 2);
                else dload(IC<9 + O / 2>{}, kt + 1, kt + 1 < nk);
            });
            kstep(na, nb, IC<9>{}, [&](auto o) { rd(fa, fb, cur, 2, decltype(o)::value); });
            kstep(fa, fb, IC<9>{}, [&](auto o) { rd(na, nb, cur, 3, decltype(o)::value); });
            // stage kt + 1 in LDS: this wave's loads, then every wave's
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            // k3: first fragments of stage kt + 1; first half of stage kt + 2's loads
            kstep(na, nb, IC<18>{}, [&](auto o) {
                constexpr int O = decltype(o)::value;
                if constexpr (O % 2 == 0) rd(fa, fb, cur ^ 1, 0, O / 2);
                else dload(IC<O / 2>{}, kt + 2, kt + 2 < nk);
            });
        };
        // stages in pairs (static buffer indices); for odd nk the last stage of
        // the last pair reads loads past the end of k, i.e. zeros
        for (int kt = 0; kt < nk; kt += 2) {
            stage(IC<0>{}, kt);
            stage(IC<1>{}, kt + 1);
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    store_tile_limb3<WTM, WTN, FM, FN>(acc, t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
}

// Lower-triangle tiles of a SYRK task on 128 x 64 tiles: row block ti holds
// column blocks 0 .. 2 ti + 1 (those of the last may stop at tn - 1), so
// tile r is in row ti with ti (ti + 1) <= r < (ti + 1) (ti + 2).
__host__ __device__ inline int l3_syrk_tiles(int tm, int tn)
{
    int total = 0;
    for (int i = 0; i < tm; ++i) total += 2 * i + 2 < tn ? 2 * i + 2 : tn;
    return total;
}

__device__ __forceinline__ void l3_dma_tile(const ProdArgs& args, int b, int8_t* smem)
{
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) {
        ti = (int)((sqrtf(4.0f * (float)r + 1.0f) - 1.0f) * 0.5f);
        while ((ti + 1) * (ti + 2) <= r) ++ti;
        while (ti * (ti + 1) > r) --ti;
        tj = r - ti * (ti + 1);
    } else {
        ti = r / t.tn;
        tj = r - ti * t.tn;
    }
    if ((ti + 1) * 128 <= t.m && (tj + 1) * 64 <= t.n) l3_dma_body<false>(t, ti, tj, smem);
    else l3_dma_body<true>(t, ti, tj, smem);
}

__global__ __launch_bounds__(256) void prod_l3_dma_kernel(ProdArgs args, int mode)
{
    __shared__ __attribute__((aligned(1024))) int8_t smem[2 * 72 * 1024];
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) l3_dma_tile(args, b, smem);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) l3_dma_tile(args, b, smem);
}

// STAGING: 1 operands straight to LDS (DMA kernels), -1 register-staged with
// the LDS writes between the previous stage's MFMAs, 0 register-staged with
// the LDS writes after the stage's MFMAs.
template <int BM, int BN, int BK, int PLANES, int STAGING>
hipError_t launch_i8_once(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    ProdArgs args{};
    int total = 0;
    for (int i = 0; i < ntasks; ++i) {
        ProdTask& t = tasks[i];
        t.tm = (t.m + BM - 1) / BM;
        t.tn = (t.n + BN - 1) / BN;
        t.tile0 = total;
        total += t.syrk ? (BM == BN ? t.tm * (t.tm + 1) / 2 : l3_syrk_tiles(t.tm, t.tn)) : t.tm * t.tn;
    }
    if (total == 0) return hipSuccess;
    args.ntasks = ntasks;
    args.total_tiles = total;
    if (ntasks <= kInlineTasks) {
        for (int i = 0; i < ntasks; ++i) args.inl[i] = tasks[i];
    } else {
        hipError_t e = hipMemcpyAsync(dev_task_buf, tasks, sizeof(ProdTask) * ntasks,
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        args.dev_tasks = dev_task_buf;
    }
    const int mode = ntasks == 1 ? 1 : (g_persistent ? 2 : 0);
    int grid = mode == 1 ? (total + 7) / 8 * 8 : total;
    if constexpr (STAGING > 0 && PLANES == 3) {
        static_assert(BK == 128 && BM == 128 && BN == 64, "direct-to-LDS three limbs: 128 x 64 tiles");
        if (mode == 2) {
            const int resident = resident_blocks((const void*)prod_l3_dma_kernel);
            grid = total < resident ? total : resident;
        }
        g_last_variant = 14;
        hipLaunchKernelGGL(prod_l3_dma_kernel, dim3(grid), dim3(256), 0, s, args, mode);
    } else if constexpr (STAGING > 0) {
        static_assert(BK == 128 && ((PLANES == 1 && BM == 256) || (PLANES == 2 && BM == 128)) && BN == BM,
                      "direct-to-LDS variant: int8 256-tiles or two limbs on 128-tiles");
        if constexpr (PLANES == 1) {
            // a single task whose tiles leave the last round mostly idle: that
            // round's tiles split along k into chunks that fill it
            const TailScratch sc = g_tail_scratch;
            if (mode == 1 && g_split_tail && sc.ptr != nullptr && ntasks == 1) {
                const int R = resident_blocks((const void*)prod_i8_dma_split_kernel);
                const int tail = R > 0 ? total % R : 0;
                const int nst = tasks[0].k / 128;
                if (total > R && tail > 0 && 4 * tail <= R) {
                    int ns = R / tail;
                    if (ns > 8) ns = 8;
                    if (ns > nst) ns = nst;
                    while (ns > 1 && (size_t)tail * (size_t)ns * 65536u * 4u > sc.bytes) --ns;
                    if (ns >= 2) {
                        ProdArgs a2 = args;
                        a2.total_tiles = total - tail;
                        const int nfull_grid = (total - tail + 7) / 8 * 8;
                        g_last_variant = 13;
                        hipLaunchKernelGGL(prod_i8_dma_split_kernel, dim3(nfull_grid + tail * ns), dim3(256), 0, s,
                                           a2, nfull_grid, ns, (int32_t*)sc.ptr);
                        prof_mark_end(s);
                        hipLaunchKernelGGL(tail_reduce_kernel, dim3(tail * 16), dim3(256), 0, s, tasks[0],
                                           total - tail, ns, (const int32_t*)sc.ptr);
                        return hipGetLastError();
                    }
                }
            }
        }
        if (mode == 2) {
            const int resident = resident_blocks((const void*)prod_i8_dma_kernel<PLANES>);
            grid = total < resident ? total : resident;
        }
        g_last_variant = PLANES == 1 ? 6 : 7;
        hipLaunchKernelGGL((prod_i8_dma_kernel<PLANES>), dim3(grid), dim3(256), 0, s, args, mode);
    } else if constexpr (STAGING < 0) {
        static_assert(PLANES <= 2 && BK == 128, "pipelined variant: int8 or two limbs, 128-byte stages");
        if (mode == 2) {
            const int resident = resident_blocks((const void*)prod_i8_pipe_kernel<BM, BN, BK, PLANES>);
            grid = total < resident ? total : resident;
        }
        g_last_variant = PLANES == 1 ? 10 : 12;
        hipLaunchKernelGGL((prod_i8_pipe_kernel<BM, BN, BK, PLANES>), dim3(grid), dim3(256), 0, s, args, mode);
    } else {
        if (mode == 2) {
            const int resident = resident_blocks((const void*)prod_i8_kernel<BM, BN, BK, PLANES>);
            grid = total < resident ? total : resident;
        }
        g_last_variant = PLANES == 3 ? 9 : (PLANES == 2 ? 5 : (BM == 128 ? 2 : (BK == 64 ? 3 : 4)));
        const int m3 = mode == 2 && g_persistent == 2 ? 3 : mode;
        hipLaunchKernelGGL((prod_i8_kernel<BM, BN, BK, PLANES>), dim3(grid), dim3(256), 0, s, args, m3);
    }
    return hipGetLastError();
}

// The kernel accumulates a whole task in int32; when k exceeds the exact
// block length the task runs as consecutive launches over k-chunks, each
// accumulating into C (beta = 1 after the first), which reduces mod p
// between chunks.
template <int BM, int BN, int BK, int PLANES, int STAGING = 0>
hipError_t launch_i8_impl(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    int32_t maxk = 0, kblk = 1 << 30;
    for (int i = 0; i < ntasks; ++i) {
        ProdTask& t = tasks[i];
        if ((t.k % KSTEP) != 0 || (t.A.ld % 16) != 0 || (t.B.ld % 16) != 0 ||
            (((uintptr_t)t.A.p) & 15) != 0 || (((uintptr_t)t.B.p) & 15) != 0 ||
            (PLANES > 1 && ((t.A.plane % 16) != 0 || (t.B.plane % 16) != 0)))
            return hipErrorInvalidValue;
        const int64_t half = (t.p - 1) / 2;
        const int64_t per_k = PLANES == 1 ? half * half : (PLANES == 2 ? 2 * 128 * 128 : 3 * 128 * 128);
        // the kernels run whole stages of BK bytes: the k-blocks (and so the k
        // of every chunk launch) are multiples of BK
        constexpr int KU = BK > KSTEP ? BK : KSTEP;
        int64_t kb = (2147483647LL - (int64_t)t.p) / (per_k > 0 ? per_k : 1);
        kb -= kb % KU;
        t.kblk = cap_kblk(kb > (1 << 30) ? (1 << 30) : kb, KU);
        kblk = t.kblk < kblk ? t.kblk : kblk;
        maxk = t.k > maxk ? t.k : maxk;
    }
    if (maxk <= kblk) return launch_i8_once<BM, BN, BK, PLANES, STAGING>(tasks, ntasks, dev_task_buf, s);
    std::vector<ProdTask> part(tasks, tasks + ntasks);
    for (int32_t k0 = 0; k0 < maxk; k0 += kblk) {
        int np = 0;
        for (int i = 0; i < ntasks; ++i) {
            const ProdTask& t = tasks[i];
            if (k0 >= t.k && !(k0 == 0 && t.k == 0)) continue;
            ProdTask c = t;
            c.k = t.k - k0 < kblk ? t.k - k0 : kblk;
            c.A.p = (int8_t*)t.A.p + k0;
            c.B.p = (int8_t*)t.B.p + k0;
            c.beta = k0 == 0 ? t.beta : 1u;
            part[np++] = c;
        }
        // chunk launches carry their tasks inline (no staging copy outlives `part`)
        for (int q0 = 0; q0 < np; q0 += kInlineTasks) {
            const int nq = np - q0 < kInlineTasks ? np - q0 : kInlineTasks;
            hipError_t e = launch_i8_once<BM, BN, BK, PLANES, STAGING>(part.data() + q0, nq, nullptr, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

int64_t tiles_of(const ProdTask* tasks, int ntasks, int bm)
{
    int64_t total = 0;
    for (int i = 0; i < ntasks; ++i) {
        const int64_t tm = (tasks[i].m + bm - 1) / bm, tn = (tasks[i].n + bm - 1) / bm;
        total += tasks[i].syrk ? tm * (tm + 1) / 2 : tm * tn;
    }
    return total;
}

}  // namespace

bool prepare_limb3_tile_task(ProdTask* t)
{
    if ((t->k % KSTEP) != 0 || (t->A.ld % 16) != 0 || (t->B.ld % 16) != 0 ||
        (((uintptr_t)t->A.p) & 15) != 0 || (((uintptr_t)t->B.p) & 15) != 0 || (t->A.plane % 16) != 0 ||
        (t->B.plane % 16) != 0)
        return false;
    int64_t kb = (2147483647LL - (int64_t)t->p) / (3 * 128 * 128);
    kb -= kb % KSTEP;
    t->kblk = cap_kblk(kb, KSTEP);
    if (t->k > t->kblk) return false;   // would need k-chunked launches
    t->tm = (t->m + 63) / 64;
    t->tn = (t->n + 63) / 64;
    t->tile0 = 0;
    return true;
}

int g_i8_tile_override = 0;
int g_i8_bk_override = 0;
int g_i8_dma = 1;
int g_split_tail = 1;
int g_l3_dma = 1;
thread_local TailScratch g_tail_scratch = {nullptr, 0};
int g_i8_pipe = 1;

hipError_t launch_products_i8(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    // 256 x 256 tiles once they alone fill the 256 CUs twice over and
    // cover about the area 128 x 128 tiles would (many small products, as
    // in a batch, leave much of a 256-tile idle: 128-tiles then win)
    const int64_t t256 = tiles_of(tasks, ntasks, 256);
    bool big = t256 >= 512 && t256 * 4 * 10 <= tiles_of(tasks, ntasks, 128) * 11;
    const int ov = g_tile_hint ? g_tile_hint : g_i8_tile_override;
    if (ov == 128) big = false;
    if (ov == 256) big = true;
    bool k128 = true;
    for (int i = 0; i < ntasks; ++i) k128 = k128 && (tasks[i].k % 128) == 0;
    if (big) {
        if (g_i8_bk_override == 64 || !k128) return launch_i8_impl<256, 256, 64, 1>(tasks, ntasks, dev_task_buf, s);
        // the pipelined kernel addresses a 256-row panel with 32-bit offsets
        bool pipe_ok = g_i8_pipe != 0;
        for (int i = 0; i < ntasks; ++i)
            pipe_ok = pipe_ok && tasks[i].A.ld < (1 << 23) && tasks[i].B.ld < (1 << 23);
        if (pipe_ok && g_i8_dma) return launch_i8_impl<256, 256, 128, 1, 1>(tasks, ntasks, dev_task_buf, s);
        if (pipe_ok) return launch_i8_impl<256, 256, 128, 1, -1>(tasks, ntasks, dev_task_buf, s);
        return launch_i8_impl<256, 256, 128, 1>(tasks, ntasks, dev_task_buf, s);
    }
    return launch_i8_impl<128, 128, 64, 1>(tasks, ntasks, dev_task_buf, s);
}

hipError_t launch_products_limb2(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s)
{
    bool pipe = g_i8_pipe != 0;
    for (int i = 0; i < ntasks && pipe; ++i)
        pipe = (tasks[i].k % 128) == 0 && tasks[i].A.ld < (1 << 23) && tasks[i].B.ld < (1 << 23);
    if (pipe && g_i8_dma) return launch_i8_impl<128, 128, 128, 2, 1>(tasks, ntasks, dev_task_buf, s);
    if (pipe) return launch_i8_impl<128, 128, 128, 2, -1>(tasks, ntasks, dev_task_buf, s);
    return launch_i8_impl<128, 128, 64, 2>(tasks, ntasks, dev_task_buf, s);
}

hipError_t launch_products_limb3(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s)
{
    // 128 x 64 tiles with operands straight to LDS for large products (at
    // least four rounds of 128 x 64 tiles, k of at least 1024, a multiple of
    // 128; panels addressable with 32-bit offsets).  Their workgroup holds
    // 144 KB of LDS, one per CU, so on small products (batches of small
    // jobs) the 64 x 64 tiles, two workgroups per CU, hide the start of
    // each tile better.
    bool dma = g_i8_dma != 0 && g_l3_dma != 0;
    int64_t tiles = 0;
    for (int i = 0; i < ntasks && dma; ++i) {
        const ProdTask& t = tasks[i];
        // 32-bit buffer offsets: a panel's three planes, 128 rows deep, in
        // one resource (2 plane + 128 ld bytes) stay below 2^31
        dma = (t.k % 128) == 0 && (t.k >= 1024 || g_l3_dma > 1) &&
              2 * t.A.plane + 128 * t.A.ld < (1LL << 31) && 2 * t.B.plane + 128 * t.B.ld < (1LL << 31);
        const int tm = (t.m + 127) / 128, tn = (t.n + 63) / 64;
        tiles += t.syrk ? l3_syrk_tiles(tm, tn) : (int64_t)tm * tn;
    }
    if (dma && (tiles >= 1024 || g_l3_dma > 1)) return launch_i8_impl<128, 64, 128, 3, 1>(tasks, ntasks, dev_task_buf, s);
    return launch_i8_impl<64, 64, 64, 3>(tasks, ntasks, dev_task_buf, s);
}

}  // namespace ffp
