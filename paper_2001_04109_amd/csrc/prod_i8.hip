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
#include "prod_common.h"

#include <type_traits>
#include <vector>

namespace ffp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
// 16-byte vector in the global address space (global_load rather than flat)
typedef __attribute__((address_space(1))) const v4i GV4;

namespace {

constexpr int KSTEP = 64;           // k granularity of every launch (bytes)
constexpr int GBAND = 4;            // tile rows per band

__device__ inline int32_t mod_i32(int32_t x, double p, double pinv)
{
    return (int32_t)mod_f64((double)x, p, pinv);
}

// r-th tile of a tm x tn grid in banded order.
__device__ inline void band_rect(int r, int tm, int tn, int* ti, int* tj)
{
    const int per_band = GBAND * tn;
    const int b = r / per_band;
    const int loc = r - b * per_band;
    const int rows = min(GBAND, tm - b * GBAND);
    *tj = loc / rows;
    *ti = b * GBAND + loc % rows;
}

// r-th lower-triangle tile (tj <= ti) of a T x T grid in banded order:
// band b holds tile rows [bG, bG + rows); its rectangular part (tj < bG) is
// walked column by column, then its own rows x rows triangle, column by column.
__device__ inline void band_tri(int r, int T, int* ti, int* tj)
{
    const int G = GBAND;
    int b = 0, start = 0;
    for (;;) {
        const int rows = min(G, T - b * G);
        if (rows <= 0) break;
        const int cnt = b * G * rows + rows * (rows + 1) / 2;
        if (r < start + cnt) break;
        start += cnt;
        ++b;
    }
    const int rows = min(G, T - b * G);
    int loc = r - start;
    const int rect = b * G * rows;
    if (loc < rect) {
        *tj = loc / rows;
        *ti = b * G + loc % rows;
        return;
    }
    loc -= rect;
    int c = 0;
    while (c < rows - 1 && loc >= rows - c) { loc -= rows - c; ++c; }
    *tj = b * G + c;
    *ti = b * G + c + loc;
}

template <int ROWS, int BK>
struct Prefetch {
    static constexpr int PITCH = BK + 16;   // padded LDS row pitch
    static constexpr int CHUNKS = BK / 16;
    static constexpr int PASSES = ROWS * CHUNKS / 256;
    static_assert(ROWS * CHUNKS % 256 == 0, "panel must split evenly over 256 threads");
    v4i v[PASSES];
};

template <int ROWS, int BK>
__device__ inline void gload(Prefetch<ROWS, BK>& pf, const int8_t* __restrict__ g, int64_t ld, int row0,
                             int nrows, int k0)
{
    constexpr int CHUNKS = Prefetch<ROWS, BK>::CHUNKS;
#pragma unroll
    for (int ps = 0; ps < Prefetch<ROWS, BK>::PASSES; ++ps) {
        const int idx = ps * 256 + threadIdx.x;
        const int r = idx / CHUNKS, c = idx % CHUNKS;
        // Rows past the end re-read the last row: they only feed output rows
        // (or columns) past the end, which the epilogue never stores.
        const int row = row0 + r;
        const int rs = row < nrows ? row : nrows - 1;
        pf.v[ps] = *(const GV4*)(g + (int64_t)rs * ld + k0 + c * 16);
    }
}

template <int ROWS, int BK>
__device__ inline void lstore(int8_t* __restrict__ lds, const Prefetch<ROWS, BK>& pf)
{
    constexpr int CHUNKS = Prefetch<ROWS, BK>::CHUNKS;
#pragma unroll
    for (int ps = 0; ps < Prefetch<ROWS, BK>::PASSES; ++ps) {
        const int idx = ps * 256 + threadIdx.x;
        const int r = idx / CHUNKS, c = idx % CHUNKS;
        *reinterpret_cast<v4i*>(lds + r * Prefetch<ROWS, BK>::PITCH + c * 16) = pf.v[ps];
    }
}

}  // namespace

// Exact reduction of an int32 accumulator mod a prime p <= 251 with integer
// arithmetic (Barrett): u = x + B with B the smallest multiple of p that is
// >= 2^31 makes u non-negative (|x| <= 2^31 - 1 - p by the block length),
// q = floor(u m / 2^32) with m = floor(2^32 / p) is floor(u / p) or one
// less, so u - q p lies in [0, 2p).
struct SmallMod {
    uint32_t p, m, bias;
    __device__ explicit SmallMod(uint32_t p_) : p(p_), m(0xFFFFFFFFu / p_),
        bias(((0x80000000u + p_ - 1u) / p_) * p_) {}
    __device__ __forceinline__ uint32_t red_u(uint32_t u) const
    {
        const uint32_t q = __umulhi(u, m);
        uint32_t r = u - q * p;
        return r >= p ? r - p : r;
    }
    __device__ __forceinline__ uint32_t red_i(int32_t x) const { return red_u((uint32_t)x + bias); }
};

// Register epilogue of a CLS_I8 wave tile: every accumulator is reduced
// where it lies.  32x32 i32 MFMA result layout: lane l, element e holds row
// 8*(e/4) + 4*(l/32) + e%4, column l%32, so for one element index the 64
// lanes store two 128-byte row segments.  Tiles that lie wholly inside C
// and below the diagonal skip the per-element bounds tests.
template <int WTM, int WTN, int FM, int FN>
__device__ __forceinline__ void store_tile_i8_reg(const v16i (&acc)[FM][FN], const ProdTask& t,
                                                  int row0, int col0, bool live)
{
    if (!live) return;
    const int lane = threadIdx.x & 63, lrow = lane & 31, lk = lane >> 5;
    const SmallMod md(t.p);
    const bool plain = t.alpha == 1u && t.beta == 0u;
    const bool inside = row0 + WTM <= t.m && col0 + WTN <= t.n && (!t.syrk || col0 + WTN - 1 <= row0);
    uint32_t* __restrict__ base = t.C + (int64_t)(row0 + 4 * lk) * t.ldc + col0 + lrow;
    // one output row of the lane at a time: one address, FN stores with
    // immediate offsets (the barrier keeps the compiler from hoisting every
    // row's address at once)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int dr = i * 32 + 8 * (e >> 2) + (e & 3);        // row offset (before 4 lk)
            uint32_t* __restrict__ rp = base + (int64_t)dr * t.ldc;
            const int row = row0 + dr + 4 * lk;
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if (!inside) {
                    const int col = col0 + j * 32 + lrow;
                    if (row >= t.m || col >= t.n || (t.syrk && col > row)) continue;
                }
                uint32_t r = md.red_i(acc[i][j][e]);
                if (!plain) {
                    uint32_t v = t.alpha * r;                        // < p^2
                    if (t.beta != 0u) v += t.beta * rp[j * 32];       // < 2 p^2
                    r = md.red_u(v);
                }
                rp[j * 32] = r;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
}

// PLANES = 1: CLS_I8;  2: CLS_LIMB2;  3: CLS_LIMB3.  BK: k bytes per stage.
template <int BM, int BN, int BK, int PLANES>
__device__ __forceinline__ void i8_tile(const ProdArgs& args, int b)
{
    constexpr int PITCH = BK + 16;
    constexpr int WTM = BM / 2, WTN = BN / 2;         // wave tile
    constexpr int FM = WTM / 32, FN = WTN / 32;       // 32x32 blocks per wave
    constexpr int NACC = PLANES == 1 ? 1 : (PLANES == 2 ? 3 : 5);
    constexpr int SA = 2 * PLANES * BM * PITCH, SB = 2 * PLANES * BN * PITCH;
    __shared__ __attribute__((aligned(16))) int8_t smem[SA + SB];
    auto sa = reinterpret_cast<int8_t(*)[PLANES][BM * PITCH]>(smem);
    auto sb = reinterpret_cast<int8_t(*)[PLANES][BN * PITCH]>(smem + SA);

    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) band_tri(r, t.tm, &ti, &tj);
    else band_rect(r, t.tm, t.tn, &ti, &tj);
    const int tile_r = ti * BM, tile_c = tj * BN;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lrow = lane & 31, lk = lane >> 5;      // lane -> (row in block, 16-byte k half)

    const int8_t* __restrict__ Ab = (const int8_t*)t.A.p;
    const int8_t* __restrict__ Bb = (const int8_t*)t.B.p;
    const double pd = (double)t.p;

    v16i acc[NACC][FM][FN];
#pragma unroll
    for (int q = 0; q < NACC; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[q][i][j][e] = 0;

    // a wave whose sub-tile lies strictly above the diagonal stores nothing
    const bool wave_live = !(t.syrk && (tile_c + wc * WTN) > (tile_r + wr * WTM + WTM - 1));

    const int nk = t.k / BK;
    Prefetch<BM, BK> pa[PLANES];
    Prefetch<BN, BK> pb[PLANES];
    if (nk > 0) {
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            gload<BM, BK>(pa[pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, 0);
            gload<BN, BK>(pb[pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, 0);
        }
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            lstore<BM, BK>(sa[0][pl], pa[pl]);
            lstore<BN, BK>(sb[0][pl], pb[pl]);
        }
    }
    __syncthreads();
    // Fragments of the current k-step are in fa/fb; those of the next one are
    // read from LDS while the current MFMAs run (the scheduling hints keep the
    // compiler from sinking the reads next to their uses).
    constexpr int KS = BK / 32;
    v4i fa[PLANES][FM], fb[PLANES][FN];
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
                } else if constexpr (PLANES == 3) {
                    // planes: 0 = l, 1 = m, 2 = h; accumulator q has weight 2^(8 q)
#pragma unroll
                    for (int u = 0; u < 3; ++u)
#pragma unroll
                        for (int v = 0; v < 3; ++v)
                            acc[u + v][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[u][i], xb[v][j], acc[u + v][i][j], 0, 0, 0);
                } else {
                    acc[0][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[0][i], xb[0][j], acc[0][i][j], 0, 0, 0);
                    acc[NACC - 2][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[PLANES - 1][i], xb[PLANES - 1][j], acc[NACC - 2][i][j], 0, 0, 0);
                    acc[NACC - 1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[0][i], xb[PLANES - 1][j], acc[NACC - 1][i][j], 0, 0, 0);
                    acc[NACC - 1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[PLANES - 1][i], xb[0][j], acc[NACC - 1][i][j], 0, 0, 0);
                }
            }
    };
    constexpr int NREAD = PLANES * (FM + FN);
    constexpr int NMFMA = FM * FN * PLANES * PLANES;
    if (nk > 0) read_frags(fa, fb, 0, 0);
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) {
                gload<BM, BK>(pa[pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, (kt + 1) * BK);
                gload<BN, BK>(pb[pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, (kt + 1) * BK);
            }
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks + 1 < KS) {
                v4i na[PLANES][FM], nb[PLANES][FN];
                read_frags(na, nb, cur, ks + 1);
                mfmas(fa, fb);
                // interleave: one LDS read, then a share of the MFMAs
#pragma unroll
                for (int q = 0; q < NREAD; ++q) {
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / NREAD > 0 ? NMFMA / NREAD : 1, 0);
                }
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl) {
#pragma unroll
                    for (int i = 0; i < FM; ++i) fa[pl][i] = na[pl][i];
#pragma unroll
                    for (int j = 0; j < FN; ++j) fb[pl][j] = nb[pl][j];
                }
            } else {
                mfmas(fa, fb);
            }
        }
        if (more) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) {
                lstore<BM, BK>(sa[cur ^ 1][pl], pa[pl]);
                lstore<BN, BK>(sb[cur ^ 1][pl], pb[pl]);
            }
        }
        __syncthreads();
        if (more) read_frags(fa, fb, cur ^ 1, 0);
    }

    // Epilogue.  32x32 i32 MFMA result layout: lane l, element e holds
    // row 8*(e/4) + 4*(l/32) + e%4, column l%32.
    const double alpha = (double)t.alpha, beta = (double)t.beta;
    if constexpr (PLANES == 1) {
        store_tile_i8_reg<WTM, WTN, FM, FN>(acc[0], t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
    } else if constexpr (PLANES == 3) {
        if (!wave_live) return;
        // 2^(8 q) mod p for the five weights
        double cw[5];
        cw[0] = 1.0;
#pragma unroll
        for (int q = 1; q < 5; ++q) cw[q] = mod_f64(cw[q - 1] * 256.0, pd, t.pinv);
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
                    double v = 0.0;                      // five terms below p^2 < 2^46: exact
#pragma unroll
                    for (int q = 0; q < 5; ++q) v += mod_f64((double)acc[q][i][j][e], pd, t.pinv) * cw[q];
                    v = mod_f64(v, pd, t.pinv);
                    uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                    double x = alpha * v;
                    if (t.beta != 0u) x += beta * (double)(*dst);
                    *dst = (uint32_t)mod_f64(x, pd, t.pinv);
                }
            }
    } else {
        if (!wave_live) return;
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
                    const double ll = mod_f64((double)acc[NACC - 2][i][j][e], pd, t.pinv);
                    const double xx = mod_f64((double)acc[NACC - 1][i][j][e], pd, t.pinv);
                    const double v = mod_f64(hh * r16 + xx * r8 + ll, pd, t.pinv);
                    uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                    double x = alpha * v;
                    if (t.beta != 0u) x += beta * (double)(*dst);
                    *dst = (uint32_t)mod_f64(x, pd, t.pinv);
                }
            }
    }
}

// ---- CLS_I8 with direct-to-LDS operand loads ---------------------------
//
// Same tile and wave decomposition as i8_tile with BK = 64, but the operand
// panels go from global memory straight into LDS (global_load_lds_dwordx4:
// each wave instruction fills 1 KB of LDS, lane L at byte 16 L) through a
// ring of NS stages, so loads run NS - 2 stages ahead without staging
// registers or LDS write instructions.  A stage holds the BM + BN rows of
// 64 bytes of the A and B panels; the four 16-byte chunks of row r are
// stored in the order c ^ s(r) with s(r) = (r >> 2) & 3, which keeps the
// fragment reads (consecutive rows, one chunk) free of LDS bank conflicts
// (measured: the plain row-major order costs four times as much).  The compiler does not order these loads against LDS
// reads, so completion is waited for explicitly (vmcnt) before the
// workgroup barrier that publishes a stage.

__device__ __forceinline__ int swz64(int r) { return (r >> 2) & 3; }

// Workgroup barrier without the compiler's fence (which would wait for every
// direct-to-LDS load in flight); LDS reads of this wave are complete first.
__device__ __forceinline__ void ring_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Waits until at most n of this wave's vector-memory loads are in flight.
template <int L>
__device__ __forceinline__ void wait_loads(int stages_after)
{
    static_assert(3 * L < 64, "vmcnt range");
    if (stages_after >= 3) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(3 * L) : "memory");
    else if (stages_after == 2) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * L) : "memory");
    else if (stages_after == 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(L) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

typedef __attribute__((address_space(1))) const void GVoid;
typedef __attribute__((address_space(3))) void LVoid;

template <int BM, int BN>
__device__ __forceinline__ void ring_load(int8_t* stage, const int8_t* __restrict__ A, int64_t lda,
                                          int a_row0, int a_rows, const int8_t* __restrict__ B,
                                          int64_t ldb, int b_row0, int b_rows, int k0)
{
    constexpr int BLOCKS = (BM + BN) / 16;
    constexpr int PER_WAVE = BLOCKS / 4;
    static_assert(BLOCKS % 4 == 0 && (BM / 16) % PER_WAVE == 0, "a wave loads from one panel");
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const bool isA = wave * PER_WAVE < BM / 16;             // uniform per wave
    const int8_t* __restrict__ g = isA ? A : B;
    const int64_t ld = isA ? lda : ldb;
    const int prow0 = isA ? a_row0 : b_row0, prows = isA ? a_rows : b_rows;
    const int blk0 = isA ? wave * PER_WAVE : wave * PER_WAVE - BM / 16;
#pragma unroll
    for (int q = 0; q < PER_WAVE; ++q) {
        const int r = (blk0 + q) * 16 + (lane >> 2);           // row within the panel
        const int c = (lane & 3) ^ swz64(r);
        // rows past the end re-read the last row (their outputs are not stored)
        const int row = prow0 + r < prows ? prow0 + r : prows - 1;
        const int8_t* src = g + (int64_t)row * ld + k0 + c * 16;
        __builtin_amdgcn_global_load_lds((GVoid*)src, (LVoid*)(stage + (wave * PER_WAVE + q) * 1024),
                                         16, 0, 0);
    }
}

template <int BM, int BN, int NS>
__device__ __forceinline__ void i8_ring_tile(const ProdArgs& args, int b)
{
    constexpr int BK = 64;
    constexpr int STAGE = (BM + BN) * BK;
    constexpr int WTM = BM / 2, WTN = BN / 2;
    constexpr int FM = WTM / 32, FN = WTN / 32;
    constexpr int LOADS = (BM + BN) / 16 / 4;              // per wave and stage
    __shared__ __attribute__((aligned(1024))) int8_t smem[NS * STAGE];

    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) band_tri(r, t.tm, &ti, &tj);
    else band_rect(r, t.tm, t.tn, &ti, &tj);
    const int tile_r = ti * BM, tile_c = tj * BN;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lrow = lane & 31, lk = lane >> 5;
    const int8_t* __restrict__ Ab = (const int8_t*)t.A.p;
    const int8_t* __restrict__ Bb = (const int8_t*)t.B.p;

    v16i acc[FM][FN];
    // the task is the same for the whole workgroup: keep its loop bounds scalar
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0;
    const bool wave_live = !(t.syrk && (tile_c + wc * WTN) > (tile_r + wr * WTM + WTM - 1));

    // byte offsets of this lane's fragment rows inside a stage; the chunk of
    // k-step ks is (2 ks + lk) ^ s(row), and s(row) only depends on lrow
    const int sw = swz64(lrow);
    const int ch0 = ((0 + lk) ^ sw) * 16, ch1 = ((2 + lk) ^ sw) * 16;
    const int offA = (wr * WTM + lrow) * BK, offB = BM * BK + (wc * WTN + lrow) * BK;

    const int nk = __builtin_amdgcn_readfirstlane(t.k / BK);
    auto load_stage = [&](int s) {
        ring_load<BM, BN>(smem + (s % NS) * STAGE, Ab, t.A.ld, tile_r, t.m, Bb, t.B.ld, tile_c, t.n,
                          s * BK);
    };
    auto read_frags = [&](v4i (&xa)[FM], v4i (&xb)[FN], int s, int ch) {
        const int8_t* st = smem + (s % NS) * STAGE;
#pragma unroll
        for (int i = 0; i < FM; ++i)
            xa[i] = *reinterpret_cast<const v4i*>(st + offA + i * 32 * BK + ch);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            xb[j] = *reinterpret_cast<const v4i*>(st + offB + j * 32 * BK + ch);
    };
    auto mfmas = [&](const v4i (&xa)[FM], const v4i (&xb)[FN]) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[i], xb[j], acc[i][j], 0, 0, 0);
    };
    // one LDS read per MFMA over the first FM + FN MFMAs of a k-step, so the
    // reads have the rest of the k-step to land; with mfma_first the k-step
    // opens with an MFMA (its operands' wait then precedes the new reads)
    auto interleave = [&](auto mfma_first) {
        constexpr int lead = decltype(mfma_first)::value ? 1 : 0;
        if constexpr (lead) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
        for (int q = 0; q < FM + FN; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - (FM + FN) - lead, 0);
    };

    if (nk > 0) {
        for (int s = 0; s < NS - 1 && s < nk; ++s) load_stage(s);
        // stage 0 complete: the later prologue stages may stay in flight
        wait_loads<LOADS>((nk < NS - 1 ? nk : NS - 1) - 1);
        ring_barrier();
        v4i fa[FM], fb[FN], na[FM], nb[FN];
        read_frags(fa, fb, 0, ch0);
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) {
                // publish stage kt + 1; this also ends every read of the
                // buffer the next load overwrites (stage kt - 1)
                const int issued = kt + NS - 1 < nk ? kt + NS - 1 : nk;
                wait_loads<LOADS>(issued - (kt + 2));
                ring_barrier();
                if (kt + NS - 1 < nk) load_stage(kt + NS - 1);
            }
            // fa/fb (read during the previous k-step) have landed; stated to
            // the compiler so that it adds no wait inside the MFMA stream
            __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
            read_frags(na, nb, kt, ch1);
            mfmas(fa, fb);
            interleave(std::false_type{});
            // first k-step of the next stage; after the last stage this reads
            // an idle ring buffer whose values are never used
            read_frags(fa, fb, kt + 1, ch0);
            mfmas(na, nb);
            interleave(std::true_type{});
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    ring_barrier();
    store_tile_i8_reg<WTM, WTN, FM, FN>(acc, t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
}

template <int BM, int BN, int NS>
__global__ __launch_bounds__(256) void prod_i8_ring_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) i8_ring_tile<BM, BN, NS>(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) i8_ring_tile<BM, BN, NS>(args, b);
}

// mode 0: one workgroup per tile; 1: same, XCD-aware order; 2: persistent.
template <int BM, int BN, int BK, int PLANES>
__global__ __launch_bounds__(256) void prod_i8_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x)
            i8_tile<BM, BN, BK, PLANES>(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) i8_tile<BM, BN, BK, PLANES>(args, b);
}

namespace {

template <int BM, int BN, int BK, int PLANES, int RING>
hipError_t launch_i8_once(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    ProdArgs args{};
    int total = 0;
    for (int i = 0; i < ntasks; ++i) {
        ProdTask& t = tasks[i];
        t.tm = (t.m + BM - 1) / BM;
        t.tn = (t.n + BN - 1) / BN;
        t.tile0 = total;
        total += t.syrk ? t.tm * (t.tm + 1) / 2 : t.tm * t.tn;
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
    if constexpr (RING > 0) {
        static_assert(PLANES == 1 && BK == 64, "ring variant: CLS_I8, 64-byte stages");
        if (mode == 2) {
            const int resident = resident_blocks((const void*)prod_i8_ring_kernel<BM, BN, RING>);
            grid = total < resident ? total : resident;
        }
        g_last_variant = 6 + (RING - 4);
        hipLaunchKernelGGL((prod_i8_ring_kernel<BM, BN, RING>), dim3(grid), dim3(256), 0, s, args, mode);
    } else {
        if (mode == 2) {
            const int resident = resident_blocks((const void*)prod_i8_kernel<BM, BN, BK, PLANES>);
            grid = total < resident ? total : resident;
        }
        g_last_variant = PLANES == 3 ? 9 : (PLANES == 2 ? 5 : (BM == 128 ? 2 : (BK == 64 ? 3 : 4)));
        hipLaunchKernelGGL((prod_i8_kernel<BM, BN, BK, PLANES>), dim3(grid), dim3(256), 0, s, args, mode);
    }
    return hipGetLastError();
}

// The kernel accumulates a whole task in int32; when k exceeds the exact
// block length the task runs as consecutive launches over k-chunks, each
// accumulating into C (beta = 1 after the first), which reduces mod p
// between chunks.
template <int BM, int BN, int BK, int PLANES, int RING = 0>
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
        int64_t kb = (2147483647LL - (int64_t)t.p) / (per_k > 0 ? per_k : 1);
        kb -= kb % KSTEP;
        t.kblk = cap_kblk(kb > (1 << 30) ? (1 << 30) : kb, KSTEP);
        kblk = t.kblk < kblk ? t.kblk : kblk;
        maxk = t.k > maxk ? t.k : maxk;
    }
    if (maxk <= kblk) return launch_i8_once<BM, BN, BK, PLANES, RING>(tasks, ntasks, dev_task_buf, s);
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
            hipError_t e = launch_i8_once<BM, BN, BK, PLANES, RING>(part.data() + q0, nq, nullptr, s);
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

int g_i8_tile_override = 0;
int g_i8_bk_override = 0;
int g_i8_ring = 0;

hipError_t launch_products_i8(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    // 256 x 256 tiles once they alone fill the 256 CUs twice over
    bool big = tiles_of(tasks, ntasks, 256) >= 512;
    const int ov = g_tile_hint ? g_tile_hint : g_i8_tile_override;
    if (ov == 128) big = false;
    if (ov == 256) big = true;
    bool k128 = true;
    for (int i = 0; i < ntasks; ++i) k128 = k128 && (tasks[i].k % 128) == 0;
    if (big) {
        if (g_i8_ring == 4) return launch_i8_impl<256, 256, 64, 1, 4>(tasks, ntasks, dev_task_buf, s);
        if (g_i8_ring == 5) return launch_i8_impl<256, 256, 64, 1, 5>(tasks, ntasks, dev_task_buf, s);
        if (g_i8_bk_override == 64 || !k128) return launch_i8_impl<256, 256, 64, 1>(tasks, ntasks, dev_task_buf, s);
        return launch_i8_impl<256, 256, 128, 1>(tasks, ntasks, dev_task_buf, s);
    }
    return launch_i8_impl<128, 128, 64, 1>(tasks, ntasks, dev_task_buf, s);
}

hipError_t launch_products_limb2(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s)
{
    return launch_i8_impl<128, 128, 64, 2>(tasks, ntasks, dev_task_buf, s);
}

hipError_t launch_products_limb3(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s)
{
    return launch_i8_impl<64, 64, 64, 3>(tasks, ntasks, dev_task_buf, s);
}

}  // namespace ffp
