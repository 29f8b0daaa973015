// Tiles of the int8 matrix-core base products (see prod_i8.hip): centred
// int8, two and three int8 limbs.  Shared with the LDL^T step kernel, which
// runs three-limb tiles for its Schur updates inside its per-level launch.
#pragma once
#include <type_traits>

#include "prod_common.h"

namespace ffp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
// 16-byte vector in the global address space (global_load rather than flat)
typedef __attribute__((address_space(1))) const v4i GV4;
// a result word in the global address space (global_store rather than flat)
typedef __attribute__((address_space(1))) uint32_t GU32;

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

// Epilogue of a CLS_LIMB3 wave tile: the five accumulators of weights
// 2^(8 q) are combined mod p (for p < 2^19 in one exact double: five terms
// below 2^52, one reduction; otherwise each term reduced first), then
// alpha / beta applied.  A sub-tile wholly inside C and not above the
// diagonal takes one row address per output row and no per-element tests.
template <int WTM, int WTN, int FM, int FN>
__device__ __forceinline__ void store_tile_limb3(const v16i (&acc)[5][FM][FN], const ProdTask& t, int row0,
                                                 int col0, bool live)
{
    if (!live) return;
    const int lane = threadIdx.x & 63, lrow = lane & 31, lk = lane >> 5;
    const double pd = (double)t.p, pinv = t.pinv;
    const double alpha = (double)t.alpha, beta = (double)t.beta;
    double cw[5];
    cw[0] = 1.0;
#pragma unroll
    for (int q = 1; q < 5; ++q) cw[q] = mod_f64(cw[q - 1] * 256.0, pd, pinv);
    const bool small = t.p < (1u << 19);
    const bool plain = t.alpha == 1u && t.beta == 0u;
    const bool inside = row0 + WTM <= t.m && col0 + WTN <= t.n && (!t.syrk || col0 + WTN - 1 <= row0);
    if (inside && small) {
        GU32* base = (GU32*)(t.C + (int64_t)(row0 + 4 * lk) * t.ldc + col0 + lrow);
        // output rows one at a time (the barrier keeps the compiler from
        // hoisting every row's address at once)
        auto rows = [&](auto with_ab) {
            constexpr bool AB = decltype(with_ab)::value;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    GU32* rp = base + (int64_t)(i * 32 + 8 * (e >> 2) + (e & 3)) * t.ldc;
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        double v = (double)acc[0][i][j][e];
#pragma unroll
                        for (int q = 1; q < 5; ++q) v = fma((double)acc[q][i][j][e], cw[q], v);
                        double r = mod_f64(v, pd, pinv);
                        if constexpr (AB)
                            r = mod_f64(fma(alpha, r, t.beta != 0u ? beta * (double)rp[j * 32] : 0.0), pd, pinv);
                        rp[j * 32] = (uint32_t)r;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
        };
        if (plain) rows(std::false_type{});
        else rows(std::true_type{});
        return;
    }
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
                double v = 0.0;
                if (small) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) v = fma((double)acc[q][i][j][e], cw[q], v);
                } else {
                    // five reduced terms below p^2 < 2^46: exact
#pragma unroll
                    for (int q = 0; q < 5; ++q) v += mod_f64((double)acc[q][i][j][e], pd, pinv) * cw[q];
                }
                v = mod_f64(v, pd, pinv);
                uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                if (!plain) v = mod_f64(fma(alpha, v, t.beta != 0u ? beta * (double)(*dst) : 0.0), pd, pinv);
                *dst = (uint32_t)v;
            }
        }
}

// PLANES = 1: CLS_I8;  2: CLS_LIMB2;  3: CLS_LIMB3.  BK: k bytes per stage.
template <int BM, int BN, int BK, int PLANES>
struct I8Tile {
    static constexpr int PITCH = BK + 16;
    static constexpr int LDS = 2 * PLANES * (BM + BN) * PITCH;   // bytes of LDS a tile needs
};

// Tile r (banded order over the task's tile grid or its lower triangle) of
// one product task; smem: I8Tile<...>::LDS bytes, 16-byte aligned.
// AHEAD2: a second register set holds the next stage's operands, so each
// stage's global loads are issued two stages before their LDS writes (more
// time for the loads of short products to land, at the cost of registers).
template <int BM, int BN, int BK, int PLANES, bool AHEAD2 = false>
__device__ __forceinline__ void i8_tile_task(const ProdTask& t, int r, int8_t* smem)
{
    constexpr int PITCH = BK + 16;
    constexpr int WTM = BM / 2, WTN = BN / 2;         // wave tile
    constexpr int FM = WTM / 32, FN = WTN / 32;       // 32x32 blocks per wave
    constexpr int NACC = PLANES == 1 ? 1 : (PLANES == 2 ? 3 : 5);
    constexpr int SA = 2 * PLANES * BM * PITCH;
    auto sa = reinterpret_cast<int8_t(*)[PLANES][BM * PITCH]>(smem);
    auto sb = reinterpret_cast<int8_t(*)[PLANES][BN * PITCH]>(smem + SA);
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
    Prefetch<BM, BK> pa[PLANES], qa[AHEAD2 ? PLANES : 1];
    Prefetch<BN, BK> pb[PLANES], qb[AHEAD2 ? PLANES : 1];
    if (nk > 0) {
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            gload<BM, BK>(pa[pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, 0);
            gload<BN, BK>(pb[pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, 0);
        }
        if constexpr (AHEAD2) {
            if (nk > 1)
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl) {
                    gload<BM, BK>(qa[pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, BK);
                    gload<BN, BK>(qb[pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, BK);
                }
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
    // one stage: x holds stage kt + 1's operands (loaded a stage earlier;
    // with one set they are loaded here), y is free for stage kt + 2's
    auto stage = [&](int kt, Prefetch<BM, BK> (&xa)[PLANES], Prefetch<BN, BK> (&xb)[PLANES], auto& ya,
                     auto& yb) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if constexpr (AHEAD2) {
            if (kt + 2 < nk) {
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl) {
                    gload<BM, BK>(ya[pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, (kt + 2) * BK);
                    gload<BN, BK>(yb[pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, (kt + 2) * BK);
                }
            }
        } else if (more) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) {
                gload<BM, BK>(xa[pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, (kt + 1) * BK);
                gload<BN, BK>(xb[pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, (kt + 1) * BK);
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
                lstore<BM, BK>(sa[cur ^ 1][pl], xa[pl]);
                lstore<BN, BK>(sb[cur ^ 1][pl], xb[pl]);
            }
        }
        __syncthreads();
        if (more) read_frags(fa, fb, cur ^ 1, 0);
    };
    if constexpr (AHEAD2) {
        // even stages find stage kt + 1 in q and load kt + 2 into p; odd
        // stages the other way round
        for (int kt = 0; kt < nk; kt += 2) {
            stage(kt, qa, qb, pa, pb);
            if (kt + 1 < nk) stage(kt + 1, pa, pb, qa, qb);
        }
    } else {
        for (int kt = 0; kt < nk; ++kt) stage(kt, pa, pb, pa, pb);
    }

    // Epilogue.  32x32 i32 MFMA result layout: lane l, element e holds
    // row 8*(e/4) + 4*(l/32) + e%4, column l%32.
    const double alpha = (double)t.alpha, beta = (double)t.beta;
    if constexpr (PLANES == 1) {
        store_tile_i8_reg<WTM, WTN, FM, FN>(acc[0], t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
    } else if constexpr (PLANES == 3) {
        store_tile_limb3<WTM, WTN, FM, FN>(acc, t, tile_r + wr * WTM, tile_c + wc * WTN, wave_live);
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
                    // |acc| < 2^31, r16 < p <= 65521, r8 <= 256: the sum is below 2^49, exact
                    const double v = mod_f64(fma((double)acc[0][i][j][e], r16,
                                                 fma((double)acc[NACC - 1][i][j][e], r8,
                                                     (double)acc[NACC - 2][i][j][e])),
                                             pd, t.pinv);
                    uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                    double x = alpha * v;
                    if (t.beta != 0u) x += beta * (double)(*dst);
                    *dst = (uint32_t)mod_f64(x, pd, t.pinv);
                }
            }
    }
}

}  // namespace ffp
