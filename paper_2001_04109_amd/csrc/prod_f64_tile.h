// 64 x 64 tiles of the FP64 base products with operands straight from
// global memory (see prod_f64.hip); shared with the LDL^T step kernel, which
// runs such tiles for its small products inside its per-level launch.
#pragma once
#include <type_traits>

#include "prod_common.h"

namespace ffp {

typedef double v4d __attribute__((ext_vector_type(4)));
// 16-byte vector in the global address space (global_load rather than flat)
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4u GU4;

namespace f64tile {

constexpr int WM = 2, WN = 2;           // wave tile in 16x16 blocks
constexpr int BM = kF64TileM, BN = kF64TileN;
static_assert(BM == 2 * WM * 16 && BN == 2 * WN * 16, "2x2 waves per workgroup");

struct Loaded { uint32_t v[4]; };

__device__ inline void load4(const uint32_t* __restrict__ base, int64_t ld, int row, int nrows,
                             int kcol, int K, bool vec_ok, Loaded& out)
{
    if (row < nrows) {
        const uint32_t* src = base + (int64_t)row * ld + kcol;
        if (vec_ok && kcol + 4 <= K) {
            const v4u q = *(const GU4*)src;
            out.v[0] = q.x; out.v[1] = q.y; out.v[2] = q.z; out.v[3] = q.w;
            return;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) out.v[j] = (kcol + j < K) ? src[j] : 0u;
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) out.v[j] = 0u;
}

__device__ inline double centred(uint32_t v, uint32_t half, uint32_t p)
{
    int32_t s = (v > half) ? (int32_t)v - (int32_t)p : (int32_t)v;
    return (double)s;
}


// Tile r (row-major over the task's tile grid, or over its lower triangle
// for a SYRK task) of one product task.
template <int FORM = TILE_NT>
__device__ __forceinline__ void f64_tile_task(const ProdTask& t, int r)
{
    constexpr bool NN = FORM == TILE_NN_BLOW || FORM == TILE_NN_ALOW;
    int ti, tj;
    if (t.syrk) tri_index(r, &ti, &tj);
    else { ti = r / t.tn; tj = r - ti * t.tn; }

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row0 = ti * BM + (wave >> 1) * (WM * 16);
    const int col0 = tj * BN + (wave & 1) * (WN * 16);
    if (row0 >= t.m || col0 >= t.n) return;
    if (t.syrk && col0 > row0 + WM * 16 - 1) return;   // sub-tile strictly above the diagonal

    const int lr = lane & 15, lk = lane >> 4;
    const uint32_t* __restrict__ Ab = (const uint32_t*)t.A.p;
    const uint32_t* __restrict__ Bb = (const uint32_t*)t.B.p;
    const bool vec_ok = ((t.A.ld & 3) == 0) && (NN || (t.B.ld & 3) == 0) &&
                        ((((uintptr_t)Ab) & 15) == 0) && (NN || (((uintptr_t)Bb) & 15) == 0);
    const double pd = (double)t.p;
    const int K = t.k;
    // k-range of the tile (multiples of 16 except the end of k)
    int kbeg = 0, kend = K;
    if constexpr (FORM == TILE_NT_BLOW) kend = min(K, (tj + 1) * BN);
    if constexpr (FORM == TILE_NN_BLOW) kbeg = min(K, tj * BN);
    if constexpr (FORM == TILE_NN_ALOW) kend = min(K, (ti + 1) * BM);

    v4d acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    // When k (p - 1)^2 < 2^53 the residues enter the products as they are
    // (one conversion per value; FP64 matrix instructions do not overlap
    // other vector instructions, so the centring would cost matrix time);
    // otherwise they are centred and the accumulators reduced every kblk.
    // For p above 2^25 fewer than 16 columns fit one exact block (kblk < 16):
    // the accumulators are then reduced after every 4-column step.
    const double pm1 = (double)(t.p - 1);
    const bool raw = (double)(kend - kbeg) * pm1 * pm1 < 9007199254740992.0 - 2.0 * pd;
    auto reduce_all = [&]() {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][e] = mod_f64(acc[i][j][e], pd, t.pinv);
    };
    // B of the NN forms: element (t, c) at Bb + t ldb + c; lane (lr, lk)
    // takes rows kc .. kc + 3 of its column (16 lanes read 64 contiguous bytes)
    auto loadb = [&](int kc, Loaded (&lb)[WN]) {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if constexpr (NN) {
                const int col = col0 + j * 16 + lr;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    lb[j].v[q] = (col < t.n && kc + q < K) ? Bb[(int64_t)(kc + q) * t.B.ld + col] : 0u;
            } else {
                load4(Bb, t.B.ld, col0 + j * 16 + lr, t.n, kc, K, vec_ok, lb[j]);
            }
        }
    };
    // operands in chunks of CH 16-column steps; the next chunk is loaded
    // while the current one is multiplied
    constexpr int CH = 2;
    auto load_chunk = [&](int k0, Loaded (&a)[CH][WM], Loaded (&b)[CH][WN]) {
#pragma unroll
        for (int h = 0; h < CH; ++h) {
            const int kc = k0 + 16 * h + 4 * lk;
#pragma unroll
            for (int i = 0; i < WM; ++i) load4(Ab, t.A.ld, row0 + i * 16 + lr, t.m, kc, K, vec_ok, a[h][i]);
            loadb(kc, b[h]);
        }
    };
    auto kloop = [&](auto rawc, auto stepc) {
        constexpr bool RAW = decltype(rawc)::value;
        constexpr bool STEP = decltype(stepc)::value;
        Loaded la[CH][WM], lb[CH][WN];
        int since_red = 0;
        if (kbeg < kend) load_chunk(kbeg, la, lb);
        for (int kk = kbeg; kk < kend; kk += 16 * CH) {
            Loaded na[CH][WM], nb[CH][WN];
            if (kk + 16 * CH < kend) load_chunk(kk + 16 * CH, na, nb);
#pragma unroll
            for (int h = 0; h < CH; ++h) {
                if (kk + 16 * h >= kend) break;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    double av[WM], bv[WN];
#pragma unroll
                    for (int i = 0; i < WM; ++i)
                        av[i] = RAW ? (double)la[h][i].v[s] : centred(la[h][i].v[s], t.half, t.p);
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        bv[j] = RAW ? (double)lb[h][j].v[s] : centred(lb[h][j].v[s], t.half, t.p);
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int j = 0; j < WN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
                    if constexpr (STEP) reduce_all();
                }
                if constexpr (!RAW && !STEP) {
                    since_red += 16;
                    if (since_red >= t.kblk && kk + 16 * (h + 1) < kend) {
                        since_red = 0;
                        reduce_all();
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < CH; ++h) {
#pragma unroll
                for (int i = 0; i < WM; ++i) la[h][i] = na[h][i];
#pragma unroll
                for (int j = 0; j < WN; ++j) lb[h][j] = nb[h][j];
            }
        }
    };
    using T_ = std::integral_constant<bool, true>;
    using F_ = std::integral_constant<bool, false>;
    if (raw) kloop(T_{}, F_{});
    else if (t.kblk < 16) kloop(F_{}, T_{});
    else kloop(F_{}, F_{});

    // Epilogue.  16x16 f64 MFMA result layout: element e of lane l is row
    // 4*e + l/16, column l%16.
    const double alpha = (double)t.alpha, beta = (double)t.beta;
    // 2 (p-1)^2 >= 2^53 from p = 67108865 on; p >= 2^25 takes the split form
    const bool big = t.p >= (1u << 25);
#pragma unroll
    for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int col = col0 + j * 16 + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = row0 + i * 16 + 4 * e + lk;
                if (row >= t.m || col >= t.n) continue;
                if (t.syrk && col > row) continue;
                uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                double v = mod_f64(acc[i][j][e], pd, t.pinv);
                double x;
                if (big) {
                    // alpha v + beta c may pass 2^53: reduce each term
                    x = mod_f64(alpha * v, pd, t.pinv);
                    if (t.beta != 0u) x += mod_f64(beta * (double)(*dst), pd, t.pinv);
                } else {
                    x = alpha * v;
                    if (t.beta != 0u) x += beta * (double)(*dst);
                }
                *dst = (uint32_t)mod_f64(x, pd, t.pinv);
            }
        }
    }
}

}  // namespace f64tile

using f64tile::centred;
using f64tile::f64_tile_task;


}  // namespace ffp
