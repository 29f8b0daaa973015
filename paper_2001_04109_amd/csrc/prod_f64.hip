// Base-case products on FP64 matrix cores (CDNA4 v_mfma_f64_16x16x4f64).
//
// Residues in [0,p) are loaded as uint32, centred to [-(p-1)/2, (p-1)/2]
// and converted to double in registers; every product and partial sum is an
// integer below 2^53 in magnitude, so the accumulation is exact in any
// order.  The accumulators are reduced mod p every `kblk` columns of k
// (delayed reduction), and once more in the epilogue, which also applies
// alpha and beta.  This is the classical base case of the recursion
// (Algorithm 2 leaves and its general products P3, P4).
//
// Work decomposition: one workgroup of 4 waves per 64 x 64 output tile,
// each wave a 32 x 32 sub-tile of 2 x 2 MFMA blocks.  Operands stream
// straight from global memory (the FP64 rate leaves the L1/L2 path far from
// its limits); each lane loads 16 consecutive bytes of one row per 16-wide
// k chunk, and the four MFMA steps of the chunk consume one of the four
// values each.  A and B use the same lane-to-k assignment, so the sum over
// the chunk is exactly the sum over its 16 columns.
#include "prod_f64_tile.h"

namespace ffp {

__device__ __forceinline__ void f64_tile(const ProdArgs& args, int b)
{
    ProdTask t;
    select_task(args, b, &t);
    f64_tile_task(t, b - t.tile0);
}

// ---- 128 x 128 tiles through LDS -------------------------------------------
// Workgroup tile 128 x 128 of NW waves: 4 waves of 64 x 64 (4 x 4 MFMA
// blocks) or 8 waves of 64 x 32 (4 x 2 blocks; half the accumulators per
// wave, so that two waves share each SIMD and hide each other's LDS and
// barrier waits).  Per stage of 32 columns of k the A and B panels (128
// rows x 128 bytes each) are copied global -> registers -> LDS
// (double-buffered; the loads for the next stage are issued before the
// MFMAs of the current one).  Each lane reads 16 bytes (4 consecutive k)
// per row block from LDS and feeds them to four MFMA steps, as in the
// direct kernel.
namespace {
constexpr int BM2 = 128, BK2 = 32, PITCH2 = BK2 + 4;   // u32 units

template <int NW>
struct F64Lds {
    static constexpr int NT = 64 * NW;
    static constexpr int WCOLS = NW / 2;            // waves across the columns
    static constexpr int WTN = BM2 / WCOLS;         // wave tile columns
    static constexpr int WM = 4, WN = WTN / 16;     // 16 x 16 MFMA blocks per wave
    static constexpr int PASSES = BM2 * (BK2 / 4) / NT;
    struct Pf { uint4 v[PASSES]; };
};

template <int NW>
__device__ inline void gload2(typename F64Lds<NW>::Pf& pf, const uint32_t* __restrict__ g, int64_t ld, int row0,
                              int nrows, int k0, int K, bool vec_ok)
{
#pragma unroll
    for (int ps = 0; ps < F64Lds<NW>::PASSES; ++ps) {
        const int idx = ps * F64Lds<NW>::NT + threadIdx.x;
        const int r = idx >> 3, c = (idx & 7) * 4;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        const int row = row0 + r, kc = k0 + c;
        if (row < nrows) {
            const uint32_t* src = g + (int64_t)row * ld + kc;
            if (vec_ok && kc + 4 <= K) {
                const v4u q = *(const GU4*)src;
                v = make_uint4(q.x, q.y, q.z, q.w);
            } else {
                v.x = kc < K ? src[0] : 0u;
                v.y = kc + 1 < K ? src[1] : 0u;
                v.z = kc + 2 < K ? src[2] : 0u;
                v.w = kc + 3 < K ? src[3] : 0u;
            }
        }
        pf.v[ps] = v;
    }
}

// Residues are stored centred (as int32 bit patterns), so a fragment value
// only needs one conversion to double.
template <int NW>
__device__ inline void lstore2(uint32_t* __restrict__ lds, const typename F64Lds<NW>::Pf& pf, uint32_t half,
                               uint32_t p)
{
#pragma unroll
    for (int ps = 0; ps < F64Lds<NW>::PASSES; ++ps) {
        const int idx = ps * F64Lds<NW>::NT + threadIdx.x;
        const int r = idx >> 3, c = (idx & 7) * 4;
        const uint4 v = pf.v[ps];
        *reinterpret_cast<uint4*>(lds + r * PITCH2 + c) =
            make_uint4(v.x > half ? v.x - p : v.x, v.y > half ? v.y - p : v.y, v.z > half ? v.z - p : v.z,
                       v.w > half ? v.w - p : v.w);
    }
}

__device__ inline double sel4(const uint4& q, int s)
{
    return (double)(int32_t)(s == 0 ? q.x : s == 1 ? q.y : s == 2 ? q.z : q.w);
}
}  // namespace

// Three LDS buffers: stage t is read from buffer t % 3 while the loads of
// stage t + 2 are in flight and are written to buffer (t + 2) % 3 at its
// end (that buffer was last read in stage t - 1, before the previous
// barrier).  Stage t + 1 was published by the barrier that ended stage
// t - 1, so the fragments of its first k-group are read during the last
// MFMAs of stage t, and the k-groups inside a stage are likewise read one
// ahead: no LDS latency sits between the matrix instructions.
template <int NW>
__device__ __forceinline__ void f64_lds_tile(const ProdArgs& args, int b)
{
    using G = F64Lds<NW>;
    constexpr int WM2 = G::WM, WN2 = G::WN;
    constexpr int NBUF = 3, KG = BK2 / 16;
    __shared__ __attribute__((aligned(16))) uint32_t sa[NBUF][BM2 * PITCH2];
    __shared__ __attribute__((aligned(16))) uint32_t sb[NBUF][BM2 * PITCH2];
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) tri_index(r, &ti, &tj);
    else { ti = r / t.tn; tj = r - ti * t.tn; }
    const int tile_r = ti * BM2, tile_c = tj * BM2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave / G::WCOLS, wc = wave % G::WCOLS;
    const int lr = lane & 15, lk = lane >> 4;
    const uint32_t* __restrict__ Ab = (const uint32_t*)t.A.p;
    const uint32_t* __restrict__ Bb = (const uint32_t*)t.B.p;
    const bool vec_ok = ((t.A.ld & 3) == 0) && ((t.B.ld & 3) == 0) &&
                        ((((uintptr_t)Ab) & 15) == 0) && ((((uintptr_t)Bb) & 15) == 0);
    const double pd = (double)t.p;
    const int K = t.k;
    const int nk = (K + BK2 - 1) / BK2;

    v4d acc[WM2][WN2];
#pragma unroll
    for (int i = 0; i < WM2; ++i)
#pragma unroll
        for (int j = 0; j < WN2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    typename G::Pf pa, pb;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
        if (st < nk) {
            gload2<NW>(pa, Ab, t.A.ld, tile_r, t.m, st * BK2, K, vec_ok);
            gload2<NW>(pb, Bb, t.B.ld, tile_c, t.n, st * BK2, K, vec_ok);
            lstore2<NW>(sa[st], pa, t.half, t.p);
            lstore2<NW>(sb[st], pb, t.half, t.p);
        }
    }
    __syncthreads();
    auto read_frags = [&](uint4 (&xa)[WM2], uint4 (&xb)[WN2], int buf, int kg) {
#pragma unroll
        for (int i = 0; i < WM2; ++i)
            xa[i] = *reinterpret_cast<const uint4*>(&sa[buf][(wr * 64 + i * 16 + lr) * PITCH2 + kg * 16 + 4 * lk]);
#pragma unroll
        for (int j = 0; j < WN2; ++j)
            xb[j] = *reinterpret_cast<const uint4*>(&sb[buf][(wc * G::WTN + j * 16 + lr) * PITCH2 + kg * 16 + 4 * lk]);
    };
    // fragments double-buffered in registers: k-group g of a stage uses set
    // g & 1 (KG is even, so the first k-group of every stage uses set 0)
    static_assert(KG % 2 == 0, "fragment sets alternate per k-group");
    uint4 fa[2][WM2], fb[2][WN2];
    if (nk > 0) read_frags(fa[0], fb[0], 0, 0);
    // k-blocks of kblk columns (a multiple of BK2); the accumulators are
    // reduced mod p after every block, outside the stage loop.
    const int nkb = t.kblk / BK2;
    for (int kb0 = 0; kb0 < nk; kb0 += nkb) {
        const int kend = min(kb0 + nkb, nk);
        for (int kt = kb0; kt < kend; ++kt) {
            const int cur = kt % NBUF;
            const bool load2 = kt + 2 < nk;
            if (load2) {
                gload2<NW>(pa, Ab, t.A.ld, tile_r, t.m, (kt + 2) * BK2, K, vec_ok);
                gload2<NW>(pb, Bb, t.B.ld, tile_c, t.n, (kt + 2) * BK2, K, vec_ok);
            }
#pragma unroll
            for (int kg = 0; kg < KG; ++kg) {
                // fragments of the next k-group (this stage or the next one)
                // no branch here (one scheduling region per k-group): after
                // the last stage this reads a stale buffer, which is never used
                if (kg + 1 < KG) read_frags(fa[(kg + 1) & 1], fb[(kg + 1) & 1], cur, kg + 1);
                else read_frags(fa[(kg + 1) & 1], fb[(kg + 1) & 1], (kt + 1) % NBUF, 0);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    double av[WM2], bv[WN2];
#pragma unroll
                    for (int i = 0; i < WM2; ++i) av[i] = sel4(fa[kg & 1][i], s);
#pragma unroll
                    for (int j = 0; j < WN2; ++j) bv[j] = sel4(fb[kg & 1][j], s);
#pragma unroll
                    for (int i = 0; i < WM2; ++i)
#pragma unroll
                        for (int j = 0; j < WN2; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
                }
            }
            if (load2) {
                lstore2<NW>(sa[(kt + 2) % NBUF], pa, t.half, t.p);
                lstore2<NW>(sb[(kt + 2) % NBUF], pb, t.half, t.p);
            }
            __syncthreads();
        }
        if (kend < nk) {
#pragma unroll
            for (int i = 0; i < WM2; ++i)
#pragma unroll
                for (int j = 0; j < WN2; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[i][j][e] = mod_f64(acc[i][j][e], pd, t.pinv);
        }
    }

    const double alpha = (double)t.alpha, beta = (double)t.beta;
#pragma unroll
    for (int i = 0; i < WM2; ++i) {
#pragma unroll
        for (int j = 0; j < WN2; ++j) {
            const int col = tile_c + wc * G::WTN + j * 16 + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = tile_r + wr * 64 + i * 16 + 4 * e + lk;
                if (row >= t.m || col >= t.n) continue;
                if (t.syrk && col > row) continue;
                uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                double v = mod_f64(acc[i][j][e], pd, t.pinv);
                double x = alpha * v;
                if (t.beta != 0u) x += beta * (double)(*dst);
                *dst = (uint32_t)mod_f64(x, pd, t.pinv);
            }
        }
    }
}

// ---- 128 x 128 tiles, operands as doubles in LDS ---------------------------
// Same tile and 8-wave decomposition as f64_lds_tile<8>, for tasks with
// k <= kblk (no reduction inside the k-loop), k a multiple of 4 and aligned
// rows.  Matrix-core instructions do not run while the SIMD executes other
// vector instructions, so this variant minimises them: every operand value
// is converted to double once per workgroup, when it is written to LDS,
// instead of once per wave that reads it (four waves read each A value, two
// each B value), and is not centred (residues in [0, p), so it needs
// k (p - 1)^2 < 2^53 instead of k ((p - 1) / 2)^2 < 2^53).  Two LDS buffers of 128 x 32 doubles per
// operand; two register sets hold the raw panels of the next two stages
// (loaded through buffer resources with one 32-bit offset per load; chunks
// past the end of k or of the rows return zero); stage t writes the panels
// of stage t + 1 into the free buffer during its first k-group, the barrier
// sits between its two k-groups, and the second k-group's MFMAs cover the
// reads of stage t + 1's first fragments.  Stages run in pairs (static
// register sets); for an odd count the last stage is all zeros.
namespace {
constexpr int PD = BK2 + 2;   // LDS pitch in doubles: 16 rows of a 16-byte column hit distinct banks

__device__ __forceinline__ __amdgpu_buffer_rsrc_t f64_panel_rsrc(const uint32_t* p, int64_t bytes)
{
    const uint64_t a = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const int nb = __builtin_amdgcn_readfirstlane((int)(bytes < 0x7FFFFFFF ? bytes : 0x7FFFFFFF));
    void* base = (void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nb, 0x00020000);
}

struct F64Raw { v4u v[2]; };   // 2 passes of 512 threads x 4 values = 128 rows x 32 k

// Raw residues of stage k0 (columns k0 .. k0 + 31) of a 128-row panel.
__device__ __forceinline__ void f64_bload(F64Raw& pf, __amdgpu_buffer_rsrc_t rs, int ld, int k0, int K)
{
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
        const int idx = ps * 512 + threadIdx.x;
        const int r = idx >> 3, c = (idx & 7) * 4;
        // bit 31 set (out of range) for chunks past the end of k, without a branch
        const uint32_t out = (uint32_t)(K - 4 - c - k0) >> 31;
        const uint32_t off = ((uint32_t)(r * ld + k0 + c) * 4u) | (out << 31);
        pf.v[ps] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    }
}

// Pass ps of f64_bload.
__device__ __forceinline__ void f64_bload1(F64Raw& pf, __amdgpu_buffer_rsrc_t rs, int ld, int k0, int K, int ps)
{
    const int idx = ps * 512 + threadIdx.x;
    const int r = idx >> 3, c = (idx & 7) * 4;
    const uint32_t out = (uint32_t)(K - 4 - c - k0) >> 31;
    const uint32_t off = ((uint32_t)(r * ld + k0 + c) * 4u) | (out << 31);
    pf.v[ps] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
}

// Convert and write one stage's panel to LDS (row r, 4 doubles).  The
// residues stay in [0, p): one conversion per value, no centring; the
// launcher only picks this kernel when k (p - 1)^2 stays below 2^53.
__device__ __forceinline__ void f64_dstore(double* __restrict__ lds, const F64Raw& pf)
{
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
        const int idx = ps * 512 + threadIdx.x;
        const int r = idx >> 3, c = (idx & 7) * 4;
        const v4u v = pf.v[ps];
        v4d d;
        d.x = (double)v.x;
        d.y = (double)v.y;
        d.z = (double)v.z;
        d.w = (double)v.w;
        *reinterpret_cast<v4d*>(lds + r * PD + c) = d;
    }
}

// Pass ps of f64_dstore.
__device__ __forceinline__ void f64_dstore1(double* __restrict__ lds, const F64Raw& pf, int ps)
{
    const int idx = ps * 512 + threadIdx.x;
    const int r = idx >> 3, c = (idx & 7) * 4;
    const v4u v = pf.v[ps];
    v4d d;
    d.x = (double)v.x;
    d.y = (double)v.y;
    d.z = (double)v.z;
    d.w = (double)v.w;
    *reinterpret_cast<v4d*>(lds + r * PD + c) = d;
}

template <int N> using IntC = std::integral_constant<int, N>;
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(IntC<B>{});
        static_for<B + 1, E>(f);
    }
}
}  // namespace

__device__ __forceinline__ void f64_pipe_tile(const ProdArgs& args, int b)
{
    constexpr int NW = 8;
    using G = F64Lds<NW>;
    constexpr int WM2 = G::WM, WN2 = G::WN;     // 4 x 2 blocks of 16 x 16
    __shared__ __attribute__((aligned(16))) double sa[2][BM2 * PD];
    __shared__ __attribute__((aligned(16))) double sb[2][BM2 * PD];
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) tri_index(r, &ti, &tj);
    else { ti = r / t.tn; tj = r - ti * t.tn; }
    const int tile_r = ti * BM2, tile_c = tj * BM2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave / G::WCOLS, wc = wave % G::WCOLS;
    const int lr = lane & 15, lk = lane >> 4;
    const double pd = (double)t.p;
    const int K = t.k;
    const int nk = (K + BK2 - 1) / BK2;

    v4d acc[WM2][WN2];
#pragma unroll
    for (int i = 0; i < WM2; ++i)
#pragma unroll
        for (int j = 0; j < WN2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    if (nk > 0) {
        const int va = t.m - tile_r < BM2 ? t.m - tile_r : BM2;
        const int vb = t.n - tile_c < BM2 ? t.n - tile_c : BM2;
        const int lda = __builtin_amdgcn_readfirstlane((int)t.A.ld);
        const int ldb = __builtin_amdgcn_readfirstlane((int)t.B.ld);
        const __amdgpu_buffer_rsrc_t ra =
            f64_panel_rsrc((const uint32_t*)t.A.p + (int64_t)tile_r * t.A.ld, (int64_t)va * t.A.ld * 4);
        const __amdgpu_buffer_rsrc_t rb =
            f64_panel_rsrc((const uint32_t*)t.B.p + (int64_t)tile_c * t.B.ld, (int64_t)vb * t.B.ld * 4);

        // fragments: lane (lr, lk) holds k = 4 lk .. 4 lk + 3 of its row in a k-group
        auto read_frags = [&](v4d (&xa)[WM2], v4d (&xb)[WN2], int buf, int kg) {
#pragma unroll
            for (int i = 0; i < WM2; ++i)
                xa[i] = *reinterpret_cast<const v4d*>(&sa[buf][(wr * 64 + i * 16 + lr) * PD + kg * 16 + 4 * lk]);
#pragma unroll
            for (int j = 0; j < WN2; ++j)
                xb[j] = *reinterpret_cast<const v4d*>(&sb[buf][(wc * G::WTN + j * 16 + lr) * PD + kg * 16 + 4 * lk]);
        };
        auto mfmas = [&](const v4d (&xa)[WM2], const v4d (&xb)[WN2]) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int i = 0; i < WM2; ++i)
#pragma unroll
                    for (int j = 0; j < WN2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[i][s4], xb[j][s4], acc[i][j], 0, 0, 0);
        };
        constexpr int NMF = 4 * WM2 * WN2;          // MFMAs per k-group
        constexpr int NRD = 2 * (WM2 + WN2);        // 16-byte LDS reads per k-group

        F64Raw a0, b0, a1, b1;
        f64_bload(a0, ra, lda, 0, K);
        f64_bload(b0, rb, ldb, 0, K);
        f64_bload(a1, ra, lda, BK2, K);
        f64_bload(b1, rb, ldb, BK2, K);
        f64_dstore(sa[0], a0);
        f64_dstore(sb[0], b0);
        __syncthreads();
        v4d fa[WM2], fb[WN2];
        read_frags(fa, fb, 0, 0);

        // One k-group: its 32 MFMAs with the NOPS other operations between
        // them in a fixed order (a scheduling barrier after each).  Left to
        // the compiler's grouping the LDS writes and reads clustered between
        // MFMAs, which then waited for them (7 % slower).
        auto kgroup = [&](const v4d (&xa)[WM2], const v4d (&xb)[WN2], auto nops, auto&& op) {
            constexpr int NOPS = decltype(nops)::value;
            static_for<0, 4 * WM2 * WN2>([&](auto q) {
                constexpr int Q = decltype(q)::value;
                constexpr int S4 = Q / (WM2 * WN2), I = (Q / WN2) % WM2, J = Q % WN2;
                acc[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[I][S4], xb[J][S4], acc[I][J], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                static_for<Q * NOPS / (4 * WM2 * WN2), (Q + 1) * NOPS / (4 * WM2 * WN2)>([&](auto o) {
                    op(o);
                    __builtin_amdgcn_sched_barrier(0);
                });
            });
        };
        // fragment o of k-group kg: A blocks 0..WM2-1, then B blocks
        auto rd1 = [&](v4d (&xa)[WM2], v4d (&xb)[WN2], int buf, int kg, int o) {
            if (o < WM2)
                xa[o] = *reinterpret_cast<const v4d*>(&sa[buf][(wr * 64 + o * 16 + lr) * PD + kg * 16 + 4 * lk]);
            else
                xb[o - WM2] = *reinterpret_cast<const v4d*>(
                    &sb[buf][(wc * G::WTN + (o - WM2) * 16 + lr) * PD + kg * 16 + 4 * lk]);
        };
        auto stage = [&](auto par, int kt) {
            constexpr int cur = decltype(par)::value;
            F64Raw& la = cur ? a1 : a0;   // reloaded now (its stage is in LDS)
            F64Raw& lb = cur ? b1 : b0;
            F64Raw& wa = cur ? a0 : a1;   // stage kt + 1, written now
            F64Raw& wb = cur ? b0 : b1;
            v4d na[WM2], nb[WN2];
            // k-group 0: the fragments of k-group 1, stage kt + 1 converted
            // into the free LDS buffer, the loads of stage kt + 2
            static_assert(WM2 + WN2 == 6, "the operation order below assumes 6 fragments");
            kgroup(fa, fb, std::integral_constant<int, 14>{}, [&](auto o) {
                constexpr int O = decltype(o)::value;
                if constexpr (O % 2 == 0 && O < 12) rd1(na, nb, cur, 1, O / 2);
                else if constexpr (O == 1) f64_dstore1(sa[cur ^ 1], wa, 0);
                else if constexpr (O == 3) f64_dstore1(sa[cur ^ 1], wa, 1);
                else if constexpr (O == 5) f64_dstore1(sb[cur ^ 1], wb, 0);
                else if constexpr (O == 7) f64_dstore1(sb[cur ^ 1], wb, 1);
                else if constexpr (O == 9) f64_bload1(la, ra, lda, (kt + 2) * BK2, K, 0);
                else if constexpr (O == 11) f64_bload1(la, ra, lda, (kt + 2) * BK2, K, 1);
                else if constexpr (O == 12) f64_bload1(lb, rb, ldb, (kt + 2) * BK2, K, 0);
                else f64_bload1(lb, rb, ldb, (kt + 2) * BK2, K, 1);
            });
            __syncthreads();
            // k-group 1 with the first fragments of stage kt + 1
            kgroup(na, nb, std::integral_constant<int, 6>{},
                   [&](auto o) { rd1(fa, fb, cur ^ 1, 0, decltype(o)::value); });
        };
        for (int kt = 0; kt < nk; kt += 2) {
            stage(std::integral_constant<int, 0>{}, kt);
            stage(std::integral_constant<int, 1>{}, kt + 1);
        }
    }

    const double alpha = (double)t.alpha, beta = (double)t.beta;
#pragma unroll
    for (int i = 0; i < WM2; ++i) {
#pragma unroll
        for (int j = 0; j < WN2; ++j) {
            const int col = tile_c + wc * G::WTN + j * 16 + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = tile_r + wr * 64 + i * 16 + 4 * e + lk;
                if (row >= t.m || col >= t.n) continue;
                if (t.syrk && col > row) continue;
                uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                double v = mod_f64(acc[i][j][e], pd, t.pinv);
                double x = alpha * v;
                if (t.beta != 0u) x += beta * (double)(*dst);
                *dst = (uint32_t)mod_f64(x, pd, t.pinv);
            }
        }
    }
}

__global__ __launch_bounds__(512) void prod_f64_pipe_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) f64_pipe_tile(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) f64_pipe_tile(args, b);
}

// mode 0: one workgroup per tile; 1: same, XCD-aware order; 2: persistent
// (workgroups stride over the tiles, which are ordered longest first).
__global__ __launch_bounds__(256) void prod_f64_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) f64_tile(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) f64_tile(args, b);
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void prod_f64_lds_kernel(ProdArgs args, int mode)
{
    if (mode == 2) {
        for (int b = blockIdx.x; b < args.total_tiles; b += gridDim.x) f64_lds_tile<NW>(args, b);
        return;
    }
    const int b = mode == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b < args.total_tiles) f64_lds_tile<NW>(args, b);
}

int64_t f64_kblk(uint32_t p)
{
    const double half = (double)((p - 1) / 2);
    const double lim = 9007199254740992.0 - 2.0 * (double)p;  // 2^53 minus slack
    double kb = half > 0 ? floor(lim / (half * half)) : 1e18;
    if (kb > (double)(1 << 30)) kb = (double)(1 << 30);
    int64_t k = (int64_t)kb;
    k -= k % 16;
    // p above 2^25: fewer than 16 columns fit; the 64 x 64 tile then reduces
    // after every 4-column matrix-core step (a reduced accumulator plus four
    // centred products stays below p + (p-1)^2 < 2^53 for p <= kMaxPrime)
    if (k < 16) k = 4;
    return k;
}

// Delayed-reduction block of a task for a kernel that reduces every `unit`
// columns (16 or 32); blocks under 16 columns stay as they are (only the
// 64 x 64 tile runs them).
static int32_t task_kblk(uint32_t p, int unit)
{
    const int64_t kb = f64_kblk(p);
    return kb < 16 ? (int32_t)kb : cap_kblk(kb, unit);
}

int g_f64_pipe = 1;

template <int TILE>
static hipError_t launch_f64_impl(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    ProdArgs args{};
    int total = 0;
    for (int i = 0; i < ntasks; ++i) {
        ProdTask& t = tasks[i];
        t.kblk = task_kblk(t.p, TILE == 128 ? BK2 : 16);
        t.tm = (t.m + TILE - 1) / TILE;
        t.tn = (t.n + TILE - 1) / TILE;
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
    const bool w8 = TILE == 128;
    // the doubles-in-LDS variant: whole k in one exact block, 16-byte rows,
    // 128-row panels addressable with 32-bit byte offsets
    bool pipe = w8 && g_f64_pipe != 0;
    for (int i = 0; i < ntasks && pipe; ++i) {
        const ProdTask& t = tasks[i];
        const double pm1 = (double)(t.p - 1);
        pipe = t.k <= t.kblk && (double)t.k * pm1 * pm1 < 9007199254740992.0 - 2.0 * (double)t.p &&
               (t.k & 3) == 0 && (t.A.ld & 3) == 0 && (t.B.ld & 3) == 0 &&
               (((uintptr_t)t.A.p) & 15) == 0 && (((uintptr_t)t.B.p) & 15) == 0 && t.A.ld < (1 << 22) &&
               t.B.ld < (1 << 22);
    }
    const void* kern = TILE != 128 ? (const void*)prod_f64_kernel
                       : pipe      ? (const void*)prod_f64_pipe_kernel
                                   : (const void*)prod_f64_lds_kernel<8>;
    const int threads = w8 ? 512 : 256;
    if (mode == 2) {
        const int resident = resident_blocks(kern, threads);
        grid = total < resident ? total : resident;
    }
    g_last_variant = TILE == 128 ? (pipe ? 11 : 8) : 0;
    if (TILE != 128)
        hipLaunchKernelGGL(prod_f64_kernel, dim3(grid), dim3(256), 0, s, args, mode);
    else if (pipe)
        hipLaunchKernelGGL(prod_f64_pipe_kernel, dim3(grid), dim3(512), 0, s, args, mode);
    else
        hipLaunchKernelGGL((prod_f64_lds_kernel<8>), dim3(grid), dim3(512), 0, s, args, mode);
    return hipGetLastError();
}

bool prepare_f64_tile_task(ProdTask* t)
{
    t->kblk = task_kblk(t->p, 16);
    t->tm = (t->m + kF64TileM - 1) / kF64TileM;
    t->tn = (t->n + kF64TileN - 1) / kF64TileN;
    t->tile0 = 0;
    return true;
}

int g_f64_tile_override = 0;

hipError_t launch_products_f64(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    // 128 x 128 tiles (half the operand traffic per flop) once they alone
    // give every CU at least two workgroups; 64 x 64 tiles otherwise.
    int64_t tiles128 = 0;
    for (int i = 0; i < ntasks; ++i) {
        const int64_t tm = (tasks[i].m + 127) / 128, tn = (tasks[i].n + 127) / 128;
        tiles128 += tasks[i].syrk ? tm * (tm + 1) / 2 : tm * tn;
    }
    bool big = tiles128 >= 512;
    const int ov = g_tile_hint ? g_tile_hint : g_f64_tile_override;
    if (ov == 64) big = false;
    if (ov == 128) big = true;
    // the 128 x 128 kernels reduce once per 32-column stage at most often
    for (int i = 0; i < ntasks; ++i)
        if (f64_kblk(tasks[i].p) < BK2) big = false;
    return big ? launch_f64_impl<128>(tasks, ntasks, dev_task_buf, s)
               : launch_f64_impl<64>(tasks, ntasks, dev_task_buf, s);
}

}  // namespace ffp
