// Base-case products on int8 matrix cores (CDNA4 v_mfma_i32_32x32x32_i8).
//
// CLS_I8: centred int8 residues (|x| <= 125 for p <= 251); each product is
// at most 125^2 in magnitude, so an int32 accumulator is exact for more than
// 137 000 columns of k; the accumulators are reduced mod p every `kblk`
// columns and in the epilogue.
//
// CLS_LIMB2: value = 256*hi + lo with int8 limbs; the tile accumulates
// hh = Ahi Bhi^T, ll = Alo Blo^T and x = Ahi Blo^T + Alo Bhi^T in three
// int32 accumulators and combines 2^16 hh + 2^8 x + ll mod p in the
// epilogue.
//
// Both kernels stage A and B tiles through LDS (double-buffered): a 256-
// thread workgroup computes a BM x BN tile, each of its 4 waves a
// (BM/2) x (BN/2) sub-tile of 32 x 32 MFMA blocks.  Every lane feeds one MFMA
// with 16 consecutive k-bytes of one row; A and B use the same lane-to-k
// assignment, so the result is exact whatever the hardware's k order inside
// the instruction.
#include "prod_common.h"

namespace ffp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int BK = 64;          // k bytes per LDS stage
constexpr int LDS_PITCH = BK + 16;   // padded row pitch (bytes), 16-byte aligned

template <int BM, int BN, int PLANES>
struct Smem {
    int8_t a[2][PLANES][BM * LDS_PITCH];
    int8_t b[2][PLANES][BN * LDS_PITCH];
};

__device__ inline int32_t mod_i32(int32_t x, double p, double pinv)
{
    return (int32_t)mod_f64((double)x, p, pinv);
}

// Global -> LDS copy of a ROWS x BK byte tile, 16 bytes per thread per pass.
template <int ROWS>
__device__ inline void stage_tile(int8_t* __restrict__ lds, const int8_t* __restrict__ g, int64_t ld,
                                  int row0, int nrows, int k0)
{
    constexpr int CHUNKS = BK / 16;                 // 16-byte chunks per row
    constexpr int PASSES = ROWS * CHUNKS / 256;
    static_assert(ROWS * CHUNKS % 256 == 0, "tile must split evenly over 256 threads");
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        const int idx = ps * 256 + threadIdx.x;
        const int r = idx / CHUNKS, c = idx % CHUNKS;
        v4i val = {0, 0, 0, 0};
        if (row0 + r < nrows)
            val = *reinterpret_cast<const v4i*>(g + (int64_t)(row0 + r) * ld + k0 + c * 16);
        *reinterpret_cast<v4i*>(lds + r * LDS_PITCH + c * 16) = val;
    }
}

}  // namespace

// PLANES = 1: CLS_I8;  PLANES = 2: CLS_LIMB2.
template <int BM, int BN, int PLANES>
__global__ __launch_bounds__(256) void prod_i8_kernel(ProdArgs args, int remap)
{
    constexpr int WTM = BM / 2, WTN = BN / 2;         // wave tile
    constexpr int FM = WTM / 32, FN = WTN / 32;       // 32x32 blocks per wave
    constexpr int NACC = PLANES == 1 ? 1 : 3;
    __shared__ Smem<BM, BN, PLANES> sm;

    const int b = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b >= args.total_tiles) return;
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
    int ti, tj;
    if (t.syrk) tri_index(r, &ti, &tj);
    else { ti = r / t.tn; tj = r - ti * t.tn; }
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

    // a wave whose sub-tile lies strictly above the diagonal skips the math
    const bool wave_live = !(t.syrk && (tile_c + wc * WTN) > (tile_r + wr * WTM + WTM - 1));

    const int K = t.k;
    const int nk = K / BK;
    if (nk > 0) {
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            stage_tile<BM>(sm.a[0][pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, 0);
            stage_tile<BN>(sm.b[0][pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, 0);
        }
    }
    __syncthreads();
    int since_red = 0;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl) {
                stage_tile<BM>(sm.a[cur ^ 1][pl], Ab + pl * t.A.plane, t.A.ld, tile_r, t.m, (kt + 1) * BK);
                stage_tile<BN>(sm.b[cur ^ 1][pl], Bb + pl * t.B.plane, t.B.ld, tile_c, t.n, (kt + 1) * BK);
            }
        }
        if (wave_live) {
#pragma unroll
            for (int ks = 0; ks < BK / 32; ++ks) {
                v4i fa[PLANES][FM], fb[PLANES][FN];
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl) {
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        fa[pl][i] = *reinterpret_cast<const v4i*>(
                            &sm.a[cur][pl][(wr * WTM + i * 32 + lrow) * LDS_PITCH + ks * 32 + lk * 16]);
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        fb[pl][j] = *reinterpret_cast<const v4i*>(
                            &sm.b[cur][pl][(wc * WTN + j * 32 + lrow) * LDS_PITCH + ks * 32 + lk * 16]);
                }
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        if constexpr (PLANES == 1) {
                            acc[0][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[0][i], fb[0][j], acc[0][i][j], 0, 0, 0);
                        } else {
                            acc[0][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[0][i], fb[0][j], acc[0][i][j], 0, 0, 0);
                            acc[NACC - 2][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[PLANES - 1][i], fb[PLANES - 1][j], acc[NACC - 2][i][j], 0, 0, 0);
                            acc[NACC - 1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[0][i], fb[PLANES - 1][j], acc[NACC - 1][i][j], 0, 0, 0);
                            acc[NACC - 1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[PLANES - 1][i], fb[0][j], acc[NACC - 1][i][j], 0, 0, 0);
                        }
                    }
            }
            since_red += BK;
            if (since_red >= t.kblk && kt + 1 < nk) {
                since_red = 0;
#pragma unroll
                for (int q = 0; q < NACC; ++q)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
#pragma unroll
                            for (int e = 0; e < 16; ++e) acc[q][i][j][e] = mod_i32(acc[q][i][j][e], pd, t.pinv);
            }
        }
        __syncthreads();
    }
    if (!wave_live) return;

    // Epilogue.  32x32 i32 MFMA result layout: lane l, element e holds
    // row 8*(e/4) + 4*(l/32) + e%4, column l%32.
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
                double v;
                if constexpr (PLANES == 1) {
                    v = mod_f64((double)acc[0][i][j][e], pd, t.pinv);
                } else {
                    const double hh = mod_f64((double)acc[0][i][j][e], pd, t.pinv);
                    const double ll = mod_f64((double)acc[NACC - 2][i][j][e], pd, t.pinv);
                    const double xx = mod_f64((double)acc[NACC - 1][i][j][e], pd, t.pinv);
                    v = mod_f64(hh * r16 + xx * r8 + ll, pd, t.pinv);
                }
                uint32_t* dst = t.C + (int64_t)row * t.ldc + col;
                double x = alpha * v;
                if (t.beta != 0u) x += beta * (double)(*dst);
                *dst = (uint32_t)mod_f64(x, pd, t.pinv);
            }
        }
}

namespace {

template <int BM, int BN, int PLANES>
hipError_t launch_i8_impl(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    ProdArgs args{};
    int total = 0;
    for (int i = 0; i < ntasks; ++i) {
        ProdTask& t = tasks[i];
        if ((t.k % BK) != 0 || (t.A.ld % 16) != 0 || (t.B.ld % 16) != 0 ||
            (((uintptr_t)t.A.p) & 15) != 0 || (((uintptr_t)t.B.p) & 15) != 0 ||
            (PLANES == 2 && ((t.A.plane % 16) != 0 || (t.B.plane % 16) != 0)))
            return hipErrorInvalidValue;
        const int64_t half = (t.p - 1) / 2;
        const int64_t per_k = PLANES == 1 ? half * half : 2 * 128 * 128;
        int64_t kb = (2147483647LL - (int64_t)t.p) / (per_k > 0 ? per_k : 1);
        kb -= kb % BK;
        t.kblk = cap_kblk(kb > (1 << 30) ? (1 << 30) : kb, BK);
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
    const int remap = (ntasks == 1) ? 1 : 0;
    const int grid = remap ? (total + 7) / 8 * 8 : total;
    hipLaunchKernelGGL((prod_i8_kernel<BM, BN, PLANES>), dim3(grid), dim3(256), 0, s, args, remap);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_products_i8(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    return launch_i8_impl<128, 128, 1>(tasks, ntasks, dev_task_buf, s);
}

hipError_t launch_products_limb2(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf,
                                 hipStream_t s)
{
    return launch_i8_impl<128, 128, 2>(tasks, ntasks, dev_task_buf, s);
}

}  // namespace ffp
