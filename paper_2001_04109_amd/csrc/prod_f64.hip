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
#include "prod_common.h"

namespace ffp {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

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
            uint4 q = *reinterpret_cast<const uint4*>(src);
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

}  // namespace

__global__ __launch_bounds__(256) void prod_f64_kernel(ProdArgs args, int remap)
{
    const int b = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (b >= args.total_tiles) return;
    ProdTask t;
    select_task(args, b, &t);
    const int r = b - t.tile0;
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
    const bool vec_ok = ((t.A.ld & 3) == 0) && ((t.B.ld & 3) == 0) &&
                        ((((uintptr_t)Ab) & 15) == 0) && ((((uintptr_t)Bb) & 15) == 0);
    const double pd = (double)t.p;
    const int K = t.k;

    v4d acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    Loaded la[WM], lb[WN];
    int since_red = 0;
    for (int kk = 0; kk < K; kk += 16) {
        const int kc = kk + 4 * lk;
#pragma unroll
        for (int i = 0; i < WM; ++i) load4(Ab, t.A.ld, row0 + i * 16 + lr, t.m, kc, K, vec_ok, la[i]);
#pragma unroll
        for (int j = 0; j < WN; ++j) load4(Bb, t.B.ld, col0 + j * 16 + lr, t.n, kc, K, vec_ok, lb[j]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double av[WM], bv[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) av[i] = centred(la[i].v[s], t.half, t.p);
#pragma unroll
            for (int j = 0; j < WN; ++j) bv[j] = centred(lb[j].v[s], t.half, t.p);
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        since_red += 16;
        if (since_red >= t.kblk && kk + 16 < K) {
            since_red = 0;
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[i][j][e] = mod_f64(acc[i][j][e], pd, t.pinv);
        }
    }

    // Epilogue.  16x16 f64 MFMA result layout: element e of lane l is row
    // 4*e + l/16, column l%16.
    const double alpha = (double)t.alpha, beta = (double)t.beta;
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
                double x = alpha * v;
                if (t.beta != 0u) x += beta * (double)(*dst);
                *dst = (uint32_t)mod_f64(x, pd, t.pinv);
            }
        }
    }
}

int64_t f64_kblk(uint32_t p)
{
    const double half = (double)((p - 1) / 2);
    const double lim = 9007199254740992.0 - 2.0 * (double)p;  // 2^53 minus slack
    double kb = half > 0 ? floor(lim / (half * half)) : 1e18;
    if (kb > (double)(1 << 30)) kb = (double)(1 << 30);
    int64_t k = (int64_t)kb;
    k -= k % 16;
    return k;
}

hipError_t launch_products_f64(ProdTask* tasks, int ntasks, ProdTask* dev_task_buf, hipStream_t s)
{
    ProdArgs args{};
    int total = 0;
    for (int i = 0; i < ntasks; ++i) {
        ProdTask& t = tasks[i];
        t.kblk = cap_kblk(f64_kblk(t.p), 16);
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
    hipLaunchKernelGGL(prod_f64_kernel, dim3(grid), dim3(256), 0, s, args, remap);
    return hipGetLastError();
}

}  // namespace ffp
