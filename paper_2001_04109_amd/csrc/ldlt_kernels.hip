// Kernels of the LDL^T factorisation (Section 5): leaf factorisation,
// unit-lower triangular solve, and Algorithm 5's factorisation D = Delta
// Delta^T (square roots of residues, Algorithm 4 on pairs of non-residues)
// applied as column operations on L21.
#include "ldlt.h"
#include "modp.h"

namespace ffp {

namespace {

constexpr int NB = kLdltLeaf;   // leaf order and triangular-solve block

// In-place LDL^T of an nb x nb block held in LDS (nb <= NB), right-looking.
__global__ __launch_bounds__(256) void ldlt_leaf_kernel(Fp f, int nb, uint32_t* S, int64_t lds,
                                                       int64_t* info, int64_t offset)
{
    __shared__ uint32_t s[NB][NB + 1];
    __shared__ uint32_t w[NB], l[NB];
    __shared__ int stop;
    const uint32_t p = f.p;
    const int tid = threadIdx.x;
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j <= i) s[i][j] = S[(int64_t)i * lds + j];
    }
    if (tid == 0) stop = 0;
    __syncthreads();
    int jend = nb;
    for (int j = 0; j < nb; ++j) {
        const uint32_t d = s[j][j];
        if (d == 0) {
            if (tid == 0) {
                stop = 1;
                if (*info == 0) *info = offset + j + 1;
            }
            jend = j;
            break;
        }
        const uint32_t dinv = inv_m(d, p, f.pinv);
        for (int i = j + 1 + tid; i < nb; i += blockDim.x) {
            w[i] = s[i][j];
            l[i] = mul_m(s[i][j], dinv, p, f.pinv);
        }
        __syncthreads();
        // trailing update s[i][c] -= l_i * d * l_c = l_i * w_c  for j < c <= i
        const int r = nb - j - 1;
        for (int e = tid; e < r * r; e += blockDim.x) {
            const int i = j + 1 + e / r, c = j + 1 + e % r;
            if (c <= i) s[i][c] = sub_m(s[i][c], mul_m(l[i], w[c], p, f.pinv), p);
        }
        for (int i = j + 1 + tid; i < nb; i += blockDim.x) s[i][j] = l[i];
        __syncthreads();
    }
    (void)jend;
    __syncthreads();
    if (stop) return;   // contents unspecified after a zero pivot
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j <= i) S[(int64_t)i * lds + j] = s[i][j];
    }
}

// X <- X * L^-T for an nrows x nb block X and an nb x nb unit lower
// triangular L (strict lower part stored; diagonal ignored), nb <= NB.
// 128 rows per block; each thread solves one row in LDS.
constexpr int TR = 128;
__global__ __launch_bounds__(TR) void trsm_leaf_kernel(Fp f, int64_t nrows, int nb, uint32_t* X,
                                                      int64_t ldx, const uint32_t* L, int64_t ldl)
{
    __shared__ uint32_t sl[NB][NB + 1];
    __shared__ uint32_t sx[TR][NB + 1];
    const uint32_t p = f.p;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * TR;
    for (int e = tid; e < nb * nb; e += TR) {
        const int i = e / nb, j = e % nb;
        sl[i][j] = j < i ? L[(int64_t)i * ldl + j] : 0u;
    }
    for (int e = tid; e < TR * nb; e += TR) {
        const int i = e / nb, j = e % nb;
        if (r0 + i < nrows) sx[i][j] = X[(r0 + i) * ldx + j];
    }
    __syncthreads();
    if (r0 + tid < nrows) {
        for (int j = 1; j < nb; ++j) {
            uint32_t acc = sx[tid][j];
            for (int c = 0; c < j; ++c) acc = sub_m(acc, mul_m(sx[tid][c], sl[j][c], p, f.pinv), p);
            sx[tid][j] = acc;
        }
    }
    __syncthreads();
    for (int e = tid; e < TR * nb; e += TR) {
        const int i = e / nb, j = e % nb;
        if (r0 + i < nrows) X[(r0 + i) * ldx + j] = sx[i][j];
    }
}

// Per pivot j: non-residue flag, square root of residues, inverse.
__global__ __launch_bounds__(256) void classify_kernel(Fp f, int n1, const uint32_t* S, int64_t lds,
                                                      uint32_t z, int32_t* flag, uint32_t* root,
                                                      uint32_t* dinv)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n1) return;
    const uint32_t d = S[(int64_t)j * lds + j];
    const bool nr = is_nonresidue(d, f.p, f.pinv);
    flag[j] = nr ? 1 : 0;
    root[j] = nr ? 0u : sqrt_m(d, z, f.p, f.pinv);
    dinv[j] = inv_m(d, f.p, f.pinv);
}

// One workgroup: rank the non-residues (prefix count), pair them in index
// order, factor each pair with Algorithm 4 and emit the column operations
// of Algorithm 5 for the n1 + 1 columns of Abar (the last column is the
// extra zero column, used when the number of non-residues is odd).
//   desc[c] = (j1, s1, j2, s2):  Abar[:, c] = s1 L[:, j1] + s2 L[:, j2]
// (an index of -1 contributes nothing).
__global__ __launch_bounds__(1024) void pair_kernel(Fp f, int n1, const uint32_t* S, int64_t lds,
                                                   const int32_t* flag, const uint32_t* root,
                                                   int32_t* rank_idx, uint32_t s_lqnr,
                                                   uint32_t c_lqnr, uint32_t z, ColOp* desc)
{
    __shared__ int32_t part[1024];
    __shared__ int32_t base;
    const int tid = threadIdx.x;
    const uint32_t p = f.p;
    if (tid == 0) base = 0;
    __syncthreads();
    // ordered list of non-residue indices: rank_idx[r] = j
    for (int c0 = 0; c0 < n1; c0 += 1024) {
        const int j = c0 + tid;
        const int v = (j < n1) ? flag[j] : 0;
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int t = (tid >= off) ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += t;
            __syncthreads();
        }
        if (v) rank_idx[base + part[tid] - 1] = j;
        __syncthreads();
        if (tid == 1023) base += part[1023];
        __syncthreads();
    }
    const int total = base;
    const uint32_t s_inv = inv_m(s_lqnr, p, f.pinv);
    // residues: scale by a square root
    for (int j = tid; j < n1; j += 1024)
        if (!flag[j]) desc[j] = ColOp{j, root[j], -1, 0u};
    // non-residue pairs (rank 2t, 2t+1); an odd one out pairs with the extra column
    for (int t = tid; 2 * t < total; t += 1024) {
        const int i = rank_idx[2 * t];
        const bool has_partner = 2 * t + 1 < total;
        const int j = has_partner ? rank_idx[2 * t + 1] : -1;
        const uint32_t al = S[(int64_t)i * lds + i];
        const uint32_t be = has_partner ? S[(int64_t)j * lds + j] : al;
        // Algorithm 3 for the non-residue alpha: alpha = a^2 + b^2 with
        // a = sqrt(alpha / s), b = a * sqrt(s - 1), s the smallest non-residue
        const uint32_t a = sqrt_m(mul_m(al, s_inv, p, f.pinv), z, p, f.pinv);
        const uint32_t b = mul_m(a, c_lqnr, p, f.pinv);
        // Algorithm 4: d = a sqrt(beta / alpha), c = -b d / a
        const uint32_t q = mul_m(be, inv_m(al, p, f.pinv), p, f.pinv);
        const uint32_t d = mul_m(a, sqrt_m(q, z, p, f.pinv), p, f.pinv);
        const uint32_t c = sub_m(0u, mul_m(mul_m(b, d, p, f.pinv), inv_m(a, p, f.pinv), p, f.pinv), p);
        // [Abar_i Abar_j] = [L_i L_j] [[a, b], [c, d]]
        desc[i] = ColOp{i, a, j, c};
        if (has_partner) desc[j] = ColOp{i, b, j, d};
        else desc[n1] = ColOp{i, b, -1, 0u};
    }
    if (tid == 0 && (total & 1) == 0) desc[n1] = ColOp{-1, 0u, -1, 0u};
}

// L21 = W D^-1 in place (column j scaled by dinv[j]).
__global__ __launch_bounds__(256) void scale_cols_kernel(Fp f, int64_t rows, int n1, uint32_t* W,
                                                        int64_t ldw, const uint32_t* dinv)
{
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= n1) return;
    const uint32_t s = dinv[c];
    for (int64_t r = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gridDim.y * 4)
        W[r * ldw + c] = mul_m(W[r * ldw + c], s, f.p, f.pinv);
}

// Abar[:, c] from the column operations (zero beyond ncols, up to kpad).
__global__ __launch_bounds__(256) void build_abar_kernel(Fp f, int64_t rows, int ncols, int kpad,
                                                        const uint32_t* L, int64_t ldl,
                                                        const ColOp* desc, uint32_t* Ab,
                                                        int64_t ldab)
{
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= kpad) return;
    ColOp o = c < ncols ? desc[c] : ColOp{-1, 0u, -1, 0u};
    for (int64_t r = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gridDim.y * 4) {
        uint32_t v = 0;
        if (o.j1 >= 0) v = mul_m(L[r * ldl + o.j1], o.s1, f.p, f.pinv);
        if (o.j2 >= 0) v = add_m(v, mul_m(L[r * ldl + o.j2], o.s2, f.p, f.pinv), f.p);
        Ab[r * ldab + c] = v;
    }
}

__global__ void zero_i64_kernel(int64_t* p) { if (threadIdx.x == 0) *p = 0; }

inline dim3 grid2(int64_t rows, int64_t cols)
{
    int64_t gx = (cols + 63) / 64, gy = (rows + 3) / 4;
    if (gy > 16384) gy = 16384;
    return dim3((unsigned)(gx < 1 ? 1 : gx), (unsigned)(gy < 1 ? 1 : gy));
}

}  // namespace

hipError_t launch_zero_i64(int64_t* p, hipStream_t s)
{
    hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_ldlt_leaf(const Fp& f, int nb, uint32_t* S, int64_t lds, int64_t* info,
                            int64_t offset, hipStream_t s)
{
    hipLaunchKernelGGL(ldlt_leaf_kernel, dim3(1), dim3(256), 0, s, f, nb, S, lds, info, offset);
    return hipGetLastError();
}

hipError_t launch_trsm_leaf(const Fp& f, int64_t nrows, int nb, uint32_t* X, int64_t ldx,
                            const uint32_t* L, int64_t ldl, hipStream_t s)
{
    if (nrows <= 0 || nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(trsm_leaf_kernel, dim3((unsigned)((nrows + TR - 1) / TR)), dim3(TR), 0, s, f,
                       nrows, nb, X, ldx, L, ldl);
    return hipGetLastError();
}

hipError_t launch_alg5(const Fp& f, int n1, const uint32_t* S11, int64_t lds, uint32_t s_lqnr,
                       uint32_t c_lqnr, uint32_t z, Alg5Scratch sc, hipStream_t s)
{
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, f, n1,
                       S11, lds, z, sc.flag, sc.root, sc.dinv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pair_kernel, dim3(1), dim3(1024), 0, s, f, n1, S11, lds, sc.flag, sc.root,
                       sc.rank_idx, s_lqnr, c_lqnr, z, sc.desc);
    return hipGetLastError();
}

hipError_t launch_scale_cols(const Fp& f, int64_t rows, int n1, uint32_t* W, int64_t ldw,
                             const uint32_t* dinv, hipStream_t s)
{
    if (rows <= 0 || n1 <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_cols_kernel, grid2(rows, n1), dim3(256), 0, s, f, rows, n1, W, ldw, dinv);
    return hipGetLastError();
}

hipError_t launch_build_abar(const Fp& f, int64_t rows, int ncols, int kpad, const uint32_t* L,
                             int64_t ldl, const ColOp* desc, uint32_t* Ab, int64_t ldab,
                             hipStream_t s)
{
    if (rows <= 0 || kpad <= 0) return hipSuccess;
    hipLaunchKernelGGL(build_abar_kernel, grid2(rows, kpad), dim3(256), 0, s, f, rows, ncols, kpad, L,
                       ldl, desc, Ab, ldab);
    return hipGetLastError();
}

}  // namespace ffp
