// Kernels of the LDL^T factorisation (Section 5): leaf factorisation,
// unit-lower triangular solve, and Algorithm 5's factorisation D = Delta
// Delta^T (square roots of residues, Algorithm 4 on pairs of non-residues)
// applied as column operations on L21.
#include "ldlt.h"
#include "modp.h"
#include "prod_f64_tile.h"
#include "prod_i8_tile.h"

namespace ffp {

namespace {

constexpr int NB = kLdltLeaf;   // leaf order and triangular-solve block

// In-place LDL^T of an nb x nb block (nb <= NB) in LDS, followed (when
// every pivot is nonzero) by the inverse of its unit lower triangular
// factor, written to linv (row i at linv + 64 i, columns <= i), which the
// triangular solves against this block use.  kb: number of products of two
// residues whose sum stays below 2^53.
//
// The elimination is division-free, so no modular inverse sits on the
// sequential path: step k replaces M[i][j] by a_k M[i][j] - M[i][k] M[j][k]
// (i >= j > k) with a_k = M[k][k].  By induction M = g_k S_k on the
// trailing block, where S_k is the true Schur complement and
// g_k = a_0 ... a_{k-1}; hence D[k] = a_k / g_k and L[i][k] = M[i][k] / a_k
// (M taken at step k), and a_k = 0 exactly when the true pivot is 0.  The
// inverses are then formed in parallel.  The inverse of L is built from its
// 8 x 8 diagonal blocks up: [[A, 0], [B, C]]^-1 = [[A^-1, 0], [-C^-1 B A^-1,
// C^-1]] on blocks of 8, 16 and 32.
struct LeafLds {
    uint32_t sm[NB][NB + 1];
    uint32_t li[NB][NB + 1];
    uint32_t tq[NB][NB + 1];
    uint32_t ainv[NB];
    __attribute__((aligned(16))) double colk[2][NB];
};

// The residue in [0, p) of a double congruent to it in [-p, 2p).
__device__ __forceinline__ double canon(double x, double pd)
{
    return x < 0.0 ? x + pd : (x >= pd ? x - pd : x);
}

__device__ __forceinline__ void ldlt_leaf_body(Fp f, int kb, int nb, uint32_t* S, int64_t lds, int64_t* info,
                                               int64_t offset, uint32_t* linv, LeafLds& L)
{
    auto& sm = L.sm;
    auto& li = L.li;
    auto& tq = L.tq;
    auto& ainv = L.ainv;
    auto& colk = L.colk;
    const uint32_t p = f.p;
    const double pd = (double)p, pinv = f.pinv;
    const int tid = threadIdx.x;
    // The elimination keeps the whole (symmetric, both triangles) block in
    // registers: thread t owns the 4 x 4 block of rows r0.. r0+3 and columns
    // c0.. c0+3.  Step k only needs column k, which its 16 owners publish
    // in LDS (double-buffered, one barrier per step); by symmetry M[j][k] is
    // the column entry of row j.  Entries are kept as doubles congruent to
    // their residue in [-p, 2p) (one quotient estimate, no correction):
    // a M[i][j] - M[i][k] M[j][k] then stays below 8 p^2 < 2^53, so every
    // product is exact; entries are brought into [0, p) at the end, the
    // pivot at every step for the zero test.  For p >= 2^25 every entry is
    // brought into [0, p) after each update instead.
    const int r0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;
    const bool big = p >= (1u << 25);
    double m[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = r0 + a, j = c0 + b;
            uint32_t v = 0u;
            if (i < nb && j < nb) v = j <= i ? S[(int64_t)i * lds + j] : S[(int64_t)j * lds + i];
            m[a][b] = (double)v;
        }
    if (c0 == 0)
#pragma unroll
        for (int a = 0; a < 4; ++a) colk[0][r0 + a] = m[a][0];
    __syncthreads();
    bool stop = false;
    for (int k0 = 0; k0 < nb && !stop; k0 += 4) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = k0 + kk;
            if (k >= nb) break;
            const double* col = colk[k & 1];
            const double a = col[k];
            if (canon(a, pd) == 0.0) {
                if (tid == 0 && *info == 0) *info = offset + k + 1;
                stop = true;                          // every thread read the same a
                break;
            }
            double ci[4], cj[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                ci[x] = col[r0 + x];
                cj[x] = col[c0 + x];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    if (r0 + x > k && c0 + y > k) {
                        const double v = fma(a, m[x][y], -(ci[x] * cj[y]));   // |v| < 8 p^2
                        m[x][y] = fma(-floor(v * pinv), pd, v);               // in [-p, 2p)
                        // p >= 2^25: 8 p^2 passes 2^53, so entries stay in
                        // [0, p) (then |v| < p^2 < 2^53)
                        if (big) m[x][y] = canon(m[x][y], pd);
                    }
            // owners of column k + 1 publish it for the next step
            if (kk < 3) {
                if (c0 == k0)
#pragma unroll
                    for (int x = 0; x < 4; ++x) colk[(k + 1) & 1][r0 + x] = m[x][kk + 1];
            } else {
                if (c0 == k0 + 4)
#pragma unroll
                    for (int x = 0; x < 4; ++x) colk[(k + 1) & 1][r0 + x] = m[x][0];
            }
            __syncthreads();
        }
    }
    if (!stop) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = r0 + a, j = c0 + b;
                if (i < nb && j <= i) sm[i][j] = (uint32_t)canon(m[a][b], pd);
            }
    }
    __syncthreads();
    if (stop) return;   // contents unspecified after a zero pivot
    // D[k] = a_k / g_k, L[i][k] = M[i][k] / a_k
    uint32_t dk = 0u;
    if (tid < nb) {
        const int k = tid;
        uint32_t g = 1u;
        for (int t = 0; t < k; ++t) g = mul_m(g, sm[t][t], p, pinv);
        const uint32_t a = sm[k][k];
        ainv[k] = pow_m(a, p - 2, p, pinv);
        dk = mul_m(a, pow_m(g, p - 2, p, pinv), p, pinv);
    }
    __syncthreads();                 // every a_k read before D overwrites the diagonal
    if (tid < nb) sm[tid][tid] = dk;
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j < i) sm[i][j] = mul_m(sm[i][j], ainv[j], p, pinv);
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j <= i) S[(int64_t)i * lds + j] = sm[i][j];
    }
    // inverse of the unit lower factor; rows and columns past nb act as an
    // identity block.  Strict lower entries of L: lo(i, j).
    auto lo = [&](int i, int j) -> uint32_t { return (i < nb && j < nb) ? sm[i][j] : 0u; };
    // 8 x 8 diagonal blocks by forward substitution, one column per thread
    if (tid < NB) {
        const int q = tid >> 3, c = tid & 7, b0 = q * 8;
        li[b0 + c][b0 + c] = 1u;
        for (int i = c + 1; i < 8; ++i) {
            double acc = 0.0;
            int cnt = 1;
            for (int t = c; t < i; ++t) {   // at most 7 terms
                acc = fma((double)lo(b0 + i, b0 + t), (double)li[b0 + t][b0 + c], acc);
                if (++cnt == kb) { acc = (double)mod53(acc, p, pinv); cnt = 1; }
            }
            const uint32_t v = mod53(acc, p, pinv);
            li[b0 + i][b0 + c] = v == 0u ? 0u : p - v;
        }
    }
    __syncthreads();
    for (int b = 8; b < NB; b *= 2) {
        const int pairs = NB / (2 * b);
        // T = B A^-1 for each pair: B = L[C rows][A cols], A^-1 lower triangular
        for (int e = tid; e < pairs * b * b; e += blockDim.x) {
            const int q = e / (b * b), rem = e - q * b * b, i = rem / b, j = rem - i * b;
            const int a0 = q * 2 * b, c0 = a0 + b;
            double acc = 0.0;
            int cnt = 1;   // slots of a block: the (reduced) accumulator and kb - 1 products
            for (int t = j; t < b; ++t) {
                acc = fma((double)lo(c0 + i, a0 + t), (double)li[a0 + t][a0 + j], acc);
                if (++cnt == kb) { acc = (double)mod53(acc, p, pinv); cnt = 1; }
            }
            tq[c0 + i][a0 + j] = mod53(acc, p, pinv);
        }
        __syncthreads();
        // X21 = -C^-1 T
        for (int e = tid; e < pairs * b * b; e += blockDim.x) {
            const int q = e / (b * b), rem = e - q * b * b, i = rem / b, j = rem - i * b;
            const int a0 = q * 2 * b, c0 = a0 + b;
            double acc = 0.0;
            int cnt = 1;
            for (int t = 0; t <= i; ++t) {
                acc = fma((double)li[c0 + i][c0 + t], (double)tq[c0 + t][a0 + j], acc);
                if (++cnt == kb) { acc = (double)mod53(acc, p, pinv); cnt = 1; }
            }
            const uint32_t v = mod53(acc, p, pinv);
            li[c0 + i][a0 + j] = v == 0u ? 0u : p - v;
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j <= i) linv[i * NB + j] = li[i][j];
    }
}

// X <- X L^-T for an nrows x nb block X, given Linv = L^-1 of the unit lower
// triangular nb x nb factor (row i at linv + 64 i, columns <= i):
// X'[r][c] = sum_{t <= c} X[r][t] Linv[c][t].  64 rows per workgroup; each
// thread forms a 4 x 4 block of entries in FP64 with delayed reduction
// (Linv is zero above the diagonal in LDS, so every sum runs over all t).
constexpr int TR = 64;
struct TrsmLds {
    double sl[NB][NB + 1];
    double sx[TR][NB + 1];
};

__device__ __forceinline__ void trsm_inv_body(Fp f, int kb, int64_t nrows, int nb, uint32_t* X, int64_t ldx,
                                              const uint32_t* linv, int lb, TrsmLds& L)
{
    auto& sl = L.sl;
    auto& sx = L.sx;
    const uint32_t p = f.p;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)lb * TR;
    for (int e = tid; e < NB * NB; e += 256) {
        const int i = e / NB, j = e % NB;
        sl[i][j] = (i < nb && j <= i) ? (double)linv[i * NB + j] : 0.0;
    }
    for (int e = tid; e < TR * NB; e += 256) {
        const int i = e / NB, j = e % NB;
        sx[i][j] = (r0 + i < nrows && j < nb) ? (double)X[(r0 + i) * ldx + j] : 0.0;
    }
    __syncthreads();
    const int tr = (tid >> 4) * 4, tc = (tid & 15) * 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    int cnt = 1;   // slots of a block: the (reduced) accumulator and kb - 1 products
    for (int t = 0; t < NB; ++t) {
        double xv[4], lv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) xv[a] = sx[tr + a][t];
#pragma unroll
        for (int b = 0; b < 4; ++b) lv[b] = sl[tc + b][t];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(xv[a], lv[b], acc[a][b]);
        if (++cnt == kb) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = (double)mod53(acc[a][b], p, f.pinv);
            cnt = 1;
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t r = r0 + tr + a;
        if (r >= nrows) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (tc + b < nb) X[r * ldx + tc + b] = mod53(acc[a][b], p, f.pinv);
    }
}

// Per pivot j: non-residue flag, square root of residues, inverse.
__device__ __forceinline__ void classify_body(Fp f, int n1, const uint32_t* S, int64_t lds, uint32_t z,
                                              int32_t* flag, uint32_t* root, uint32_t* dinv, int lb)
{
    const int j = lb * 256 + (int)threadIdx.x;
    if (j >= n1) return;
    const uint32_t d = S[(int64_t)j * lds + j];
    const bool nr = is_nonresidue(d, f.p, f.pinv);
    flag[j] = nr ? 1 : 0;
    root[j] = nr ? 0u : sqrt_m(d, z, f.p, f.pinv);
    dinv[j] = inv_m(d, f.p, f.pinv);
}

// One workgroup of 256 threads: rank the non-residues (prefix count by
// wave ballots), pair them in index order, factor each pair with
// Algorithm 4 and emit the column operations of Algorithm 5 for the n1 + 1
// columns of Abar (the last column is the extra zero column, used when the
// number of non-residues is odd).
//   desc[c] = (j1, s1, j2, s2):  Abar[:, c] = s1 L[:, j1] + s2 L[:, j2]
// (an index of -1 contributes nothing).
struct PairLds {
    int32_t wave_cnt[4];
    int32_t base;
};

__device__ __forceinline__ void pair_body(Fp f, int n1, const uint32_t* S, int64_t lds, const int32_t* flag,
                                          const uint32_t* root, int32_t* rank_idx, uint32_t s_lqnr,
                                          uint32_t c_lqnr, uint32_t z, ColOp* desc, PairLds& L)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t p = f.p;
    if (tid == 0) L.base = 0;
    __syncthreads();
    // ordered list of non-residue indices: rank_idx[r] = j
    for (int c0 = 0; c0 < n1; c0 += 256) {
        const int j = c0 + tid;
        const bool v = j < n1 && flag[j] != 0;
        const uint64_t mask = __ballot(v);
        const int below = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) L.wave_cnt[wv] = __popcll(mask);
        __syncthreads();
        int off = L.base;
        for (int w = 0; w < wv; ++w) off += L.wave_cnt[w];
        if (v) rank_idx[off + below] = j;
        __syncthreads();
        if (tid == 0) L.base += L.wave_cnt[0] + L.wave_cnt[1] + L.wave_cnt[2] + L.wave_cnt[3];
        __syncthreads();
    }
    const int total = L.base;
    const uint32_t s_inv = inv_m(s_lqnr, p, f.pinv);
    // residues: scale by a square root
    for (int j = tid; j < n1; j += 256)
        if (!flag[j]) desc[j] = ColOp{j, root[j], -1, 0u};
    // non-residue pairs (rank 2t, 2t+1); an odd one out pairs with the extra column
    for (int t = tid; 2 * t < total; t += 256) {
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

// Abar (uint32 residues, rows x ncols at X) into three int8 limb planes of
// rows_pad x kpad at Ab (zero padded), for the three-limb Schur product.
__device__ __forceinline__ void pack3_body(const LdltDesc& d, int bx, int by, int gy)
{
    const int64_t c = (int64_t)bx * 64 + (threadIdx.x & 63);
    if (c >= d.kpad) return;
    int8_t* __restrict__ dst = (int8_t*)d.Ab;
    for (int64_t r = (int64_t)by * 4 + (threadIdx.x >> 6); r < d.rows_pad; r += (int64_t)gy * 4) {
        const uint32_t v = (r < d.rows && c < d.ncols) ? d.X[r * d.ldx + c] : 0u;
        const int64_t o = r * d.ldab + c;
        limb3_split(v > d.f.half ? (int)v - (int)d.f.p : (int)v, &dst[o], &dst[d.pplane + o], &dst[2 * d.pplane + o]);
    }
}

// L21 = W D^-1 in place (column j scaled by dinv[j]).
__device__ __forceinline__ void scale_cols_body(Fp f, int64_t rows, int n1, uint32_t* W, int64_t ldw,
                                                const uint32_t* dinv, int bx, int by, int gy)
{
    const int64_t c = (int64_t)bx * 64 + (threadIdx.x & 63);
    if (c >= n1) return;
    const uint32_t s = dinv[c];
    for (int64_t r = (int64_t)by * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gy * 4)
        W[r * ldw + c] = mul_m(W[r * ldw + c], s, f.p, f.pinv);
}

// Abar[:, c] from the column operations (zero beyond ncols, up to kpad).
__device__ __forceinline__ void build_abar_body(Fp f, int64_t rows, int ncols, int kpad, const uint32_t* L,
                                                int64_t ldl, const ColOp* desc, uint32_t* Ab, int64_t ldab,
                                                int bx, int by, int gy)
{
    const int64_t c = (int64_t)bx * 64 + (threadIdx.x & 63);
    if (c >= kpad) return;
    ColOp o = c < ncols ? desc[c] : ColOp{-1, 0u, -1, 0u};
    for (int64_t r = (int64_t)by * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gy * 4) {
        uint32_t v = 0;
        if (o.j1 >= 0) v = mul_m(L[r * ldl + o.j1], o.s1, f.p, f.pinv);
        if (o.j2 >= 0) v = add_m(v, mul_m(L[r * ldl + o.j2], o.s2, f.p, f.pinv), f.p);
        Ab[r * ldab + c] = v;
    }
}

// Algorithm 6, odd characteristic (Section 5.2): B = M Dbar M^T with M
// the identity except for the 2 x 2 blocks of B, where eq. (antidiagonal)
// gives [[0, b], [b, 0]] = [[1, 1], [1, -1]] diag(b/2, -b/2) [[1, 1], [1, -1]]^T,
// so A B A^T = Abar Dbar Abar^T with Abar = A M:
//   first column j of a block:  Abar_j = A_j + A_(j+1),  Dbar_j = b/2
//   second column:              Abar_(j+1) = A_j - A_(j+1),  Dbar_(j+1) = -b/2
//   scalar block:               Abar_j = A_j,  Dbar_j = B_jj.
// B is given by its diagonal bd (n) and off-diagonal bo (n - 1); bo[j] != 0
// marks the block (j, j + 1).  One workgroup.  *info (if not null) is the
// 1-based index of the first column of a malformed block (two blocks
// overlapping, a nonzero diagonal entry inside a 2 x 2 block, an entry not
// below p), else 0.
struct BdiagLds {
    int32_t wave_min[4];
};

__device__ __forceinline__ void bdiag_body(Fp f, int n, const uint32_t* bd, const uint32_t* bo, ColOp* desc1,
                                           uint32_t* dbar, int64_t* info, BdiagLds& L)
{
    const uint32_t p = f.p, half = (p + 1u) / 2u;   // the inverse of 2
    int bad = 0x7FFFFFFF;
    for (int j = threadIdx.x; j < n; j += 256) {
        const uint32_t prev = j > 0 ? bo[j - 1] : 0u;
        const uint32_t next = j + 1 < n ? bo[j] : 0u;
        const uint32_t dj = bd[j];
        if (dj >= p || prev >= p || next >= p) bad = min(bad, j);
        if (next != 0u) {
            if (prev != 0u || dj != 0u || bd[j + 1] != 0u) bad = min(bad, j);
            desc1[j] = ColOp{j, 1u, j + 1, 1u};
            dbar[j] = mul_m(next, half, p, f.pinv);
        } else if (prev != 0u) {
            desc1[j] = ColOp{j - 1, 1u, j, p - 1u};
            dbar[j] = sub_m(0u, mul_m(prev, half, p, f.pinv), p);
        } else {
            desc1[j] = ColOp{j, 1u, -1, 0u};
            dbar[j] = dj;
        }
    }
    for (int o = 32; o > 0; o >>= 1) bad = min(bad, __shfl_xor(bad, o));
    if ((threadIdx.x & 63) == 0) L.wave_min[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0 && info != nullptr) {
        const int b = min(min(L.wave_min[0], L.wave_min[1]), min(L.wave_min[2], L.wave_min[3]));
        *info = b == 0x7FFFFFFF ? 0 : (int64_t)b + 1;
    }
}

// Abar[:, c] = s1 Abar1_(j1) + s2 Abar1_(j2) for the column ops desc (Algorithm 5
// on Dbar) over the columns Abar1 = A desc1 (Algorithm 6), formed straight
// from A; zero beyond ncols, up to kpad.
__device__ __forceinline__ void build_abar2_body(Fp f, int64_t rows, int ncols, int kpad, const uint32_t* A,
                                                 int64_t lda, const ColOp* desc1, const ColOp* desc,
                                                 uint32_t* Ab, int64_t ldab, int bx, int by, int gy)
{
    const int64_t c = (int64_t)bx * 64 + (threadIdx.x & 63);
    if (c >= kpad) return;
    // up to four columns of A with their factors
    int32_t col[4] = {-1, -1, -1, -1};
    uint32_t fac[4] = {0u, 0u, 0u, 0u};
    if (c < ncols) {
        const ColOp o = desc[c];
        const int32_t js[2] = {o.j1, o.j2};
        const uint32_t ss[2] = {o.s1, o.s2};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (js[u] < 0) continue;
            const ColOp q = desc1[js[u]];
            col[2 * u] = q.j1;
            fac[2 * u] = mul_m(ss[u], q.s1, f.p, f.pinv);
            col[2 * u + 1] = q.j2;
            fac[2 * u + 1] = q.j2 >= 0 ? mul_m(ss[u], q.s2, f.p, f.pinv) : 0u;
        }
    }
    for (int64_t r = (int64_t)by * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gy * 4) {
        uint32_t v = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (col[u] >= 0) v = add_m(v, mul_m(A[r * lda + col[u]], fac[u], f.p, f.pinv), f.p);
        Ab[r * ldab + c] = v;
    }
}

// ---- launches over descriptor arrays ---------------------------------------

// Descriptor owning workgroup b (descriptors sorted by block0; uniform).
__device__ inline int desc_of(const LdltDesc* D, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (D[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int kRowBands = 256;   // scale, abar: at most this many bands of 4 rows per descriptor

__host__ __device__ inline int row_bands(int64_t rows)
{
    const int64_t g = (rows + 3) / 4;
    return (int)(g < 1 ? 1 : (g > kRowBands ? kRowBands : g));
}

// One launch runs the device steps of one level, whatever their kinds:
// workgroup b takes the descriptor whose block range holds b and runs the
// step of its kind (uniform per workgroup).  The steps share one LDS area.
union StepLds {
    LeafLds leaf;
    TrsmLds trsm;
    PairLds pair;
    BdiagLds bdiag;
    int8_t i8[I8Tile<64, 64, 64, 3>::LDS];
};

__global__ __launch_bounds__(256) void ldlt_step_kernel(const LdltDesc* D, int n)
{
    __shared__ __attribute__((aligned(16))) StepLds lds;
    const LdltDesc& d = D[desc_of(D, n, blockIdx.x)];
    const int lb = blockIdx.x - d.block0;
    switch (d.kind) {
    case LK_ZERO:
        if (threadIdx.x == 0) *d.info = 0;
        break;
    case LK_LEAF:
        ldlt_leaf_body(d.f, d.kb, d.nb, d.X, d.ldx, d.info, d.offset, d.linv, lds.leaf);
        break;
    case LK_TRSM:
        trsm_inv_body(d.f, d.kb, d.rows, d.nb, d.X, d.ldx, d.linv, lb, lds.trsm);
        break;
    case LK_CLASSIFY:
        classify_body(d.f, d.nb, d.X, d.ldx, d.s_lqnr, d.sc.flag, d.sc.root, d.sc.dinv, lb);
        break;
    case LK_PAIR:
        pair_body(d.f, d.nb, d.X, d.ldx, d.sc.flag, d.sc.root, d.sc.rank_idx, d.s_lqnr, d.c_lqnr, d.s_lqnr,
                  d.sc.desc, lds.pair);
        break;
    case LK_SCALE:
        scale_cols_body(d.f, d.rows, d.nb, d.X, d.ldx, d.sc.dinv, lb % d.gx, lb / d.gx, row_bands(d.rows));
        break;
    case LK_ABAR:
        build_abar_body(d.f, d.rows, d.ncols, d.kpad, d.X, d.ldx, d.sc.desc, d.Ab, d.ldab, lb % d.gx, lb / d.gx,
                        row_bands(d.rows));
        break;
    case LK_PRODF:
        f64_tile_task(d.t, lb);
        break;
    case LK_PACK3:
        pack3_body(d, lb % d.gx, lb / d.gx, row_bands(d.rows_pad));
        break;
    case LK_PRODL3:
        i8_tile_task<64, 64, 64, 3>(d.t, lb, lds.i8);
        break;
    case LK_BDIAG:
        bdiag_body(d.f, d.nb, d.bd, d.bo, d.desc1, d.dbar, d.info, lds.bdiag);
        break;
    case LK_ABAR2:
        build_abar2_body(d.f, d.rows, d.ncols, d.kpad, d.X, d.ldx, d.desc1, d.sc.desc, d.Ab, d.ldab, lb % d.gx,
                         lb / d.gx, row_bands(d.rows));
        break;
    default:
        break;
    }
}

}  // namespace

int ldlt_dot_block(uint32_t p)
{
    // kb slots per block: the accumulator (a residue below p after each
    // reduction, 0 at the start) and kb - 1 products of two residues, each at
    // most (p-1)^2; the sum stays below 2^53 when (kb - 1)(p-1)^2 + p - 1 does.
    const double pm = (double)(p - 1);
    const double kb = 1.0 + floor((9007199254740991.0 - pm) / (pm * pm + 1.0));
    return kb > 64.0 ? 64 : (kb < 2.0 ? 2 : (int)kb);
}

int ldlt_blocks(int kind, LdltDesc* d)
{
    switch (kind) {
    case LK_ZERO:
    case LK_LEAF:
    case LK_BDIAG:
    case LK_PAIR: return 1;
    case LK_TRSM: return (int)((d->rows + TR - 1) / TR);
    case LK_CLASSIFY: return (d->nb + 255) / 256;
    case LK_SCALE:
        d->gx = (d->nb + 63) / 64;
        return d->rows > 0 ? d->gx * row_bands(d->rows) : 0;
    case LK_ABAR:
    case LK_ABAR2:
        d->gx = (d->kpad + 63) / 64;
        return d->rows > 0 ? d->gx * row_bands(d->rows) : 0;
    case LK_PACK3:
        d->gx = (d->kpad + 63) / 64;
        return d->rows_pad > 0 ? d->gx * row_bands(d->rows_pad) : 0;
    case LK_PRODF:
    case LK_PRODL3:
        return d->t.syrk ? d->t.tm * (d->t.tm + 1) / 2 : d->t.tm * d->t.tn;
    default: return 0;
    }
}

hipError_t launch_ldlt_steps(const LdltDesc* dev, int n, int total_blocks, hipStream_t s)
{
    if (n <= 0 || total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(ldlt_step_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, dev, n);
    return hipGetLastError();
}

}  // namespace ffp
