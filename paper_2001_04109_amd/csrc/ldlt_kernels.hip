// Kernels of the LDL^T factorisation (Section 5): leaf factorisation with
// the classification of its pivots and the inverse of its unit factor, and
// Algorithm 5's factorisation D = Delta Delta^T (square roots of residues,
// Algorithm 4 on pairs of non-residues) applied as column operations.
#include "ldlt.h"
#include "modp.h"
#include "prod_f64_tile.h"
#include "prod_i8_tile.h"

namespace ffp {

namespace {

constexpr int NB = kLdltLeaf;   // leaf order and triangular-solve block

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

// Exclusive prefix product over the 64 lanes of a wave (lane 0: 1).
__device__ __forceinline__ uint32_t wave_prefix_mul(uint32_t v, uint32_t p, double pinv)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)v, d, 64);
        if (lane >= d) v = mul_m(v, u, p, pinv);
    }
    const uint32_t e = (uint32_t)__shfl_up((int)v, 1, 64);
    return lane == 0 ? 1u : e;
}

// Division-free elimination of the block held in registers (see
// ldlt_leaf_body).  BIG: p >= 2^25, entries kept in [0, p).  Returns false
// at a zero pivot (uniform: every thread reads the same pivot).
template <bool BIG>
__device__ __forceinline__ bool leaf_eliminate(double (&m)[4][4], int nb, int r0, int c0, double pd, double pinv,
                                               double (&colk)[2][NB], int64_t* info, int64_t offset)
{
    for (int k0 = 0; k0 < nb; k0 += 4) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = k0 + kk;
            if (k >= nb) break;
            const double* col = colk[k & 1];
            const double a = col[k];
            if (canon(a, pd) == 0.0) {
                if (threadIdx.x == 0 && *info == 0) *info = offset + k + 1;
                return false;
            }
            double ci[4], cj[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                ci[x] = col[r0 + x];
                cj[x] = col[c0 + x];
            }
            // every entry is updated and the rows or columns <= k keep their
            // value by selection, so the 16 updates are independent
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const double v = fma(a, m[x][y], -(ci[x] * cj[y]));   // |v| < 8 p^2
                    double u = fma(-floor(v * pinv), pd, v);                // in [-p, 2p)
                    if constexpr (BIG) u = canon(u, pd);
                    m[x][y] = (r0 + x > k && c0 + y > k) ? u : m[x][y];
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
    return true;
}

// The centred residue of an integer-valued double |v| < 2^53: in
// [-(p + 1)/2, (p + 1)/2] (the rounded quotient is off by at most one only
// next to a half-integer, where either choice stays in that range).
__device__ __forceinline__ double cred(double v, double pd, double pinv)
{
    return fma(-rint(v * pinv), pd, v);
}

// The same elimination for p < 2^18 with entries centred and every second
// step unreduced: after an unreduced step |M| <= (p + 1)^2 / 2, and the next
// step's a M - c c' (pivot and published column always reduced) stays below
// (p + 1)^3 / 4 + (p + 1)^2 / 4 < 2^53.  Entries start centred; the owners of
// the next column reduce it before publishing; every entry is reduced at
// the end.
__device__ __forceinline__ bool leaf_eliminate_lazy(double (&m)[4][4], int nb, int r0, int c0, double pd,
                                                    double pinv, double (&colk)[2][NB], int64_t* info,
                                                    int64_t offset)
{
    for (int k0 = 0; k0 < nb; k0 += 4) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = k0 + kk;
            if (k >= nb) break;
            const double* col = colk[k & 1];
            const double a = col[k];
            if (a == 0.0) {
                if (threadIdx.x == 0 && *info == 0) *info = offset + k + 1;
                return false;
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
                for (int y = 0; y < 4; ++y) {
                    double v = fma(a, m[x][y], -(ci[x] * cj[y]));
                    if (kk & 1) v = cred(v, pd, pinv);
                    m[x][y] = (r0 + x > k && c0 + y > k) ? v : m[x][y];
                }
            if (kk < 3) {
                if (c0 == k0)
#pragma unroll
                    for (int x = 0; x < 4; ++x)
                        colk[(k + 1) & 1][r0 + x] = (kk & 1) ? m[x][kk + 1] : cred(m[x][kk + 1], pd, pinv);
            } else {
                if (c0 == k0 + 4)
#pragma unroll
                    for (int x = 0; x < 4; ++x) colk[(k + 1) & 1][r0 + x] = m[x][0];
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) m[x][y] = cred(m[x][y], pd, pinv);
    return true;
}

// One doubling step of the inverse of the unit lower factor: for each pair
// of consecutive diagonal blocks of size B, [[A, 0], [X, C]]^-1 =
// [[A^-1, 0], [-C^-1 X A^-1, C^-1]] from the inverses of A and C (in li,
// zero above the diagonal).  RED: reduce after every product (p too large
// for B products in one exact sum).
template <int B, bool RED>
__device__ __forceinline__ void leaf_inverse_step(LeafLds& L, uint32_t p, double pinv)
{
    constexpr int PAIRS = NB / (2 * B), NE = PAIRS * B * B;
    constexpr int PER = (NE + 255) / 256;
    const int tid = threadIdx.x;
    // T = X A^-1
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (NE % 256 == 0 || e < NE) {
            const int pr = e / (B * B), rem = e - pr * B * B, i = rem / B, j = rem - i * B;
            const int a0 = pr * 2 * B, c0 = a0 + B;
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const double x = (c0 + i > a0 + t) ? (double)L.sm[c0 + i][a0 + t] : 0.0;
                acc = fma(x, (double)L.li[a0 + t][a0 + j], acc);
                if constexpr (RED) acc = (double)mod53(acc, p, pinv);
            }
            L.tq[c0 + i][a0 + j] = mod53(acc, p, pinv);
        }
    }
    __syncthreads();
    // X' = -C^-1 T
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (NE % 256 == 0 || e < NE) {
            const int pr = e / (B * B), rem = e - pr * B * B, i = rem / B, j = rem - i * B;
            const int a0 = pr * 2 * B, c0 = a0 + B;
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < B; ++t) {
                acc = fma((double)L.li[c0 + i][c0 + t], (double)L.tq[c0 + t][a0 + j], acc);
                if constexpr (RED) acc = (double)mod53(acc, p, pinv);
            }
            const uint32_t v = mod53(acc, p, pinv);
            L.li[c0 + i][a0 + j] = v == 0u ? 0u : p - v;
        }
    }
    __syncthreads();
}

// In-place LDL^T of an nb x nb block (nb <= NB).  The elimination is
// division-free, so no modular inverse sits on the sequential path: step k
// replaces M[i][j] by a_k M[i][j] - M[i][k] M[j][k] (i >= j > k) with
// a_k = M[k][k].  By induction M = g_k S_k on the trailing block, where S_k
// is the true Schur complement and g_k = a_0 ... a_{k-1}; hence
// D[k] = a_k / g_k and L[i][k] = M[i][k] / a_k (M taken at step k), and
// a_k = 0 exactly when the true pivot is 0.
//
// With every pivot nonzero the leaf then writes, when linv is not null,
// the inverse of its unit lower factor to linv (ld ldi; nb x nb, zero above
// the diagonal), built from the diagonal up: [[A, 0], [X, C]]^-1 =
// [[A^-1, 0], [-C^-1 X A^-1, C^-1]] on blocks of 1, 2, 4, ..., 32.
__device__ __forceinline__ void ldlt_leaf_body(const LdltDesc& d, LeafLds& L)
{
    const Fp f = d.f;
    const int nb = d.nb;
    uint32_t* S = d.X;
    const int64_t lds = d.ldx;
    auto& sm = L.sm;
    auto& li = L.li;
    auto& ainv = L.ainv;
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
    double m[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = r0 + a, j = c0 + b;
            uint32_t v = 0u;
            if (i < nb && j < nb) v = j <= i ? S[(int64_t)i * lds + j] : S[(int64_t)j * lds + i];
            m[a][b] = (double)v;
            if (p < (1u << 18) && v > f.half) m[a][b] -= pd;   // centred for the lazy elimination
        }
    if (c0 == 0)
#pragma unroll
        for (int a = 0; a < 4; ++a) L.colk[0][r0 + a] = m[a][0];
    __syncthreads();
    const bool ok = p < (1u << 18)  ? leaf_eliminate_lazy(m, nb, r0, c0, pd, pinv, L.colk, d.info, d.offset)
                    : p >= (1u << 25) ? leaf_eliminate<true>(m, nb, r0, c0, pd, pinv, L.colk, d.info, d.offset)
                                      : leaf_eliminate<false>(m, nb, r0, c0, pd, pinv, L.colk, d.info, d.offset);
    if (!ok) return;   // contents unspecified after a zero pivot
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = r0 + a, j = c0 + b;
            if (i < nb && j <= i) sm[i][j] = (uint32_t)canon(m[a][b], pd);
        }
    __syncthreads();
    // one wave: D[k] = a_k / g_k with 1/g_k the prefix product of the 1/a
    if (tid < 64) {
        const int k = tid;
        const uint32_t a = k < nb ? sm[k][k] : 1u;
        const uint32_t ai = pow_m(a, p - 2, p, pinv);
        const uint32_t gi = wave_prefix_mul(ai, p, pinv);
        ainv[k] = ai;
        if (k < nb) sm[k][k] = mul_m(a, gi, p, pinv);
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j < i) sm[i][j] = mul_m(sm[i][j], ainv[j], p, pinv);
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        if (j <= i) S[(int64_t)i * lds + j] = sm[i][j];
    }
    if (d.linv == nullptr) return;
    // inverse of the unit lower factor; rows and columns past nb act as an
    // identity block
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        li[i][j] = i == j ? 1u : 0u;
        if (i >= nb || j >= nb) sm[i][j] = 0u;
    }
    __syncthreads();
    if (d.kb > NB / 2) {
        leaf_inverse_step<1, false>(L, p, pinv);
        leaf_inverse_step<2, false>(L, p, pinv);
        leaf_inverse_step<4, false>(L, p, pinv);
        leaf_inverse_step<8, false>(L, p, pinv);
        leaf_inverse_step<16, false>(L, p, pinv);
        leaf_inverse_step<32, false>(L, p, pinv);
    } else {
        leaf_inverse_step<1, true>(L, p, pinv);
        leaf_inverse_step<2, true>(L, p, pinv);
        leaf_inverse_step<4, true>(L, p, pinv);
        leaf_inverse_step<8, true>(L, p, pinv);
        leaf_inverse_step<16, true>(L, p, pinv);
        leaf_inverse_step<32, true>(L, p, pinv);
    }
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        d.linv[(int64_t)i * d.ldi + j] = li[i][j];
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

// Algorithm 5 per pivot of a factored leaf (D[k] on the diagonal of X,
// k < nb; pivot j = offset + k of the whole factorisation):
//   flag[j]  1 if D[k] is a quadratic non-residue (Euler's criterion),
//   root[j]  a square root of D[k] for a residue, of D[k] / s for a
//            non-residue (s the smallest non-residue),
//   dinv[j]  the inverse of D[k].
// It runs beside the step after the leaf: the first use of these values is
// the column step of an ancestor, after that ancestor's solve.
__device__ __forceinline__ void leaf_roots_body(const LdltDesc& d)
{
    const int k = threadIdx.x;
    if (k >= d.nb) return;
    const uint32_t p = d.f.p;
    const double pinv = d.f.pinv;
    const uint32_t dk = d.X[(int64_t)k * (d.ldx + 1)];
    const uint32_t x = pow_m(dk, (p - 3) / 2, p, pinv);            // D^((p-3)/2)
    const bool nr = mul_m(x, dk, p, pinv) == p - 1;
    const int64_t j = d.offset + k;
    d.sc.flag[j] = nr ? 1 : 0;
    d.sc.dinv[j] = mul_m(mul_m(x, x, p, pinv), dk, p, pinv);       // D^(p-2)
    d.sc.root[j] = sqrt_m(nr ? mul_m(dk, d.s_inv, p, pinv) : dk, d.s_lqnr, p, pinv);
}

// Algorithm 5 on the n1 pivots of a node (classified by the leaves), with
// L21 = W D1^-1: writes L21 (Y) and Abar = L21 Delta (n1 + 1 columns, zero
// up to kpad) in one pass over W (rows x n1).  Residue pivot j:
// Abar_j = sqrt(D_j) L_j.  The non-residues are paired in index order
// (rank 2t with rank 2t + 1); for a pair (i, j), with r_x = sqrt(D_x / s) and
// c = sqrt(s - 1) (s the smallest non-residue), Algorithm 3 gives
// D_i = a^2 + b^2 with a = r_i, b = c r_i, and Algorithm 4 takes the root
// r_j / r_i of D_j / D_i, so that
//   [Abar_i Abar_j] = [L_i L_j] [[r_i, c r_i], [-c r_j, r_j]],
// whose rows are orthogonal with squared norms D_i, D_j.  An odd one out i
// pairs with the extra column: Abar_i = r_i L_i, Abar_(n1) = c r_i L_i.
// Every workgroup finds the ranks and partners of its 64 columns itself
// (a count and the nearest non-residues outside its block from the
// pivot flags), so no separate pairing step runs.
//   amode 0: Abar as uint32 residues (ldab); 1: as three int8 limb planes
//   (ldab, plane pplane, rows zero-padded to rows_pad).
struct AbarLds {
    int32_t red[3][4];
};

__device__ __forceinline__ void build_abarx_body(const LdltDesc& d, int bx, int by, int gy, AbarLds& L)
{
    const Fp f = d.f;
    const uint32_t p = f.p;
    const int n1 = d.nb;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cb = bx * 64, c = cb + lane;
    const int32_t* flag = d.sc.flag + d.offset;
    const uint32_t* root = d.sc.root + d.offset;
    const uint32_t* dinv = d.sc.dinv + d.offset;
    // non-residues before the block (count, last index) and after it (first index)
    int cnt = 0, prev = -1, next = 0x7FFFFFFF;
    for (int t = tid; t < n1; t += 256) {
        if (t >= cb && t < cb + 64) continue;
        if (flag[t] != 0) {
            if (t < cb) {
                ++cnt;
                prev = t;   // increasing in t
            } else if (next == 0x7FFFFFFF) {
                next = t;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        prev = max(prev, __shfl_xor(prev, o, 64));
        next = min(next, __shfl_xor(next, o, 64));
    }
    if (lane == 0) {
        L.red[0][wv] = cnt;
        L.red[1][wv] = prev;
        L.red[2][wv] = next;
    }
    __syncthreads();
    cnt = L.red[0][0] + L.red[0][1] + L.red[0][2] + L.red[0][3];
    prev = max(max(L.red[1][0], L.red[1][1]), max(L.red[1][2], L.red[1][3]));
    next = min(min(L.red[2][0], L.red[2][1]), min(L.red[2][2], L.red[2][3]));
    // this lane's column: Abar_c = s1 W_j1 + s2 W_j2 (the D^-1 of L folded in)
    const bool nr = c < n1 && flag[c] != 0;
    const uint64_t bal = __ballot(nr);
    const uint64_t lt = (1ull << lane) - 1ull;
    const int rank = cnt + __popcll(bal & lt);
    const uint64_t above = lane == 63 ? 0ull : (bal >> (lane + 1)) << (lane + 1);
    const uint64_t below = bal & lt;
    auto next_nr = [&]() { return above ? cb + __ffsll((long long)above) - 1 : (next < n1 ? next : -1); };
    auto prev_nr = [&]() { return below ? cb + 63 - __clzll(below) : prev; };
    int j1 = -1, j2 = -1;
    uint32_t s1 = 0u, s2 = 0u;
    if (c < n1) {
        const uint32_t rc = root[c], dc = dinv[c];
        if (!nr) {
            j1 = c;
            s1 = mul_m(rc, dc, p, f.pinv);
        } else if ((rank & 1) == 0) {
            j1 = c;
            s1 = mul_m(rc, dc, p, f.pinv);
            const int j = next_nr();
            if (j >= 0) {
                j2 = j;
                s2 = sub_m(0u, mul_m(mul_m(d.c_lqnr, root[j], p, f.pinv), dinv[j], p, f.pinv), p);
            }
        } else {
            const int i = prev_nr();
            j1 = i;
            s1 = mul_m(mul_m(d.c_lqnr, root[i], p, f.pinv), dinv[i], p, f.pinv);
            j2 = c;
            s2 = mul_m(rc, dc, p, f.pinv);
        }
    } else if (c == n1 && (rank & 1) != 0) {
        const int i = prev_nr();   // the odd one out
        j1 = i;
        s1 = mul_m(mul_m(d.c_lqnr, root[i], p, f.pinv), dinv[i], p, f.pinv);
    }
    if (c >= d.kpad) return;
    const uint32_t dself = c < n1 ? dinv[c] : 0u;
    const uint32_t* W = d.X;
    const int64_t rows_out = d.amode == 1 ? d.rows_pad : d.rows;
    // rows in batches of four per thread, their loads issued together
    constexpr int RB = 4;
    for (int64_t rb = (int64_t)by * 4 * RB; rb < rows_out; rb += (int64_t)gy * 4 * RB) {
        uint32_t w1[RB], w2[RB], wc[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int64_t r = rb + 4 * q + wv;
            const bool in = r < d.rows;
            const uint32_t* w = W + (in ? r : 0) * d.ldx;
            w1[q] = (in && j1 >= 0) ? w[j1] : 0u;
            w2[q] = (in && j2 >= 0) ? w[j2] : 0u;
            wc[q] = (in && c < n1) ? w[c] : 0u;
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int64_t r = rb + 4 * q + wv;
            if (r >= rows_out) break;
            const uint32_t v = add_m(mul_m(w1[q], s1, p, f.pinv), mul_m(w2[q], s2, p, f.pinv), p);
            if (r < d.rows && c < n1) d.Y[r * d.ldy + c] = mul_m(wc[q], dself, p, f.pinv);
            if (d.amode == 1) {
                int8_t* dst = (int8_t*)d.Ab;
                const int64_t o = r * d.ldab + c;
                limb3_split(v > f.half ? (int)v - (int)p : (int)v, &dst[o], &dst[d.pplane + o],
                            &dst[2 * d.pplane + o]);
            } else {
                d.Ab[r * d.ldab + c] = v;
            }
        }
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

constexpr int kRowBands = 256;   // LK_ABAR2: at most this many bands of 4 rows per descriptor

__host__ __device__ inline int row_bands(int64_t rows)
{
    const int64_t g = (rows + 3) / 4;
    return (int)(g < 1 ? 1 : (g > kRowBands ? kRowBands : g));
}

// LK_ABARX: bands of 16 rows (one batch of four rows per thread), at most
// 64 bands, since each workgroup first works out the pairing of its 64
// columns from all n1 pivot flags
__host__ __device__ inline int abar_bands(int64_t rows)
{
    const int64_t g = (rows + 15) / 16;
    return (int)(g < 1 ? 1 : (g > 64 ? 64 : g));
}

// One launch runs the device steps of one level, whatever their kinds:
// workgroup b takes the descriptor whose block range holds b and runs the
// step of its kind (uniform per workgroup).  The steps share one LDS area.
union StepLds {
    LeafLds leaf;
    PairLds pair;
    BdiagLds bdiag;
    AbarLds abar;
    int8_t i8[I8Tile<64, 64, 64, 3>::LDS];
};

// D is read-only and never aliased by the steps' stores, so its fields
// need not be read again after a store.
__global__ __launch_bounds__(256) void ldlt_step_kernel(const LdltDesc* __restrict__ D, int n)
{
    __shared__ __attribute__((aligned(16))) StepLds lds;
    const LdltDesc& d = D[desc_of(D, n, blockIdx.x)];
    const int lb = blockIdx.x - d.block0;
    switch (d.kind) {
    case LK_ZERO:
        if (threadIdx.x == 0) *d.info = 0;
        break;
    case LK_LEAF:
        ldlt_leaf_body(d, lds.leaf);
        break;
    case LK_ROOTS:
        leaf_roots_body(d);
        break;
    case LK_CLASSIFY:
        classify_body(d.f, d.nb, d.X, d.ldx, d.s_lqnr, d.sc.flag, d.sc.root, d.sc.dinv, lb);
        break;
    case LK_PAIR:
        pair_body(d.f, d.nb, d.X, d.ldx, d.sc.flag, d.sc.root, d.sc.rank_idx, d.s_lqnr, d.c_lqnr, d.s_lqnr,
                  d.sc.desc, lds.pair);
        break;
    case LK_ABARX:
        build_abarx_body(d, lb % d.gx, lb / d.gx, abar_bands(d.amode == 1 ? d.rows_pad : d.rows), lds.abar);
        break;
    case LK_PRODF: {
        const ProdTask t = d.t;
        switch (d.pform) {
        case TILE_NT_BLOW: f64_tile_task<TILE_NT_BLOW>(t, lb); break;
        case TILE_NN_BLOW: f64_tile_task<TILE_NN_BLOW>(t, lb); break;
        case TILE_NN_ALOW: f64_tile_task<TILE_NN_ALOW>(t, lb); break;
        default: f64_tile_task<TILE_NT>(t, lb); break;
        }
        break;
    }
    case LK_PRODL3: {
        const ProdTask t = d.t;
        i8_tile_task<64, 64, 64, 3>(t, lb, lds.i8);
        break;
    }
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
    case LK_ROOTS:
    case LK_BDIAG:
    case LK_PAIR: return 1;
    case LK_CLASSIFY: return (d->nb + 255) / 256;
    case LK_ABARX: {
        d->gx = (d->kpad + 63) / 64;
        const int64_t rows = d->amode == 1 ? d->rows_pad : d->rows;
        return rows > 0 ? d->gx * abar_bands(rows) : 0;
    }
    case LK_ABAR2:
        d->gx = (d->kpad + 63) / 64;
        return d->rows > 0 ? d->gx * row_bands(d->rows) : 0;
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
