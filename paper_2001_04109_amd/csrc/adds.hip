// Block additions of Algorithm 2 and representation changes.
//
// These kernels are bound by HBM bandwidth: every thread handles a few
// elements with coalesced row-major accesses; transposed accesses (the P4
// versus P4^T reads of the post-additions, the Up/Low copies of Table 4 and
// of the final mirror) go through 32 x 32 LDS tiles so that global traffic
// stays coalesced.
#include "modp.h"
#include "prod_common.h"

#include <initializer_list>

namespace ffp {

namespace {

// ---- class storage access ---------------------------------------------
__device__ inline uint32_t ld_res(int cls, const Fp& f, const DView& v, int64_t i, int64_t j)
{
    if (cls == CLS_F64) return ((const uint32_t*)v.p)[i * v.ld + j];
    if (cls == CLS_I8) {
        int x = ((const int8_t*)v.p)[i * v.ld + j];
        return x < 0 ? (uint32_t)(x + (int)f.p) : (uint32_t)x;
    }
    const int8_t* b = (const int8_t*)v.p;
    int x;
    if (cls == CLS_LIMB3)
        x = (int)b[i * v.ld + j] + 256 * (int)b[v.plane + i * v.ld + j] + 65536 * (int)b[2 * v.plane + i * v.ld + j];
    else
        x = 256 * (int)b[i * v.ld + j] + (int)b[v.plane + i * v.ld + j];
    x %= (int)f.p;
    return x < 0 ? (uint32_t)(x + (int)f.p) : (uint32_t)x;
}

__device__ inline void st_res(int cls, const Fp& f, const DView& v, int64_t i, int64_t j, uint32_t r)
{
    if (cls == CLS_F64) { ((uint32_t*)v.p)[i * v.ld + j] = r; return; }
    if (cls == CLS_I8) {
        int x = r > f.half ? (int)r - (int)f.p : (int)r;
        ((int8_t*)v.p)[i * v.ld + j] = (int8_t)x;
        return;
    }
    if (cls == CLS_LIMB3) {
        int8_t* b = (int8_t*)v.p;
        limb3_split(r > f.half ? (int)r - (int)f.p : (int)r, &b[i * v.ld + j], &b[v.plane + i * v.ld + j],
                    &b[2 * v.plane + i * v.ld + j]);
        return;
    }
    // limb pair with value in [-32896, 32639]
    int x = r <= 32639u ? (int)r : (int)r - (int)f.p;
    int lo = ((x + 128) & 255) - 128;
    int hi = (x - lo) >> 8;
    int8_t* b = (int8_t*)v.p;
    b[i * v.ld + j] = (int8_t)hi;
    b[v.plane + i * v.ld + j] = (int8_t)lo;
}

template <int CLS>
__global__ __launch_bounds__(256) void preadd_s1s2_kernel(Fp f, int64_t m, int64_t h, DView A11,
                                                         DView A21, DView A22, DView S1, DView S2)
{
    const int64_t ncol = f.yb ? h / 2 : h;   // columns, or column pairs (c, c + h/2)
    const int64_t h2 = h / 2;
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= ncol) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        if (f.yb == 0) {
            // Y = a I:  S1 = a (A21 - A11),  S2 = A22 - a A21
            uint32_t a11 = ld_res(CLS, f, A11, i, c), a21 = ld_res(CLS, f, A21, i, c);
            uint32_t a22 = ld_res(CLS, f, A22, i, c);
            uint32_t s1 = mul_m(sub_m(a21, a11, f.p), f.ya, f.p, f.pinv);
            uint32_t s2 = sub_m(a22, mul_m(a21, f.ya, f.p, f.pinv), f.p);
            st_res(CLS, f, S1, i, c, s1);
            st_res(CLS, f, S2, i, c, s2);
        } else {
            // X Y = [a X_L - b X_R, b X_L + a X_R] for Y = [[aI, bI], [-bI, aI]]
            const int64_t cl = c, cr = c + h2;
            uint32_t a11l = ld_res(CLS, f, A11, i, cl), a11r = ld_res(CLS, f, A11, i, cr);
            uint32_t a21l = ld_res(CLS, f, A21, i, cl), a21r = ld_res(CLS, f, A21, i, cr);
            uint32_t a22l = ld_res(CLS, f, A22, i, cl), a22r = ld_res(CLS, f, A22, i, cr);
            uint32_t dl = sub_m(a21l, a11l, f.p), dr = sub_m(a21r, a11r, f.p);
            uint32_t s1l = sub_m(mul_m(dl, f.ya, f.p, f.pinv), mul_m(dr, f.yb, f.p, f.pinv), f.p);
            uint32_t s1r = add_m(mul_m(dl, f.yb, f.p, f.pinv), mul_m(dr, f.ya, f.p, f.pinv), f.p);
            uint32_t tl = sub_m(mul_m(a21l, f.ya, f.p, f.pinv), mul_m(a21r, f.yb, f.p, f.pinv), f.p);
            uint32_t tr = add_m(mul_m(a21l, f.yb, f.p, f.pinv), mul_m(a21r, f.ya, f.p, f.pinv), f.p);
            st_res(CLS, f, S1, i, cl, s1l);
            st_res(CLS, f, S1, i, cr, s1r);
            st_res(CLS, f, S2, i, cl, sub_m(a22l, tl, f.p));
            st_res(CLS, f, S2, i, cr, sub_m(a22r, tr, f.p));
        }
    }
}

template <int CLS>
__global__ __launch_bounds__(256) void preadd_s34_kernel(Fp f, int mode, int64_t m, int64_t h,
                                                        DView S1, DView A22, DView A12, DView S3,
                                                        DView S4)
{
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= h) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        uint32_t s3;
        if (mode & 1) {
            s3 = sub_m(ld_res(CLS, f, S1, i, c), ld_res(CLS, f, A22, i, c), f.p);   // S3 = S1 - A22
            st_res(CLS, f, S3, i, c, s3);
        } else {
            s3 = ld_res(CLS, f, S3, i, c);
        }
        if (mode & 2) {
            uint32_t s4 = add_m(s3, ld_res(CLS, f, A12, i, c), f.p);               // S4 = S3 + A12
            st_res(CLS, f, S4, i, c, s4);
        }
    }
}

// FP64 class (uint32 residues) with 4 consecutive columns per thread; the
// launchers take these when every row start is 16-byte aligned and the
// column count (of pairs, for Y = [[aI, bI], [-bI, aI]]) is a multiple of 4.
__device__ __forceinline__ uint4 ld4(const DView& v, int64_t i, int64_t j)
{
    return *reinterpret_cast<const uint4*>((const uint32_t*)v.p + i * v.ld + j);
}

__device__ __forceinline__ void st4(const DView& v, int64_t i, int64_t j, uint4 x)
{
    *reinterpret_cast<uint4*>((uint32_t*)v.p + i * v.ld + j) = x;
}

__device__ __forceinline__ uint32_t comp(const uint4& x, int e) { return e == 0 ? x.x : e == 1 ? x.y : e == 2 ? x.z : x.w; }

__global__ __launch_bounds__(256) void preadd_s1s2_u32x4_kernel(Fp f, int64_t m, int64_t h, DView A11, DView A21,
                                                               DView A22, DView S1, DView S2)
{
    const int64_t ncol = f.yb ? h / 2 : h;
    const int64_t h2 = h / 2;
    const int64_t c = ((int64_t)blockIdx.x * 64 + (threadIdx.x & 63)) * 4;
    if (c >= ncol) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        if (f.yb == 0) {
            const uint4 a11 = ld4(A11, i, c), a21 = ld4(A21, i, c), a22 = ld4(A22, i, c);
            uint32_t s1[4], s2[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t x11 = comp(a11, e), x21 = comp(a21, e), x22 = comp(a22, e);
                s1[e] = mul_m(sub_m(x21, x11, f.p), f.ya, f.p, f.pinv);
                s2[e] = sub_m(x22, mul_m(x21, f.ya, f.p, f.pinv), f.p);
            }
            st4(S1, i, c, make_uint4(s1[0], s1[1], s1[2], s1[3]));
            st4(S2, i, c, make_uint4(s2[0], s2[1], s2[2], s2[3]));
        } else {
            const int64_t cl = c, cr = c + h2;
            const uint4 a11l = ld4(A11, i, cl), a11r = ld4(A11, i, cr), a21l = ld4(A21, i, cl),
                        a21r = ld4(A21, i, cr), a22l = ld4(A22, i, cl), a22r = ld4(A22, i, cr);
            uint32_t s1l[4], s1r[4], s2l[4], s2r[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t xl = comp(a21l, e), xr = comp(a21r, e);
                const uint32_t dl = sub_m(xl, comp(a11l, e), f.p), dr = sub_m(xr, comp(a11r, e), f.p);
                s1l[e] = sub_m(mul_m(dl, f.ya, f.p, f.pinv), mul_m(dr, f.yb, f.p, f.pinv), f.p);
                s1r[e] = add_m(mul_m(dl, f.yb, f.p, f.pinv), mul_m(dr, f.ya, f.p, f.pinv), f.p);
                const uint32_t tl = sub_m(mul_m(xl, f.ya, f.p, f.pinv), mul_m(xr, f.yb, f.p, f.pinv), f.p);
                const uint32_t tr = add_m(mul_m(xl, f.yb, f.p, f.pinv), mul_m(xr, f.ya, f.p, f.pinv), f.p);
                s2l[e] = sub_m(comp(a22l, e), tl, f.p);
                s2r[e] = sub_m(comp(a22r, e), tr, f.p);
            }
            st4(S1, i, cl, make_uint4(s1l[0], s1l[1], s1l[2], s1l[3]));
            st4(S1, i, cr, make_uint4(s1r[0], s1r[1], s1r[2], s1r[3]));
            st4(S2, i, cl, make_uint4(s2l[0], s2l[1], s2l[2], s2l[3]));
            st4(S2, i, cr, make_uint4(s2r[0], s2r[1], s2r[2], s2r[3]));
        }
    }
}

__global__ __launch_bounds__(256) void preadd_s34_u32x4_kernel(Fp f, int mode, int64_t m, int64_t h, DView S1,
                                                              DView A22, DView A12, DView S3, DView S4)
{
    const int64_t c = ((int64_t)blockIdx.x * 64 + (threadIdx.x & 63)) * 4;
    if (c >= h) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        uint4 s3;
        if (mode & 1) {
            const uint4 x = ld4(S1, i, c), y = ld4(A22, i, c);
            s3 = make_uint4(sub_m(x.x, y.x, f.p), sub_m(x.y, y.y, f.p), sub_m(x.z, y.z, f.p), sub_m(x.w, y.w, f.p));
            st4(S3, i, c, s3);
        } else {
            s3 = ld4(S3, i, c);
        }
        if (mode & 2) {
            const uint4 y = ld4(A12, i, c);
            st4(S4, i, c, make_uint4(add_m(s3.x, y.x, f.p), add_m(s3.y, y.y, f.p), add_m(s3.z, y.z, f.p),
                                     add_m(s3.w, y.w, f.p)));
        }
    }
}

// int8 storage classes (centred int8, two or three int8 limbs) with 16
// consecutive columns per thread: one 16-byte access per plane.  Values are
// decoded to a signed representative x of the residue (|x| < 2^22), the
// block arithmetic runs on exact doubles (every term below 2^53), and the
// result is encoded back to the class's representative (centred; for two
// limbs the one in [-32896, 32639]).  The launchers take these when every
// row start and plane offset is 16-byte aligned and the column count (of
// pairs, for Y = [[aI, bI], [-bI, aI]]) is a multiple of 16.
typedef int v4i __attribute__((ext_vector_type(4)));

template <int CLS>
struct Vec16 {
    static constexpr int PL = CLS == CLS_I8 ? 1 : (CLS == CLS_LIMB2 ? 2 : 3);
    v4i w[PL];
};

template <int CLS>
__device__ __forceinline__ void ld16(const DView& v, int64_t i, int64_t j, Vec16<CLS>& o)
{
#pragma unroll
    for (int q = 0; q < Vec16<CLS>::PL; ++q)
        o.w[q] = *reinterpret_cast<const v4i*>((const int8_t*)v.p + q * v.plane + i * v.ld + j);
}

template <int CLS>
__device__ __forceinline__ void st16(const DView& v, int64_t i, int64_t j, const Vec16<CLS>& o)
{
#pragma unroll
    for (int q = 0; q < Vec16<CLS>::PL; ++q)
        *reinterpret_cast<v4i*>((int8_t*)v.p + q * v.plane + i * v.ld + j) = o.w[q];
}

__device__ __forceinline__ int sbyte(const v4i& w, int e) { return (int)(int8_t)((uint32_t)w[e >> 2] >> (8 * (e & 3))); }

// signed value of element e (a representative of its residue)
template <int CLS>
__device__ __forceinline__ double dec(const Vec16<CLS>& x, int e)
{
    if constexpr (CLS == CLS_I8) return (double)sbyte(x.w[0], e);
    else if constexpr (CLS == CLS_LIMB2) return (double)(256 * sbyte(x.w[0], e) + sbyte(x.w[1], e));
    else return (double)(sbyte(x.w[0], e) + 256 * sbyte(x.w[1], e) + 65536 * sbyte(x.w[2], e));
}

// store the residue of the exact integer v (|v| < 2^53) as element e
template <int CLS>
__device__ __forceinline__ void enc(Vec16<CLS>& x, int e, double v, const Fp& f)
{
    const uint32_t r = (uint32_t)mod_f64(v, (double)f.p, f.pinv);
    int y;
    if constexpr (CLS == CLS_LIMB2) y = r <= 32639u ? (int)r : (int)r - (int)f.p;
    else y = r > f.half ? (int)r - (int)f.p : (int)r;
    const int sh = 8 * (e & 3), wi = e >> 2;
    auto put = [&](int q, int b) {
        uint32_t w = (uint32_t)x.w[q][wi];
        w = (w & ~(0xFFu << sh)) | ((uint32_t)(b & 0xFF) << sh);
        x.w[q][wi] = (int)w;
    };
    if constexpr (CLS == CLS_I8) {
        put(0, y);
    } else if constexpr (CLS == CLS_LIMB2) {
        const int lo = ((y + 128) & 255) - 128;
        put(0, (y - lo) >> 8);
        put(1, lo);
    } else {
        int8_t l, mid, h;
        limb3_split(y, &l, &mid, &h);
        put(0, l);
        put(1, mid);
        put(2, h);
    }
}

template <int CLS>
__global__ __launch_bounds__(256) void preadd_s1s2_vec_kernel(Fp f, int64_t m, int64_t h, DView A11, DView A21,
                                                             DView A22, DView S1, DView S2)
{
    const int64_t ncol = f.yb ? h / 2 : h;
    const int64_t h2 = h / 2;
    const int64_t c = ((int64_t)blockIdx.x * 64 + (threadIdx.x & 63)) * 16;
    if (c >= ncol) return;
    // centred Y entries: a, b small signed integers, products exact in doubles
    const double a = (double)(f.ya > f.half ? (int)f.ya - (int)f.p : (int)f.ya);
    const double b = (double)(f.yb > f.half ? (int)f.yb - (int)f.p : (int)f.yb);
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        if (f.yb == 0) {
            // Y = a I:  S1 = a (A21 - A11),  S2 = A22 - a A21
            Vec16<CLS> x11, x21, x22, s1, s2;
            ld16(A11, i, c, x11);
            ld16(A21, i, c, x21);
            ld16(A22, i, c, x22);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const double v11 = dec(x11, e), v21 = dec(x21, e), v22 = dec(x22, e);
                enc(s1, e, a * (v21 - v11), f);
                enc(s2, e, v22 - a * v21, f);
            }
            st16(S1, i, c, s1);
            st16(S2, i, c, s2);
        } else {
            // X Y = [a X_L - b X_R, b X_L + a X_R]
            const int64_t cl = c, cr = c + h2;
            Vec16<CLS> x11l, x11r, x21l, x21r, x22l, x22r, s1l, s1r, s2l, s2r;
            ld16(A11, i, cl, x11l);
            ld16(A11, i, cr, x11r);
            ld16(A21, i, cl, x21l);
            ld16(A21, i, cr, x21r);
            ld16(A22, i, cl, x22l);
            ld16(A22, i, cr, x22r);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const double xl = dec(x21l, e), xr = dec(x21r, e);
                const double dl = xl - dec(x11l, e), dr = xr - dec(x11r, e);
                enc(s1l, e, a * dl - b * dr, f);
                enc(s1r, e, b * dl + a * dr, f);
                enc(s2l, e, dec(x22l, e) - (a * xl - b * xr), f);
                enc(s2r, e, dec(x22r, e) - (b * xl + a * xr), f);
            }
            st16(S1, i, cl, s1l);
            st16(S1, i, cr, s1r);
            st16(S2, i, cl, s2l);
            st16(S2, i, cr, s2r);
        }
    }
}

template <int CLS>
__global__ __launch_bounds__(256) void preadd_s34_vec_kernel(Fp f, int mode, int64_t m, int64_t h, DView S1,
                                                            DView A22, DView A12, DView S3, DView S4)
{
    const int64_t c = ((int64_t)blockIdx.x * 64 + (threadIdx.x & 63)) * 16;
    if (c >= h) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        Vec16<CLS> s3, t;
        if (mode & 1) {
            Vec16<CLS> x1, x22;
            ld16(S1, i, c, x1);
            ld16(A22, i, c, x22);
#pragma unroll
            for (int e = 0; e < 16; ++e) enc(s3, e, dec(x1, e) - dec(x22, e), f);          // S3 = S1 - A22
            st16(S3, i, c, s3);
        } else {
            ld16(S3, i, c, s3);
        }
        if (mode & 2) {
            Vec16<CLS> x12;
            ld16(A12, i, c, x12);
#pragma unroll
            for (int e = 0; e < 16; ++e) enc(t, e, dec(s3, e) + dec(x12, e), f);           // S4 = S3 + A12
            st16(S4, i, c, t);
        }
    }
}

constexpr int T = 32;

__global__ __launch_bounds__(256) void postadd_kernel(Fp f, int m, const uint32_t* __restrict__ P1,
                                                     int64_t ld1, const uint32_t* __restrict__ P5,
                                                     int64_t ld5, uint32_t* C22, int64_t ld22,
                                                     uint32_t* C21, int64_t ld21, uint32_t beta,
                                                     const uint32_t* __restrict__ up, int64_t ldu,
                                                     const uint32_t* __restrict__ dvec)
{
    __shared__ uint32_t sU1[T][T + 1];   // U1 on tile (bi,bj), lower elements
    __shared__ uint32_t sT[T][T + 1];    // P4^T tile (bi,bj)
    __shared__ uint32_t sTt[T][T + 1];   // P4^T tile (bj,bi)
    __shared__ uint32_t sUp[T][T + 1];   // C11 tile (bj,bi): saved Low(C22)^T
    int bi, bj;
    tri_index(blockIdx.x, &bi, &bj);
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const uint32_t p = f.p;

    for (int rr = ty; rr < T; rr += 8) {
        const int I = bi * T + rr, J = bj * T + tx;        // element of tile (bi,bj)
        const int Jr = bj * T + rr, Ic = bi * T + tx;      // element of tile (bj,bi)
        if (I < m && J < m) {
            sT[rr][tx] = C22[(int64_t)I * ld22 + J];
            if (I >= J) sU1[rr][tx] = add_m(P1[(int64_t)I * ld1 + J], P5[(int64_t)I * ld5 + J], p);
        }
        if (Jr < m && Ic < m) {
            sTt[rr][tx] = C22[(int64_t)Jr * ld22 + Ic];
            if (beta) sUp[rr][tx] = up[(int64_t)Jr * ldu + Ic];
        }
    }
    __syncthreads();

    // lower tile (bi,bj): U4 -> C21, U5 -> C22
    for (int rr = ty; rr < T; rr += 8) {
        const int I = bi * T + rr, J = bj * T + tx;
        if (I >= m || J >= m || I < J) continue;
        const uint32_t u1 = sU1[rr][tx];
        const uint32_t u2 = add_m(u1, sTt[tx][rr], p);                 // + P4[I][J] = P4^T[J][I]
        uint32_t* c21 = C21 + (int64_t)I * ld21 + J;
        *c21 = add_m(u2, *c21, p);                                      // U4 = U2 + P3
        uint32_t u5 = add_m(u2, sT[rr][tx], p);                        // U5 = U2 + P4^T
        if (beta) {
            const uint32_t cin = (I == J) ? dvec[I] : sUp[tx][rr];     // C22_in[I][J]
            u5 = add_m(u5, mul_m(beta, cin, p, f.pinv), p);
        }
        C22[(int64_t)I * ld22 + J] = u5;
    }
    // upper tile (bj,bi): element (J, I) with I > J, U4 only
    for (int rr = ty; rr < T; rr += 8) {
        const int Jr = bj * T + rr, Ic = bi * T + tx;                  // position (Jr, Ic), Ic > Jr
        if (Jr >= m || Ic >= m || Ic <= Jr) continue;
        const uint32_t u1 = sU1[tx][rr];                               // U1[Ic][Jr] (symmetric)
        const uint32_t u2 = add_m(u1, sT[tx][rr], p);                  // + P4[Jr][Ic] = P4^T[Ic][Jr]
        uint32_t* c21 = C21 + (int64_t)Jr * ld21 + Ic;
        *c21 = add_m(u2, *c21, p);
    }
}

__global__ __launch_bounds__(256) void add_lower_kernel(uint32_t p, int64_t m, const uint32_t* X,
                                                       int64_t ldx, const uint32_t* Y, int64_t ldy,
                                                       uint32_t* Z, int64_t ldz)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        if (j > i) continue;
        Z[i * ldz + j] = add_m(X[i * ldx + j], Y[i * ldy + j], p);
    }
}

// dst[J][I] = src[I][J] for I > J (lower tile (bi,bj) -> upper tile (bj,bi));
// dvec[I] = src[I][I] when dvec is not null.
__global__ __launch_bounds__(256) void lower_to_upper_kernel(int m, const uint32_t* src, int64_t lds,
                                                            uint32_t* dst, int64_t ldd,
                                                            uint32_t* dvec)
{
    __shared__ uint32_t s[T][T + 1];
    int bi, bj;
    tri_index(blockIdx.x, &bi, &bj);
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int rr = ty; rr < T; rr += 8) {
        const int I = bi * T + rr, J = bj * T + tx;
        if (I < m && J < m && I >= J) {
            const uint32_t v = src[(int64_t)I * lds + J];
            s[rr][tx] = v;
            if (I == J && dvec) dvec[I] = v;
        }
    }
    __syncthreads();
    for (int rr = ty; rr < T; rr += 8) {
        const int Jr = bj * T + rr, Ic = bi * T + tx;   // destination (Jr, Ic), Ic > Jr
        if (Jr < m && Ic < m && Ic > Jr) dst[(int64_t)Jr * ldd + Ic] = s[tx][rr];
    }
}

template <int SRC, int DST>
__global__ __launch_bounds__(256) void pack_kernel(Fp f, DView src, int64_t n, int64_t k, DView dst,
                                                  int64_t n_pad, int64_t k_pad)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (j >= k_pad) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < n_pad; i += (int64_t)gridDim.y * 4) {
        uint32_t r = (i < n && j < k) ? ld_res(SRC, f, src, i, j) : 0u;
        st_res(DST, f, dst, i, j, r);
    }
}

// Grouped representation change: block b belongs to the descriptor whose
// block range holds it; each block converts 4 rows x 64 columns.
template <int SRC, int DST>
__global__ __launch_bounds__(256) void pack_grouped_kernel(Fp f, const PackDesc* __restrict__ d,
                                                          int nd)
{
    const int b = blockIdx.x;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    const PackDesc q = d[lo];
    Fp g = f;
    g.p = q.p;
    g.half = (q.p - 1) / 2;
    g.pinv = q.pinv;
    const int local = b - q.block0;
    const int64_t bx = (q.k_pad + 63) / 64;
    const int64_t j = (local % bx) * 64 + (threadIdx.x & 63);
    const int64_t i = (local / bx) * 4 + (threadIdx.x >> 6);
    if (j >= q.k_pad || i >= q.n_pad) return;
    uint32_t r = (i < q.n && j < q.k) ? ld_res(SRC, g, q.src, i, j) : 0u;
    st_res(DST, g, q.dst, i, j, r);
}

// Representation change from uint32 residues with 4 columns per thread: a
// block converts 16 rows x 256 columns, each thread reading 4 consecutive
// residues (one 16-byte load when the row allows it) and writing them with
// one store per destination plane (4 bytes for int8 planes, 16 for uint32);
// padding rows and columns get zero.  For the grouped form the block looks
// up its descriptor once for 4096 elements.  The launcher checks that the
// destination rows, planes and k_pad keep those stores aligned.
constexpr int PV_ROWS = 16, PV_COLS = 256;

template <int DST>
__device__ __forceinline__ void pack_vec_store(const PackDesc& q, int64_t i, int64_t j, const uint32_t (&v)[4])
{
    const uint32_t p = q.p, half = (p - 1) / 2;
    if constexpr (DST == CLS_F64) {
        *reinterpret_cast<uint4*>((uint32_t*)q.dst.p + i * q.dst.ld + j) = make_uint4(v[0], v[1], v[2], v[3]);
    } else if constexpr (DST == CLS_I8) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int x = v[e] > half ? (int)v[e] - (int)p : (int)v[e];
            w |= ((uint32_t)x & 255u) << (8 * e);
        }
        *reinterpret_cast<uint32_t*>((int8_t*)q.dst.p + i * q.dst.ld + j) = w;
    } else if constexpr (DST == CLS_LIMB2) {
        uint32_t wh = 0, wl = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int x = v[e] <= 32639u ? (int)v[e] : (int)v[e] - (int)p;
            const int lo = ((x + 128) & 255) - 128;
            const int hi = (x - lo) >> 8;
            wh |= ((uint32_t)hi & 255u) << (8 * e);
            wl |= ((uint32_t)lo & 255u) << (8 * e);
        }
        int8_t* b = (int8_t*)q.dst.p + i * q.dst.ld + j;
        *reinterpret_cast<uint32_t*>(b) = wh;
        *reinterpret_cast<uint32_t*>(b + q.dst.plane) = wl;
    } else {
        uint32_t w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int8_t l, m, h;
            limb3_split(v[e] > half ? (int)v[e] - (int)p : (int)v[e], &l, &m, &h);
            w0 |= ((uint32_t)(uint8_t)l) << (8 * e);
            w1 |= ((uint32_t)(uint8_t)m) << (8 * e);
            w2 |= ((uint32_t)(uint8_t)h) << (8 * e);
        }
        int8_t* b = (int8_t*)q.dst.p + i * q.dst.ld + j;
        *reinterpret_cast<uint32_t*>(b) = w0;
        *reinterpret_cast<uint32_t*>(b + q.dst.plane) = w1;
        *reinterpret_cast<uint32_t*>(b + 2 * q.dst.plane) = w2;
    }
}

template <int DST>
__global__ __launch_bounds__(256) void pack_vec_kernel(const PackDesc* __restrict__ d, int nd, PackDesc one)
{
    const int b = blockIdx.x;
    PackDesc q = one;
    if (d != nullptr) {
        int lo = 0, hi = nd - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].block0 <= b) lo = mid; else hi = mid - 1;
        }
        q = d[lo];
    }
    const int local = b - q.block0;
    const int64_t bx = (q.k_pad + PV_COLS - 1) / PV_COLS;
    const int64_t j = (local % bx) * PV_COLS + (threadIdx.x & 63) * 4;
    const int64_t i0 = (local / bx) * PV_ROWS + (threadIdx.x >> 6);
    if (j >= q.k_pad) return;
    const uint32_t* __restrict__ src = (const uint32_t*)q.src.p;
    const bool vec = (q.src.ld & 3) == 0 && (((uintptr_t)src) & 15) == 0 && j + 4 <= q.k;
#pragma unroll
    for (int rr = 0; rr < PV_ROWS / 4; ++rr) {
        const int64_t i = i0 + 4 * rr;
        if (i >= q.n_pad) break;
        uint32_t v[4] = {0u, 0u, 0u, 0u};
        if (i < q.n) {
            const uint32_t* row = src + i * q.src.ld;
            if (vec) {
                const uint4 x = *reinterpret_cast<const uint4*>(row + j);
                v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = j + e < q.k ? row[j + e] : 0u;
            }
        }
        pack_vec_store<DST>(q, i, j, v);
    }
}

// Linear combination out = sum of +-in[i] mod p of uint32 residue blocks
// (the additions of Strassen-Winograd): 4 columns per thread when every row
// start is 16-byte aligned, else one.  Each term is added or subtracted
// with one conditional correction, so the result stays in [0, p).
struct LinIn { const uint32_t* p[5]; int64_t ld[5]; };

template <int VEC>
__global__ __launch_bounds__(256) void lincomb_kernel(uint32_t p, int64_t m, int64_t k, int nin, LinIn in,
                                                     unsigned neg, uint32_t* __restrict__ out, int64_t ldo)
{
    const int64_t j = ((int64_t)blockIdx.x * 64 + (threadIdx.x & 63)) * VEC;
    if (j >= k) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < m; i += (int64_t)gridDim.y * 4) {
        uint32_t acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = 0u;
        for (int t = 0; t < nin; ++t) {
            uint32_t v[VEC];
            const uint32_t* row = in.p[t] + i * in.ld[t] + j;
            if constexpr (VEC == 4) {
                const uint4 x = *reinterpret_cast<const uint4*>(row);
                v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
            } else {
                v[0] = row[0];
            }
            const bool sub = (neg >> t) & 1u;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] = sub ? sub_m(acc[e], v[e], p) : add_m(acc[e], v[e], p);
        }
        uint32_t* o = out + i * ldo + j;
        if constexpr (VEC == 4) *reinterpret_cast<uint4*>(o) = make_uint4(acc[0], acc[1], acc[2], acc[3]);
        else o[0] = acc[0];
    }
}

// out = sum_i coef[i] * op_i(in[i]) mod p over an m x k block, op_i the
// identity or the transpose (the additions of the complex products: 3M
// combinations, the multiplication by Y of the pre-additions, the post-
// additions with P4 read transposed).  A workgroup forms a 64 x 64 tile of
// out, each thread 4 consecutive columns of 4 rows; a transposed input goes
// through a 64 x 65 LDS tile so that its global reads stay coalesced.
// Coefficients 1 and p - 1 are a modular addition or subtraction, others a
// modular multiply-add.  VEC: every non-transposed row start and out are
// 16-byte aligned (4 columns per 16-byte access).
struct LctIn { const uint32_t* p[5]; int64_t ld[5]; uint32_t c[5]; };

template <bool VEC>
__global__ __launch_bounds__(256) void lct_kernel(uint32_t p, double pinv, int64_t m, int64_t k, int nin, LctIn in,
                                                  unsigned trans, int lower, uint32_t* __restrict__ out, int64_t ldo)
{
    __shared__ uint32_t tl[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    if (lower && c0 > r0 + 63) return;     // the whole tile above the diagonal (uniform)
    const int tid = threadIdx.x;
    const int cx = (tid & 15) * 4, ry = tid >> 4;           // columns cx..cx+3 of rows ry + 16 e
    uint32_t acc[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[e][u] = 0u;
    auto fold = [&](uint32_t& a, uint32_t v, uint32_t cf) {
        if (cf == 1u) a = add_m(a, v, p);
        else if (cf == p - 1u) a = sub_m(a, v, p);
        else a = add_m(a, mul_m(cf, v, p, pinv), p);
    };
    for (int t = 0; t < nin; ++t) {
        const uint32_t cf = in.c[t];
        if (cf == 0u) continue;
        if ((trans >> t) & 1u) {
            // out[r][c] += cf * in[c][r]: stage rows c0.., columns r0.. of in
            __syncthreads();
            for (int e = tid; e < 64 * 64; e += 256) {
                const int a = e >> 6, b = e & 63;
                const int64_t sr = c0 + a, sc = r0 + b;
                tl[a][b] = (sr < k && sc < m) ? in.p[t][sr * in.ld[t] + sc] : 0u;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int u = 0; u < 4; ++u) fold(acc[e][u], tl[cx + u][ry + 16 * e], cf);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t r = r0 + ry + 16 * e, c = c0 + cx;
                if (r >= m) continue;
                const uint32_t* src = in.p[t] + r * in.ld[t] + c;
                uint32_t v[4];
                if (VEC && c + 4 <= k) {
                    const uint4 x = *reinterpret_cast<const uint4*>(src);
                    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = c + u < k ? src[u] : 0u;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) fold(acc[e][u], v[u], cf);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t r = r0 + ry + 16 * e, c = c0 + cx;
        if (r >= m) continue;
        uint32_t* dst = out + r * ldo + c;
        if (VEC && c + 4 <= k && (!lower || c + 3 <= r)) {
            *reinterpret_cast<uint4*>(dst) = make_uint4(acc[e][0], acc[e][1], acc[e][2], acc[e][3]);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c + u < k && (!lower || c + u <= r)) dst[u] = acc[e][u];
        }
    }
}

// Up(C) <- -Low(C)^T mod p, through 32 x 32 LDS tiles (as lower_to_upper_kernel).
__global__ __launch_bounds__(256) void lower_to_upper_neg_kernel(uint32_t p, int m, uint32_t* C, int64_t ldc)
{
    __shared__ uint32_t s[T][T + 1];
    int bi, bj;
    tri_index(blockIdx.x, &bi, &bj);
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int rr = ty; rr < T; rr += 8) {
        const int I = bi * T + rr, J = bj * T + tx;
        if (I < m && J < m && I >= J) s[rr][tx] = C[(int64_t)I * ldc + J];
    }
    __syncthreads();
    for (int rr = ty; rr < T; rr += 8) {
        const int Jr = bj * T + rr, Ic = bi * T + tx;
        if (Jr < m && Ic < m && Ic > Jr) {
            const uint32_t v = s[tx][rr];
            C[(int64_t)Jr * ldc + Ic] = v == 0u ? 0u : p - v;
        }
    }
}

__global__ __launch_bounds__(256) void copy_u32_kernel(int64_t rows, int64_t cols, const uint32_t* src,
                                                      int64_t lds, uint32_t* dst, int64_t ldd,
                                                      int lower_only)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (j >= cols) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < rows; i += (int64_t)gridDim.y * 4) {
        if (lower_only && j > i) continue;
        dst[i * ldd + j] = src[i * lds + j];
    }
}

// Pseudo-random residues (splitmix64 of the element index and a seed, mod
// p) in the storage of the operand: uint32 in [0,p), centred int8, or two
// int8 limb planes (256 hi + lo); for the autotuner's synthetic operands.
__global__ __launch_bounds__(256) void fill_residues_kernel(int64_t rows, int64_t cols, void* dst, int64_t ld,
                                                           int64_t plane, int dtype, uint32_t p, uint64_t seed)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (j >= cols) return;
    for (int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); i < rows; i += (int64_t)gridDim.y * 4) {
        uint64_t z = seed + (uint64_t)(i * cols + j) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const uint32_t r = (uint32_t)(z % p);
        if (dtype == 0) {
            ((uint32_t*)dst)[i * ld + j] = r;
            continue;
        }
        const int32_t x = r > (p - 1) / 2 ? (int32_t)r - (int32_t)p : (int32_t)r;
        if (dtype == 1) {
            ((int8_t*)dst)[i * ld + j] = (int8_t)x;
        } else {
            const int32_t lo = ((x + 128) & 255) - 128;
            ((int8_t*)dst)[i * ld + j] = (int8_t)((x - lo) >> 8);
            ((int8_t*)dst)[plane + i * ld + j] = (int8_t)lo;
        }
    }
}

inline dim3 grid2d(int64_t rows, int64_t cols)
{
    int64_t gx = (cols + 63) / 64;
    int64_t gy = (rows + 3) / 4;
    if (gy > 16384) gy = 16384;
    if (gx < 1) gx = 1;
    if (gy < 1) gy = 1;
    return dim3((unsigned)gx, (unsigned)gy);
}

// every view's rows start 16-byte aligned and the column count is a multiple of 4
inline bool u32x4_ok(int64_t ncol, std::initializer_list<DView> views)
{
    if (!g_pack_vec || (ncol & 3) != 0) return false;
    for (const DView& v : views)
        if ((v.ld & 3) != 0 || (((uintptr_t)v.p) & 15) != 0) return false;
    return true;
}

// int8 storage: every row start and plane offset 16-byte aligned, column count a multiple of 16
inline bool i8x16_ok(int64_t ncol, std::initializer_list<DView> views)
{
    if (!g_pack_vec || (ncol & 15) != 0) return false;
    for (const DView& v : views)
        if ((v.ld & 15) != 0 || (((uintptr_t)v.p) & 15) != 0 || (v.plane & 15) != 0) return false;
    return true;
}

inline unsigned tri_blocks(int64_t m)
{
    const int64_t t = (m + T - 1) / T;
    return (unsigned)(t * (t + 1) / 2);
}

}  // namespace

hipError_t launch_preadd_s1s2(int cls, const Fp& f, int64_t m, int64_t h, DView A11, DView A21,
                              DView A22, DView S1, DView S2, hipStream_t s)
{
    if (m <= 0 || h <= 0) return hipSuccess;
    const int64_t ncol = f.yb ? h / 2 : h;
    if (cls == CLS_F64 && u32x4_ok(ncol, {A11, A21, A22, S1, S2})) {
        hipLaunchKernelGGL(preadd_s1s2_u32x4_kernel, grid2d(m, ncol / 4), dim3(256), 0, s, f, m, h, A11, A21, A22,
                           S1, S2);
        return hipGetLastError();
    }
    if (cls != CLS_F64 && i8x16_ok(ncol, {A11, A21, A22, S1, S2})) {
        const dim3 g = grid2d(m, ncol / 16);
        switch (cls) {
        case CLS_I8: hipLaunchKernelGGL(preadd_s1s2_vec_kernel<CLS_I8>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
        case CLS_LIMB2: hipLaunchKernelGGL(preadd_s1s2_vec_kernel<CLS_LIMB2>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
        default: hipLaunchKernelGGL(preadd_s1s2_vec_kernel<CLS_LIMB3>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
        }
        return hipGetLastError();
    }
    dim3 g = grid2d(m, ncol);
    switch (cls) {
    case CLS_F64: hipLaunchKernelGGL(preadd_s1s2_kernel<CLS_F64>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
    case CLS_I8: hipLaunchKernelGGL(preadd_s1s2_kernel<CLS_I8>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
    case CLS_LIMB2: hipLaunchKernelGGL(preadd_s1s2_kernel<CLS_LIMB2>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
    default: hipLaunchKernelGGL(preadd_s1s2_kernel<CLS_LIMB3>, g, dim3(256), 0, s, f, m, h, A11, A21, A22, S1, S2); break;
    }
    return hipGetLastError();
}

hipError_t launch_preadd_s34(int cls, const Fp& f, int mode, int64_t m, int64_t h, DView S1,
                             DView A22, DView A12, DView S3, DView S4, hipStream_t s)
{
    if (m <= 0 || h <= 0) return hipSuccess;
    if (cls == CLS_F64 && u32x4_ok(h, {S1, A22, A12, S3, S4})) {
        hipLaunchKernelGGL(preadd_s34_u32x4_kernel, grid2d(m, h / 4), dim3(256), 0, s, f, mode, m, h, S1, A22, A12,
                           S3, S4);
        return hipGetLastError();
    }
    if (cls != CLS_F64 && i8x16_ok(h, {S1, A22, A12, S3, S4})) {
        const dim3 g = grid2d(m, h / 16);
        switch (cls) {
        case CLS_I8: hipLaunchKernelGGL(preadd_s34_vec_kernel<CLS_I8>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
        case CLS_LIMB2: hipLaunchKernelGGL(preadd_s34_vec_kernel<CLS_LIMB2>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
        default: hipLaunchKernelGGL(preadd_s34_vec_kernel<CLS_LIMB3>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
        }
        return hipGetLastError();
    }
    dim3 g = grid2d(m, h);
    switch (cls) {
    case CLS_F64: hipLaunchKernelGGL(preadd_s34_kernel<CLS_F64>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
    case CLS_I8: hipLaunchKernelGGL(preadd_s34_kernel<CLS_I8>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
    case CLS_LIMB2: hipLaunchKernelGGL(preadd_s34_kernel<CLS_LIMB2>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
    default: hipLaunchKernelGGL(preadd_s34_kernel<CLS_LIMB3>, g, dim3(256), 0, s, f, mode, m, h, S1, A22, A12, S3, S4); break;
    }
    return hipGetLastError();
}

hipError_t launch_postadd(const Fp& f, int64_t m, const uint32_t* P1, int64_t ld1,
                          const uint32_t* P5, int64_t ld5, uint32_t* C22, int64_t ld22,
                          uint32_t* C21, int64_t ld21, uint32_t beta, const uint32_t* up_c11,
                          int64_t ldu, const uint32_t* dvec, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(postadd_kernel, dim3(tri_blocks(m)), dim3(256), 0, s, f, (int)m, P1, ld1, P5,
                       ld5, C22, ld22, C21, ld21, beta, up_c11, ldu, dvec);
    return hipGetLastError();
}

hipError_t launch_add_lower(const Fp& f, int64_t m, const uint32_t* X, int64_t ldx,
                            const uint32_t* Y, int64_t ldy, uint32_t* Z, int64_t ldz,
                            hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(add_lower_kernel, grid2d(m, m), dim3(256), 0, s, f.p, m, X, ldx, Y, ldy, Z, ldz);
    return hipGetLastError();
}

hipError_t launch_save_c22(int64_t m, const uint32_t* C22, int64_t ld22, uint32_t* C11,
                           int64_t ld11, uint32_t* dvec, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(lower_to_upper_kernel, dim3(tri_blocks(m)), dim3(256), 0, s, (int)m, C22, ld22,
                       C11, ld11, dvec);
    return hipGetLastError();
}

hipError_t launch_mirror_lower(int64_t n, uint32_t* C, int64_t ldc, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lower_to_upper_kernel, dim3(tri_blocks(n)), dim3(256), 0, s, (int)n, C, ldc, C,
                       ldc, (uint32_t*)nullptr);
    return hipGetLastError();
}

namespace {
// The 4-column stores of pack_vec_kernel stay aligned for this destination.
bool pack_vec_ok(int src_cls, int dst_cls, const DView& dst, int64_t k_pad)
{
    if (src_cls != CLS_F64 || (k_pad & 3) != 0) return false;
    if (dst_cls == CLS_F64) return (dst.ld & 3) == 0 && (((uintptr_t)dst.p) & 15) == 0;
    return (dst.ld & 3) == 0 && (((uintptr_t)dst.p) & 3) == 0 && (dst_cls == CLS_I8 || (dst.plane & 3) == 0);
}

int64_t pack_vec_blocks(int64_t n_pad, int64_t k_pad)
{
    return ((n_pad + PV_ROWS - 1) / PV_ROWS) * ((k_pad + PV_COLS - 1) / PV_COLS);
}

hipError_t launch_pack_vec(int dst_cls, const PackDesc* dev, int nd, const PackDesc& one, int64_t blocks,
                           hipStream_t s)
{
    switch (dst_cls) {
    case CLS_F64: hipLaunchKernelGGL(pack_vec_kernel<CLS_F64>, dim3((unsigned)blocks), dim3(256), 0, s, dev, nd, one); break;
    case CLS_I8: hipLaunchKernelGGL(pack_vec_kernel<CLS_I8>, dim3((unsigned)blocks), dim3(256), 0, s, dev, nd, one); break;
    case CLS_LIMB2: hipLaunchKernelGGL(pack_vec_kernel<CLS_LIMB2>, dim3((unsigned)blocks), dim3(256), 0, s, dev, nd, one); break;
    default: hipLaunchKernelGGL(pack_vec_kernel<CLS_LIMB3>, dim3((unsigned)blocks), dim3(256), 0, s, dev, nd, one); break;
    }
    return hipGetLastError();
}
}  // namespace

int g_pack_vec = 1;

hipError_t launch_pack(const Fp& f, int src_cls, DView src, int64_t n, int64_t k, int dst_cls,
                       DView dst, int64_t n_pad, int64_t k_pad, hipStream_t s)
{
    if (n_pad <= 0 || k_pad <= 0) return hipSuccess;
    // a single small pack keeps one element per thread (more workgroups for
    // the same latency)
    const int64_t vb = pack_vec_blocks(n_pad, k_pad);
    if (g_pack_vec && pack_vec_ok(src_cls, dst_cls, dst, k_pad) && vb >= 256 && vb < (1LL << 31)) {
        PackDesc one{};
        one.src = src;
        one.dst = dst;
        one.n = n;
        one.k = k;
        one.n_pad = n_pad;
        one.k_pad = k_pad;
        one.p = f.p;
        one.pinv = f.pinv;
        one.block0 = 0;
        return launch_pack_vec(dst_cls, nullptr, 0, one, vb, s);
    }
    dim3 g = grid2d(n_pad, k_pad);
#define FFP_PACK(SC, DC)                                                                       \
    if (src_cls == SC && dst_cls == DC) {                                                      \
        hipLaunchKernelGGL((pack_kernel<SC, DC>), g, dim3(256), 0, s, f, src, n, k, dst, n_pad, \
                           k_pad);                                                             \
        return hipGetLastError();                                                              \
    }
    FFP_PACK(CLS_F64, CLS_F64) FFP_PACK(CLS_F64, CLS_I8) FFP_PACK(CLS_F64, CLS_LIMB2)
    FFP_PACK(CLS_I8, CLS_I8) FFP_PACK(CLS_I8, CLS_F64) FFP_PACK(CLS_LIMB2, CLS_LIMB2)
    FFP_PACK(CLS_LIMB2, CLS_F64) FFP_PACK(CLS_F64, CLS_LIMB3)
#undef FFP_PACK
    return hipErrorInvalidValue;
}

hipError_t launch_pack_grouped(int src_cls, int dst_cls, PackDesc* descs, int nd,
                               PackDesc* dev_descs, hipStream_t s)
{
    bool vec = g_pack_vec != 0;
    int64_t vtotal = 0;
    for (int i = 0; i < nd && vec; ++i) {
        vec = pack_vec_ok(src_cls, dst_cls, descs[i].dst, descs[i].k_pad);
        vtotal += pack_vec_blocks(descs[i].n_pad, descs[i].k_pad);
    }
    if (vec && vtotal > 0 && vtotal < (1LL << 31)) {
        int64_t b0 = 0;
        for (int i = 0; i < nd; ++i) {
            descs[i].block0 = (int32_t)b0;
            b0 += pack_vec_blocks(descs[i].n_pad, descs[i].k_pad);
        }
        hipError_t e = hipMemcpyAsync(dev_descs, descs, sizeof(PackDesc) * nd, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        return launch_pack_vec(dst_cls, dev_descs, nd, PackDesc{}, vtotal, s);
    }
    int total = 0;
    for (int i = 0; i < nd; ++i) {
        descs[i].block0 = total;
        total += (int)(((descs[i].n_pad + 3) / 4) * ((descs[i].k_pad + 63) / 64));
    }
    if (total == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dev_descs, descs, sizeof(PackDesc) * nd, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    Fp f{};
#define FFP_PACKG(SC, DC)                                                                        \
    if (src_cls == SC && dst_cls == DC) {                                                        \
        hipLaunchKernelGGL((pack_grouped_kernel<SC, DC>), dim3(total), dim3(256), 0, s, f,       \
                           (const PackDesc*)dev_descs, nd);                                      \
        return hipGetLastError();                                                                \
    }
    FFP_PACKG(CLS_F64, CLS_F64) FFP_PACKG(CLS_F64, CLS_I8) FFP_PACKG(CLS_F64, CLS_LIMB2)
    FFP_PACKG(CLS_I8, CLS_I8) FFP_PACKG(CLS_LIMB2, CLS_LIMB2) FFP_PACKG(CLS_F64, CLS_LIMB3)
#undef FFP_PACKG
    return hipErrorInvalidValue;
}

hipError_t launch_lincomb(const Fp& f, int64_t m, int64_t k, int nin, const DView* in, unsigned neg, DView out,
                          hipStream_t s)
{
    if (m <= 0 || k <= 0) return hipSuccess;
    if (nin < 1 || nin > 5) return hipErrorInvalidValue;
    LinIn li{};
    bool vec = (k & 3) == 0 && (out.ld & 3) == 0 && (((uintptr_t)out.p) & 15) == 0;
    for (int t = 0; t < nin; ++t) {
        li.p[t] = (const uint32_t*)in[t].p;
        li.ld[t] = in[t].ld;
        vec = vec && (in[t].ld & 3) == 0 && (((uintptr_t)in[t].p) & 15) == 0;
    }
    if (vec) {
        hipLaunchKernelGGL(lincomb_kernel<4>, grid2d(m, k / 4), dim3(256), 0, s, f.p, m, k, nin, li, neg,
                           (uint32_t*)out.p, out.ld);
    } else {
        hipLaunchKernelGGL(lincomb_kernel<1>, grid2d(m, k), dim3(256), 0, s, f.p, m, k, nin, li, neg,
                           (uint32_t*)out.p, out.ld);
    }
    return hipGetLastError();
}

hipError_t launch_lct(const Fp& f, int64_t m, int64_t k, int nin, const DView* in, const uint32_t* coef,
                      unsigned trans, int lower, DView out, hipStream_t s)
{
    if (m <= 0 || k <= 0) return hipSuccess;
    if (nin < 1 || nin > 5 || (lower && m != k)) return hipErrorInvalidValue;
    LctIn li{};
    bool vec = (out.ld & 3) == 0 && (((uintptr_t)out.p) & 15) == 0;
    for (int t = 0; t < nin; ++t) {
        li.p[t] = (const uint32_t*)in[t].p;
        li.ld[t] = in[t].ld;
        li.c[t] = coef[t] % f.p;
        if (!((trans >> t) & 1u)) vec = vec && (in[t].ld & 3) == 0 && (((uintptr_t)in[t].p) & 15) == 0;
    }
    const dim3 g((unsigned)((k + 63) / 64), (unsigned)((m + 63) / 64));
    if (vec)
        hipLaunchKernelGGL(lct_kernel<true>, g, dim3(256), 0, s, f.p, f.pinv, m, k, nin, li, trans, lower,
                           (uint32_t*)out.p, out.ld);
    else
        hipLaunchKernelGGL(lct_kernel<false>, g, dim3(256), 0, s, f.p, f.pinv, m, k, nin, li, trans, lower,
                           (uint32_t*)out.p, out.ld);
    return hipGetLastError();
}

hipError_t launch_mirror_lower_neg(uint32_t p, int64_t n, uint32_t* C, int64_t ldc, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lower_to_upper_neg_kernel, dim3(tri_blocks(n)), dim3(256), 0, s, p, (int)n, C, ldc);
    return hipGetLastError();
}

hipError_t launch_copy_u32(int64_t rows, int64_t cols, const uint32_t* src, int64_t lds,
                           uint32_t* dst, int64_t ldd, int lower_only, hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_u32_kernel, grid2d(rows, cols), dim3(256), 0, s, rows, cols, src, lds, dst,
                       ldd, lower_only);
    return hipGetLastError();
}

hipError_t launch_fill_residues(int64_t rows, int64_t cols, void* dst, int64_t ld, int64_t plane, int dtype,
                                uint32_t p, uint64_t seed, hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_residues_kernel, grid2d(rows, cols), dim3(256), 0, s, rows, cols, dst, ld, plane,
                       dtype, p, seed);
    return hipGetLastError();
}

}  // namespace ffp
