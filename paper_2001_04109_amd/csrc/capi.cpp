// C-ABI entry points of the product library (declared in include/ffp.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "ffp.h"
#include "ffp_debug.h"
#include "field.h"
#include "ldlt.h"
#include "plan.h"
#include "batch.h"
#include "cplan.h"
#include "runtime.h"
#include "serve.h"

using namespace ffp;

namespace {

}  // namespace

extern "C" {

int fsyrk_modp(int64_t n, int64_t k, uint32_t p, const void* A, int64_t lda, int a_dtype,
               uint32_t alpha, uint32_t beta, uint32_t* C, int64_t ldc, unsigned flags, void* stream)
{
    PlanRequest rq;
    int st = make_syrk_request(n, k, p, A, lda, a_dtype, alpha, beta, C, ldc, flags, &rq);
    if (st != FFP_OK) return st;
    if (n == 0) return FFP_OK;
    Plan pl;
    st = build_syrk_plan(rq, &pl);
    if (st != FFP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Workspace* ws = nullptr;
    // large int8 products may split their last round of tiles along k: 64 MiB
    // for the int32 chunks after the plan's own workspace
    const size_t base = ((size_t)pl.ws_bytes + 255) / 256 * 256;
    const size_t tail = (pl.cls == CLS_I8 && pl.n_pad >= 4096 && g_split_tail) ? ((size_t)64 << 20) : 0;
    st = acquire_workspace(s, base + tail, 0, &ws);
    if (st != FFP_OK) return st;
    TailScratchScope scope(tail ? (char*)ws->ptr + base : nullptr, tail);
    return execute_plan(pl, A, C, ws->ptr, s);
}

int fgemm_modp(int64_t m, int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda,
               const uint32_t* B, int64_t ldb, uint32_t alpha, uint32_t beta, uint32_t* C,
               int64_t ldc, void* stream)
{
    if (m < 0 || n < 0 || k < 0) return FFP_EINVAL;
    if (!supported_prime(p)) return FFP_EPRIME;
    if (alpha >= p || beta >= p) return FFP_EINVAL;
    if (m > 0 && n > 0 && (C == nullptr || ldc < n)) return FFP_EINVAL;
    if (m > 0 && n > 0 && k > 0 && (A == nullptr || B == nullptr || lda < k || ldb < k))
        return FFP_EINVAL;
    if (m > (int64_t)1 << 30 || n > (int64_t)1 << 30 || k > (int64_t)1 << 30) return FFP_EINVAL;
    if (m == 0 || n == 0) return FFP_OK;
    FieldPlan f;
    if (!make_field_plan(p, &f)) return FFP_EPRIME;
    ProdTask t{};
    init_task(&t, f);
    t.A = DView{(void*)A, lda, 0};
    t.B = DView{(void*)B, ldb, 0};
    t.C = C;
    t.ldc = ldc;
    t.m = (int32_t)m;
    t.n = (int32_t)n;
    t.k = (int32_t)k;
    t.syrk = 0;
    t.alpha = alpha;
    t.beta = beta;
    hipError_t e = launch_products(CLS_F64, &t, 1, nullptr, (hipStream_t)stream);
    return e == hipSuccess ? FFP_OK : FFP_EDEVICE;
}

size_t ffp_workspace_bytes(int64_t n, int64_t k, uint32_t p, int a_dtype, unsigned flags)
{
    PlanRequest rq;
    const uint32_t beta = (flags & FFP_WS_BETA) ? 1u : 0u;
    int64_t lda = a_dtype == FFP_U32 ? k : ((k + 15) / 16) * 16;
    int64_t ldc = ((n + 3) / 4) * 4;
    if (make_syrk_request(n, k, p, (const void*)16, lda, a_dtype, 1u % p, beta, (const uint32_t*)16, ldc,
                     flags, &rq) != FFP_OK)
        return 0;
    Plan pl;
    if (build_syrk_plan(rq, &pl) != FFP_OK) return 0;
    return (size_t)pl.ws_bytes;
}

const char* ffp_strerror(int status)
{
    switch (status) {
    case FFP_OK: return "ok";
    case FFP_EINVAL: return "invalid argument";
    case FFP_EPRIME: return "modulus not prime or out of range for the path";
    case FFP_EDTYPE: return "operand storage not valid for this modulus";
    case FFP_ENOMEM: return "device workspace allocation failed";
    case FFP_EDEVICE: return "HIP runtime error";
    case FFP_EUNSUPPORTED: return "not supported";
    case FFP_ECANCELED: return "request cancelled";
    case FFP_ETIMEDOUT: return "request deadline passed before admission";
    default: return "unknown status";
    }
}

const char* ffp_version(void) { return "ffp 0.1 (gfx950)"; }

const char* ffp_last_error_detail(void) { return last_error_detail(); }

// ---- introspection (host only; no device work) ---------------------------

int ffp_field_info(uint32_t p, uint32_t* ya, uint32_t* yb, int* ycost)
{
    FieldPlan f;
    if (!make_field_plan(p, &f)) return FFP_EPRIME;
    *ya = f.ya;
    *yb = f.yb;
    *ycost = f.ycost;
    return FFP_OK;
}

int ffp_host_sqrt(uint32_t a, uint32_t p, uint32_t* r)
{
    if (p < 3 || !is_prime_u32(p)) return FFP_EPRIME;
    uint64_t v = sqrt_mod(a, p);
    if (v == UINT64_MAX) return FFP_EINVAL;
    *r = (uint32_t)v;
    return FFP_OK;
}

int ffp_host_sos(uint32_t p, uint32_t k, uint32_t* a, uint32_t* b)
{
    if (p < 3 || !is_prime_u32(p)) return FFP_EPRIME;
    uint64_t x, y;
    sum_of_squares(p, k, &x, &y);
    *a = (uint32_t)x;
    *b = (uint32_t)y;
    return FFP_OK;
}

int ffp_host_nrsyf(uint32_t p, uint32_t alpha, uint32_t beta, uint32_t Y[4])
{
    if (p < 3 || !is_prime_u32(p)) return FFP_EPRIME;
    uint64_t y[4];
    if (!nrsyf(p, alpha, beta, y)) return FFP_EINVAL;
    for (int i = 0; i < 4; ++i) Y[i] = (uint32_t)y[i];
    return FFP_OK;
}

int ffp_plan_describe(int64_t n, int64_t k, uint32_t p, int a_dtype, int64_t lda, int64_t ldc,
                      uint32_t alpha, uint32_t beta, unsigned flags, char* buf, size_t len)
{
    PlanRequest rq;
    int st = make_syrk_request(n, k, p, (const void*)16, lda, a_dtype, alpha, beta, (const uint32_t*)16,
                          ldc, flags, &rq);
    if (st != FFP_OK) return st;
    Plan pl;
    st = build_syrk_plan(rq, &pl);
    if (st != FFP_OK) return st;
    std::string s = describe_plan(pl);
    if (buf && len > 0) {
        size_t c = s.size() < len - 1 ? s.size() : len - 1;
        memcpy(buf, s.data(), c);
        buf[c] = '\0';
    }
    return (int)s.size();
}

namespace {
ComplexRequest complex_request(int64_t n, int64_t k, uint32_t p, int herk, int64_t lda, int64_t a_plane,
                               int64_t ldc, int64_t c_plane, unsigned flags)
{
    ComplexRequest rq;
    rq.n = n;
    rq.k = k;
    rq.p = p;
    rq.herk = herk != 0;
    rq.lda = lda;
    rq.a_plane = a_plane;
    rq.ldc = ldc;
    rq.c_plane = c_plane;
    const unsigned dfield = (flags >> 4) & 0xFu;
    rq.depth = dfield ? (int)dfield - 1 : -1;
    rq.fill_upper = (flags & FFP_FILL_UPPER) != 0;
    return rq;
}
}  // namespace

int ffp_complex_plan_levels(int64_t n, int64_t k, uint32_t p, int herk, int64_t lda, int64_t a_plane,
                            int64_t ldc, int64_t c_plane, unsigned flags, int32_t* levels, size_t cap)
{
    Plan pl;
    const int st = build_complex_plan(complex_request(n, k, p, herk, lda, a_plane, ldc, c_plane, flags), &pl);
    if (st != FFP_OK) return st;
    const void* a = (const void*)((uintptr_t)1 << 44);
    void* c = (void*)((uintptr_t)2 << 44);
    void* ws = (void*)((uintptr_t)3 << 44);
    std::vector<SchedItem> items;
    for (const Op& o : pl.ops) items.push_back(SchedItem{&pl, &o, a, c, ws, 0});
    const std::vector<int> lv = schedule_levels(items);
    if (levels)
        for (size_t i = 0; i < lv.size() && i < cap; ++i) levels[i] = lv[i];
    return (int)lv.size();
}

int ffp_complex_plan_describe(int64_t n, int64_t k, uint32_t p, int herk, int64_t lda, int64_t a_plane,
                              int64_t ldc, int64_t c_plane, unsigned flags, char* buf, size_t len)
{
    ComplexRequest rq;
    rq.n = n;
    rq.k = k;
    rq.p = p;
    rq.herk = herk != 0;
    rq.lda = lda;
    rq.a_plane = a_plane;
    rq.ldc = ldc;
    rq.c_plane = c_plane;
    const unsigned dfield = (flags >> 4) & 0xFu;
    rq.depth = dfield ? (int)dfield - 1 : -1;
    rq.fill_upper = (flags & FFP_FILL_UPPER) != 0;
    Plan pl;
    const int st = build_complex_plan(rq, &pl);
    if (st != FFP_OK) return st;
    std::string s = describe_plan(pl);
    if (buf && len > 0) {
        size_t c = s.size() < len - 1 ? s.size() : len - 1;
        memcpy(buf, s.data(), c);
        buf[c] = '\0';
    }
    return (int)s.size();
}

int ffp_plan_levels(int64_t n, int64_t k, uint32_t p, int a_dtype, int64_t lda, int64_t ldc,
                    uint32_t alpha, uint32_t beta, unsigned flags, int32_t* levels, size_t cap)
{
    PlanRequest rq;
    int st = make_syrk_request(n, k, p, (const void*)16, lda, a_dtype, alpha % (p ? p : 1), beta,
                               (const uint32_t*)16, ldc, flags, &rq);
    if (st != FFP_OK) return st;
    Plan pl;
    st = build_syrk_plan(rq, &pl);
    if (st != FFP_OK) return st;
    // distinct, far-apart stand-in addresses for the three buffers
    const void* a = (const void*)((uintptr_t)1 << 44);
    void* c = (void*)((uintptr_t)2 << 44);
    void* ws = (void*)((uintptr_t)3 << 44);
    std::vector<SchedItem> items;
    for (const Op& o : pl.ops) items.push_back(SchedItem{&pl, &o, a, c, ws, 0});
    const std::vector<int> lv = schedule_levels(items);
    if (levels)
        for (size_t i = 0; i < lv.size() && i < cap; ++i) levels[i] = lv[i];
    return (int)lv.size();
}

}  // extern "C"

extern "C" {

void ffp_debug_set_kblk(int64_t kblk) { ffp::g_kblk_cap = kblk > 0 ? kblk : 0; }

int ffp_debug_set(const char* key, int64_t value)
{
    if (!key) return FFP_EINVAL;
    if (strcmp(key, "kblk") == 0) { ffp::g_kblk_cap = value > 0 ? value : 0; return FFP_OK; }
    if (strcmp(key, "f64_tile") == 0) { ffp::g_f64_tile_override = (int)value; return FFP_OK; }
    if (strcmp(key, "i8_tile") == 0) { ffp::g_i8_tile_override = (int)value; return FFP_OK; }
    if (strcmp(key, "i8_bk") == 0) { ffp::g_i8_bk_override = (int)value; return FFP_OK; }
    if (strcmp(key, "wide") == 0) { ffp::g_wide_schedule = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "winograd_min") == 0) {
        if (value < 0) return FFP_EINVAL;
        ffp::g_winograd_min = value;
        return FFP_OK;
    }
    if (strcmp(key, "leveled") == 0) { ffp::g_leveled = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "merge_products") == 0) { ffp::g_merge_products = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "merge_tiles") == 0) {
        if (value < 0 || value > (1 << 24)) return FFP_EINVAL;
        ffp::g_merge_tiles = (int)value;
        return FFP_OK;
    }
    if (strcmp(key, "i8_dma") == 0) { ffp::g_i8_dma = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "i8_split_tail") == 0) { ffp::g_split_tail = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "l3_dma") == 0) { ffp::g_l3_dma = value < 0 ? 0 : (value > 2 ? 2 : (int)value); return FFP_OK; }
    if (strcmp(key, "i8_pipe") == 0) { ffp::g_i8_pipe = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "pack_vec") == 0) { ffp::g_pack_vec = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "f64_pipe") == 0) { ffp::g_f64_pipe = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "persistent") == 0) { ffp::g_persistent = value < 0 ? 0 : (value > 2 ? 2 : (int)value); return FFP_OK; }
    if (strcmp(key, "ldlt_fold") == 0) { ffp::g_ldlt_fold = value ? 1 : 0; return FFP_OK; }
    if (strcmp(key, "serve_batch") == 0 || strcmp(key, "serve_ldlt_batch") == 0) {
        if (value < 1 || value > 4096) return FFP_EINVAL;
        (key[6] == 'l' ? ffp::g_serve_ldlt_batch : ffp::g_serve_batch) = (int)value;
        return FFP_OK;
    }
    return FFP_EINVAL;
}

void ffp_debug_profile(int enable) { prof_enable(enable != 0); }

int ffp_debug_profile_read(int cls, double* ms, double* flops, int64_t* launches)
{
    return prof_read(cls, ms, flops, launches) == 0 ? FFP_OK : FFP_EDEVICE;
}

int ffp_debug_profile_read_variant(int variant, double* ms, double* flops, int64_t* launches)
{
    return prof_read_variant(-1, variant, ms, flops, launches) == 0 ? FFP_OK : FFP_EDEVICE;
}

const char* ffp_debug_variant_name(int variant)
{
    switch (variant) {
    case 0: return "ffp::prod_f64_kernel(ffp::ProdArgs, int)";
    case 2: return "void ffp::prod_i8_kernel<128, 128, 64, 1>(ffp::ProdArgs, int)";
    case 3: return "void ffp::prod_i8_kernel<256, 256, 64, 1>(ffp::ProdArgs, int)";
    case 4: return "void ffp::prod_i8_kernel<256, 256, 128, 1>(ffp::ProdArgs, int)";
    case 5: return "void ffp::prod_i8_kernel<128, 128, 64, 2>(ffp::ProdArgs, int)";
    case 6: return "void ffp::prod_i8_dma_kernel<1>(ffp::ProdArgs, int)";
    case 7: return "void ffp::prod_i8_dma_kernel<2>(ffp::ProdArgs, int)";
    case 8: return "void ffp::prod_f64_lds_kernel<8>(ffp::ProdArgs, int)";
    case 9: return "void ffp::prod_i8_kernel<64, 64, 64, 3>(ffp::ProdArgs, int)";
    case 10: return "void ffp::prod_i8_pipe_kernel<256, 256, 128, 1>(ffp::ProdArgs, int)";
    case 11: return "ffp::prod_f64_pipe_kernel(ffp::ProdArgs, int)";
    case 12: return "void ffp::prod_i8_pipe_kernel<128, 128, 128, 2>(ffp::ProdArgs, int)";
    case 13: return "ffp::prod_i8_dma_split_kernel(ffp::ProdArgs, int, int, int*)";
    case 14: return "ffp::(anonymous namespace)::prod_l3_dma_kernel(ffp::ProdArgs, int)";
    default: return "";
    }
}

int fldlt_modp(int64_t n, uint32_t p, uint32_t* S, int64_t lds, int64_t* info, void* stream)
{
    if (n < 0 || info == nullptr) return FFP_EINVAL;
    if (p < 3 || !supported_prime(p)) return FFP_EPRIME;
    if (n > 0 && (S == nullptr || lds < n)) return FFP_EINVAL;
    if (n > (int64_t)1 << 30) return FFP_EINVAL;
    return ldlt_run(n, p, S, lds, info, (hipStream_t)stream);
}

namespace {

int complex_syrk(bool herk, int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda, int64_t a_plane,
                 uint32_t* C, int64_t ldc, int64_t c_plane, unsigned flags, void* stream)
{
    if (n < 0 || k < 0) return FFP_EINVAL;
    if (p < 3 || !supported_prime(p)) return FFP_EPRIME;
    if (flags & ~(FFP_FILL_UPPER | 0xF0u)) return FFP_EINVAL;   // fill and depth bits only
    if (n > 0 && (C == nullptr || ldc < n)) return FFP_EINVAL;
    if (n > 0 && k > 0 && (A == nullptr || lda < k)) return FFP_EINVAL;
    if (n > (int64_t)1 << 30 || k > (int64_t)1 << 30) return FFP_EINVAL;
    // the planes of A and of C must not overlap
    if (n > 0 && k > 0 && (a_plane < 0 ? -a_plane : a_plane) < (n - 1) * lda + k) return FFP_EINVAL;
    if (n > 0 && (c_plane < 0 ? -c_plane : c_plane) < (n - 1) * ldc + n) return FFP_EINVAL;
    if (n == 0) return FFP_OK;
    ComplexRequest rq;
    rq.n = n;
    rq.k = k;
    rq.p = p;
    rq.herk = herk;
    rq.lda = lda;
    rq.a_plane = a_plane;
    rq.ldc = ldc;
    rq.c_plane = c_plane;
    const unsigned dfield = (flags >> 4) & 0xFu;
    rq.depth = dfield ? (int)dfield - 1 : -1;
    rq.fill_upper = (flags & FFP_FILL_UPPER) != 0;
    Plan pl;
    int st = build_complex_plan(rq, &pl);
    if (st != FFP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Workspace* ws = nullptr;
    st = acquire_workspace(s, (size_t)pl.ws_bytes, 0, &ws);
    if (st != FFP_OK) return st;
    return execute_plan(pl, A, C, ws->ptr, s);
}

}  // namespace

int fzsyrk_modp(int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda, int64_t a_plane, uint32_t* C,
                int64_t ldc, int64_t c_plane, unsigned flags, void* stream)
{
    return complex_syrk(false, n, k, p, A, lda, a_plane, C, ldc, c_plane, flags, stream);
}

int fherk_modp(int64_t n, int64_t k, uint32_t p, const uint32_t* A, int64_t lda, int64_t a_plane, uint32_t* C,
               int64_t ldc, int64_t c_plane, unsigned flags, void* stream)
{
    return complex_syrk(true, n, k, p, A, lda, a_plane, C, ldc, c_plane, flags, stream);
}

int fsyrkbd_modp(int64_t m, int64_t n, uint32_t p, const uint32_t* A, int64_t lda, const uint32_t* bdiag,
                 const uint32_t* boff, uint32_t alpha, uint32_t beta, uint32_t* C, int64_t ldc, int64_t* info,
                 unsigned flags, void* stream)
{
    if (m < 0 || n < 0) return FFP_EINVAL;
    if (p < 3 || !supported_prime(p)) return FFP_EPRIME;
    if (n > 0 && (A == nullptr || lda < n || bdiag == nullptr || (n > 1 && boff == nullptr))) return FFP_EINVAL;
    if (n > (int64_t)1 << 30) return FFP_EINVAL;
    if (flags & (FFP_BASE_LIMB3 | FFP_WS_BETA)) return FFP_EINVAL;
    // the product on Abar (m x kpad, uint32, in the workspace: 256-byte aligned)
    const int64_t kpad = n > 0 ? syrkbd_kpad(n) : 0;
    PlanRequest rq;
    int st = make_syrk_request(m, kpad, p, (const void*)256, kpad > 0 ? kpad : 1, FFP_U32, alpha, beta, C, ldc,
                               flags, &rq);
    if (st != FFP_OK) return st;
    if (m == 0) return FFP_OK;
    const size_t need = syrkbd_workspace_bytes(m, n, rq);
    if (need == 0) return FFP_EPRIME;
    hipStream_t s = (hipStream_t)stream;
    Workspace* ws = nullptr;
    st = acquire_workspace(s, need, 0, &ws);
    if (st != FFP_OK) return st;
    return syrkbd_run(m, n, p, A, lda, bdiag, boff, rq, C, info, ws->ptr, s);
}

int fldlt_modp_batched(int njobs, const ffp_ldlt_job* jobs, void* stream)
{
    if (njobs < 0 || (njobs > 0 && jobs == nullptr)) return FFP_EINVAL;
    size_t total = 0;
    std::vector<size_t> off((size_t)njobs, 0);
    for (int j = 0; j < njobs; ++j) {
        const ffp_ldlt_job& b = jobs[j];
        if (b.n < 0 || b.info == nullptr || b.n > ((int64_t)1 << 30)) return FFP_EINVAL;
        if (b.p < 3 || !supported_prime(b.p)) return FFP_EPRIME;
        if (b.n > 0 && (b.S == nullptr || b.lds < b.n)) return FFP_EINVAL;
        off[j] = total;
        total += (ldlt_workspace_bytes(b.n, b.p, b.lds) + 255) / 256 * 256;
    }
    if (njobs == 0) return FFP_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace* w = nullptr;
    const int st = acquire_workspace(s, total, 0, &w);
    if (st != FFP_OK) return st;
    std::vector<LdltJobSpec> specs;
    for (int j = 0; j < njobs; ++j) {
        const ffp_ldlt_job& b = jobs[j];
        specs.push_back(LdltJobSpec{b.n, b.p, b.S, b.lds, b.info, (char*)w->ptr + off[j]});
    }
    return ldlt_run_multi(specs, s);
}

size_t ffp_ldlt_workspace_bytes(int64_t n, uint32_t p)
{
    if (n < 0 || p < 3 || !supported_prime(p)) return 0;
    return ldlt_workspace_bytes(n, p, n);
}

int fsyrk_modp_batched(int njobs, const ffp_job* jobs, unsigned flags, void* stream)
{
    return batched_run(njobs, jobs, flags, (hipStream_t)stream);
}

}  // extern "C"
