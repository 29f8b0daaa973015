// Autotuner of fsyrk_modp.
//
// For a shape class the tuner times whole fsyrk_modp executions on
// synthetic operands for every candidate recursion depth (Algorithm 2
// applied d times; each level trades one product in six for block
// additions, Table 1), product tile edge and placement variant, and keeps
// the fastest.  Depths are tried upwards per tile and the search stops
// once a depth is clearly slower than the best one seen, since deeper
// recursion only adds HBM-bound additions and smaller leaves after that.
// The table is process-wide and can be saved to and loaded from a text
// file.  Calls that do not force a depth (FFP_DEPTH) consult it; the
// LDL^T driver's Schur updates keep the built-in rule so that its
// workspace figure does not depend on the table.
#include "tune.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "runtime.h"

namespace ffp {

namespace {

using Key = std::tuple<int, int, int, int, int>;

std::mutex g_tune_mutex;
std::map<Key, TuneChoice> g_table;

int ceil_log2(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

Key key_of(int cls, int64_t n, int64_t k, bool accumulate, bool lowmem)
{
    return Key{cls, ceil_log2(n < 1 ? 1 : n), ceil_log2(k < 1 ? 1 : k), accumulate ? 1 : 0, lowmem ? 1 : 0};
}

bool valid_choice(int cls, const TuneChoice& c)
{
    if (c.depth < 0 || c.depth > 7 || (c.wide != 0 && c.wide != 1)) return false;
    if (c.base != 0 && !(c.base == CLS_LIMB3 && cls == CLS_F64 && c.depth == 0 && c.tile == 0)) return false;
    if (c.tile == 0) return true;
    if (cls == CLS_F64) return c.tile == 64 || c.tile == 128;
    if (cls == CLS_I8) return c.tile == 128 || c.tile == 256;
    return false;
}

int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

}  // namespace

bool tune_lookup(int cls, int64_t n, int64_t k, bool accumulate, bool lowmem, TuneChoice* out)
{
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    auto it = g_table.find(key_of(cls, n, k, accumulate, lowmem));
    if (it == g_table.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(int cls, int64_t n, int64_t k, bool accumulate, bool lowmem, const TuneChoice& c)
{
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_table[key_of(cls, n, k, accumulate, lowmem)] = c;
}

unsigned pin_flags(const ffp_job& j, unsigned flags)
{
    if ((flags >> 4) & 0xFu) return flags;
    PlanRequest rq;
    if (make_syrk_request(j.n, j.k, j.p, j.A, j.lda, j.a_dtype, j.alpha, j.beta, j.C, j.ldc, flags, &rq) !=
        FFP_OK)
        return flags;
    Plan pl;
    if (build_syrk_plan(rq, &pl) != FFP_OK) return flags;
    unsigned f = flags | FFP_DEPTH(pl.depth);
    if (!pl.wide) f |= FFP_LOW_MEMORY;
    if (pl.cls == CLS_LIMB3) f |= FFP_BASE_LIMB3;
    return f;
}

namespace {

// Average time of one execution of the request (after one untimed run).
int time_request(const PlanRequest& rq, const void* A, uint32_t* C, hipStream_t s, hipEvent_t e0,
                 hipEvent_t e1, double* ms)
{
    Plan pl;
    int st = build_syrk_plan(rq, &pl);
    if (st != FFP_OK) return st;
    Workspace* w = nullptr;
    st = acquire_workspace(s, (size_t)pl.ws_bytes, 0, &w);
    if (st != FFP_OK) return st;
    st = execute_plan(pl, A, C, w->ptr, s);
    if (st != FFP_OK) return st;
    float t = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) return FFP_EDEVICE;
    st = execute_plan(pl, A, C, w->ptr, s);
    if (st != FFP_OK) return st;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        return FFP_EDEVICE;
    // repeat short runs so that the figure covers about 20 ms
    const int reps = t <= 0.f ? 1 : (int)std::fmin(8.0, std::ceil(20.0 / t));
    if (reps > 1) {
        if (hipEventRecord(e0, s) != hipSuccess) return FFP_EDEVICE;
        for (int r = 0; r < reps && st == FFP_OK; ++r) st = execute_plan(pl, A, C, w->ptr, s);
        if (st != FFP_OK) return st;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return FFP_EDEVICE;
        t /= (float)reps;
    }
    *ms = t;
    return FFP_OK;
}

}  // namespace

}  // namespace ffp

using namespace ffp;

extern "C" {

int ffp_autotune(int64_t n, int64_t k, uint32_t p, int a_dtype, uint32_t alpha, uint32_t beta, unsigned flags,
                 void* stream, ffp_tune_result* out)
{
    if (!out) return FFP_EINVAL;
    memset(out, 0, sizeof *out);
    if (n <= 0 || k <= 0) return FFP_EINVAL;
    if ((flags >> 4) & 0xFu) return FFP_EINVAL;   // the depth is what is tuned
    const int64_t lda = a_dtype == FFP_U32 ? rup(k, 4) : rup(k, 16);
    const int64_t ldc = rup(n, 4);
    PlanRequest base;
    int st = make_syrk_request(n, k, p, (const void*)256, lda, a_dtype, alpha, beta, (const uint32_t*)256, ldc,
                               flags, &base);
    if (st != FFP_OK) return st;
    const int cls = choose_class(p, base.a_cls, base.force_f64, base.force_limb3);
    const bool accumulate = alpha != 1u || beta != 0u;
    const bool lowmem = !base.wide;

    hipStream_t s = (hipStream_t)stream;
    const int64_t planes = a_dtype == FFP_I8_LIMB2 ? 2 : 1;
    const int64_t abytes = (a_dtype == FFP_U32 ? 4 : 1) * n * lda * planes;
    void* A = nullptr;
    uint32_t* C = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (note_hip("hipMalloc (tuning operand)", hipMalloc(&A, (size_t)abytes)) != hipSuccess ||
        note_hip("hipMalloc (tuning result)", hipMalloc((void**)&C, (size_t)(n * ldc * 4))) != hipSuccess) {
        if (A) (void)hipFree(A);
        return FFP_ENOMEM;
    }
    if (note_hip("hipEventCreate", hipEventCreate(&e0)) != hipSuccess ||
        note_hip("hipEventCreate", hipEventCreate(&e1)) != hipSuccess) {
        (void)hipFree(A);
        (void)hipFree(C);
        if (e0) (void)hipEventDestroy(e0);
        return FFP_EDEVICE;
    }
    if (launch_fill_residues(n, k, A, lda, n * lda, a_dtype, p, 0x5eedull, s) != hipSuccess ||
        launch_fill_residues(n, n, C, ldc, 0, FFP_U32, p, 0xc0ffeeull, s) != hipSuccess)
        st = FFP_EDEVICE;

    std::vector<int> tiles;
    if (cls == CLS_F64) tiles = {64, 128};
    else if (cls == CLS_I8) tiles = {128, 256};
    else tiles = {0};
    int dmax = 0;
    while (dmax < 4 && (n >> (dmax + 1)) >= 64) ++dmax;
    if (cls != CLS_F64 && dmax > 2) dmax = 2;

    TuneChoice best;
    double best_ms = INFINITY;
    int tried = 0;
    // the three-limb int8 path (depth 0) as an alternative base for FP64
    // shapes with uint32 operands and p < 2^23
    if (cls == CLS_F64 && a_dtype == FFP_U32 && !base.force_f64 && p < (1u << 23)) {
        PlanRequest rq = base;
        rq.depth = 0;
        rq.force_limb3 = true;
        rq.no_tune = true;
        double ms = 0.0;
        if (st == FFP_OK) st = time_request(rq, A, C, s, e0, e1, &ms);
        if (st == FFP_OK) {
            ++tried;
            best_ms = ms;
            best.depth = 0;
            best.tile = 0;
            best.wide = lowmem ? 0 : 1;
            best.base = CLS_LIMB3;
            best.ms = ms;
        }
    }
    for (int tile : tiles) {
        if (st != FFP_OK) break;
        double tile_best = INFINITY;
        for (int d = 0; d <= dmax && st == FFP_OK; ++d) {
            double depth_best = INFINITY;
            for (int wide = lowmem ? 0 : 1; wide >= 0; --wide) {
                if (d == 0 && wide != (lowmem ? 0 : 1)) break;   // no placements without recursion
                PlanRequest rq = base;
                rq.depth = d;
                rq.wide = wide != 0;
                rq.tile = tile;
                rq.no_tune = true;
                double ms = 0.0;
                st = time_request(rq, A, C, s, e0, e1, &ms);
                if (st != FFP_OK) break;
                ++tried;
                if (ms < depth_best) depth_best = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best.depth = d;
                    best.tile = tile;
                    best.wide = wide;
                    best.base = 0;
                    best.ms = ms;
                }
            }
            if (depth_best < tile_best) tile_best = depth_best;
            else if (depth_best > 1.15 * tile_best) break;
        }
    }
    // the built-in rule, for comparison
    double rule_ms = 0.0;
    if (st == FFP_OK) {
        PlanRequest rq = base;
        rq.no_tune = true;
        st = time_request(rq, A, C, s, e0, e1, &rule_ms);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(A);
    (void)hipFree(C);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FFP_OK) return st;
    tune_store(cls, n, k, accumulate, lowmem, best);
    out->depth = best.depth;
    out->tile = best.tile;
    out->wide = best.wide;
    out->base = best.base;
    out->candidates = tried;
    out->ms = best.ms;
    out->rule_ms = rule_ms;
    return FFP_OK;
}

int ffp_tune_lookup(int64_t n, int64_t k, uint32_t p, int a_dtype, uint32_t alpha, uint32_t beta, unsigned flags,
                    ffp_tune_result* out)
{
    if (!out) return FFP_EINVAL;
    memset(out, 0, sizeof *out);
    const int64_t lda = a_dtype == FFP_U32 ? rup(k, 4) : rup(k, 16);
    PlanRequest rq;
    int st = make_syrk_request(n, k, p, (const void*)256, lda > 0 ? lda : 16, a_dtype, alpha, beta,
                               (const uint32_t*)256, rup(n > 0 ? n : 1, 4), flags, &rq);
    if (st != FFP_OK) return st;
    Plan pl;
    st = build_syrk_plan(rq, &pl);
    if (st != FFP_OK) return st;
    out->depth = pl.depth;
    out->tile = pl.tile;
    out->wide = pl.wide ? 1 : 0;
    out->base = pl.cls == CLS_LIMB3 ? CLS_LIMB3 : 0;
    TuneChoice tc;
    if (pl.tuned && tune_lookup(pl.cls, n, k, alpha != 1u || beta != 0u, !rq.wide, &tc)) out->ms = tc.ms;
    return pl.tuned ? 1 : 0;
}

int ffp_tune_save(const char* path)
{
    if (!path) return FFP_EINVAL;
    FILE* f = fopen(path, "w");
    if (!f) return FFP_EINVAL;
    fprintf(f, "# ffp tuning table 2: cls log2n log2k accumulate lowmem depth tile wide base ms\n");
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        for (const auto& [key, c] : g_table)
            fprintf(f, "%d %d %d %d %d %d %d %d %d %.6g\n", std::get<0>(key), std::get<1>(key), std::get<2>(key),
                    std::get<3>(key), std::get<4>(key), c.depth, c.tile, c.wide, c.base, c.ms);
    }
    return fclose(f) == 0 ? FFP_OK : FFP_EINVAL;
}

int ffp_tune_load(const char* path)
{
    if (!path) return FFP_EINVAL;
    FILE* f = fopen(path, "r");
    if (!f) return FFP_EINVAL;
    std::vector<std::pair<Key, TuneChoice>> rows;
    char line[512];
    int status = FFP_OK;
    while (fgets(line, sizeof line, f)) {
        const char* q = line;
        while (*q == ' ' || *q == '\t') ++q;
        if (*q == '#' || *q == '\n' || *q == '\0') continue;
        int cls, ln, lk, acc, lm;
        TuneChoice c;
        double ms = 0.0;
        if (sscanf(q, "%d %d %d %d %d %d %d %d %d %lf", &cls, &ln, &lk, &acc, &lm, &c.depth, &c.tile, &c.wide, &c.base,
                   &ms) != 10 ||
            cls < 0 || cls >= kNumCls || ln < 0 || ln > 31 || lk < 0 || lk > 31 || (acc != 0 && acc != 1) ||
            (lm != 0 && lm != 1) || !valid_choice(cls, c)) {
            status = FFP_EINVAL;
            break;
        }
        c.ms = ms;
        rows.push_back({Key{cls, ln, lk, acc, lm}, c});
    }
    fclose(f);
    if (status != FFP_OK) return status;   // nothing is applied from a malformed file
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    for (const auto& r : rows) g_table[r.first] = r.second;
    return (int)rows.size();
}

void ffp_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_table.clear();
}

int ffp_tune_entries(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    return (int)g_table.size();
}

}  // extern "C"
