// fsyrk_modp_noalloc: the symmetric product with its workspace in a static
// device buffer, for callers that cannot allocate (code under stream
// capture, serving loops that forbid allocation).
//
// The buffer is a file-scope __device__ array; every device the library runs
// on holds its own copy until the process ends.  Host code never uses the
// array's name as a device address: on the first call on a device its
// address is looked up with hipGetSymbolAddress (with that device current)
// and kept per device, and that address is what the kernels receive as
// their workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ffp.h"
#include "plan.h"
#include "runtime.h"

namespace ffp {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch` (looked up once per
// device).
int scratch_address(void** out)
{
    int dev = 0;
    if (note_hip("hipGetDevice (scratch)", hipGetDevice(&dev)) != hipSuccess) return FFP_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return FFP_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (note_hip("hipGetSymbolAddress (scratch)", hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) !=
                hipSuccess ||
            p == nullptr)
            return FFP_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FFP_OK;
}

}  // namespace
}  // namespace ffp

extern "C" {

size_t ffp_noalloc_scratch_bytes(void) { return ffp::kScratchBytes; }

int fsyrk_modp_noalloc(int64_t n, int64_t k, uint32_t p, const void* A, int64_t lda, int a_dtype,
                       uint32_t alpha, uint32_t beta, uint32_t* C, int64_t ldc, unsigned flags,
                       void* stream)
{
    using namespace ffp;
    PlanRequest rq;
    int st = make_syrk_request(n, k, p, A, lda, a_dtype, alpha, beta, C, ldc, flags, &rq);
    if (st != FFP_OK) return st;
    if (n == 0) return FFP_OK;
    Plan pl;
    st = build_syrk_plan(rq, &pl);
    if (st != FFP_OK) return st;
    if ((size_t)pl.ws_bytes > kScratchBytes) {
        note_hip("fsyrk_modp_noalloc: workspace of this shape exceeds the 64 MiB static scratch",
                 hipErrorOutOfMemory);
        return FFP_ENOMEM;
    }
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != FFP_OK) return st;
    // the schedule never relies on the workspace's previous contents: every
    // block it reads there is written earlier in the same call
    return execute_plan(pl, A, C, ws, (hipStream_t)stream, /*no_alloc=*/true);
}

}  // extern "C"
