// Device helpers shared by the product kernels: task lookup, triangular tile
// enumeration and the XCD-aware block order.
#pragma once
#include "kernels.h"

namespace ffp {

// Copy the task that owns global tile g into registers.  Tasks are sorted by
// tile0; the search is uniform across the workgroup.
__device__ inline void select_task(const ProdArgs& a, int g, ProdTask* out)
{
    if (a.ntasks <= kInlineTasks) {
        int idx = 0;
#pragma unroll
        for (int i = 1; i < kInlineTasks; ++i)
            if (i < a.ntasks && g >= a.inl[i].tile0) idx = i;
#pragma unroll
        for (int i = 0; i < kInlineTasks; ++i)
            if (i == idx) *out = a.inl[i];
        return;
    }
    int lo = 0, hi = a.ntasks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.dev_tasks[mid].tile0 <= g) lo = mid; else hi = mid - 1;
    }
    *out = a.dev_tasks[lo];
}

// r-th tile (row-major over the lower triangle) -> (ti, tj), tj <= ti.
__device__ inline void tri_index(int r, int* ti, int* tj)
{
    int i = (int)((sqrtf(8.0f * (float)r + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= r) ++i;
    while (i * (i + 1) / 2 > r) --i;
    *ti = i;
    *tj = r - i * (i + 1) / 2;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8).
// For a launch of one uniform task, give each XCD a contiguous range of
// tiles so that neighbouring tiles, which share operand panels, meet in the
// same L2.  `nblocks` is a multiple of 8.
// Tile visited i-th by workgroup w of a persistent launch of G workgroups:
// tiles are dealt to the 8 XCDs in chunks of 8 consecutive ones (round
// robin), so that neighbouring tiles, which share operand panels, meet in
// one XCD's L2, and every XCD gets a share of the long tasks at the front
// of the list; an XCD's workgroups stride over its chunks.  A tile index at
// or past the launch's tile count ends the workgroup's sequence (it grows
// with i).  For G not a multiple of 8: plain striding.
__device__ inline int persistent_tile(int w, int G, int i)
{
    if (G & 7) return w + i * G;
    const int x = w & 7, j = (w >> 3) + i * (G >> 3);
    return (((j >> 3) << 3) + x) * 8 + (j & 7);
}

__device__ inline int xcd_remap(int b, int nblocks)
{
    const int per = nblocks >> 3;
    return (b & 7) * per + (b >> 3);
}

// Three-limb storage of a centred residue x (|x| < 2^22): x = l + 256 m +
// 65536 h with l, m in [-128, 127] (and then |h| <= 65).
__device__ inline void limb3_split(int x, int8_t* l, int8_t* m, int8_t* h)
{
    const int lo = ((x + 128) & 255) - 128;
    const int y = (x - lo) >> 8;
    const int mid = ((y + 128) & 255) - 128;
    *l = (int8_t)lo;
    *m = (int8_t)mid;
    *h = (int8_t)((y - mid) >> 8);
}

__device__ inline double mod_f64(double x, double p, double pinv)
{
    // x is an integer with |x| < 2^53; the quotient estimate is off by at most one
    double q = floor(x * pinv);
    double r = fma(-q, p, x);
    if (r < 0.0) r += p;
    if (r >= p) r -= p;
    return r;
}

}  // namespace ffp
