// Host-side schedules of the symmetric products over F_p[i] (fzsyrk_modp:
// A A^T; fherk_modp: A A^H), written as block operations on the two uint32
// planes of each complex matrix (see cplan.cpp).
#pragma once
#include <cstdint>

#include "plan.h"

namespace ffp {

struct ComplexRequest {
    int64_t n = 0, k = 0;
    uint32_t p = 0;
    bool herk = false;           // A A^H (conjugate transpose) instead of A A^T
    int64_t lda = 0, a_plane = 0;   // elements; imaginary plane at A + a_plane
    int64_t ldc = 0, c_plane = 0;
    int32_t depth = -1;          // -1: default
    bool fill_upper = false;
};

int build_complex_plan(const ComplexRequest& rq, Plan* out);
int default_complex_depth(int64_t n, int64_t k);

}  // namespace ffp
