// Autotuner of fsyrk_modp: the recursion depth (cut-off of Algorithm 2),
// the placements (Table 3/4 or the wide variant) and the product tile,
// measured on the device per shape class and kept in a process-wide table.
#pragma once
#include <cstdint>

#include "ffp.h"

namespace ffp {

struct TuneChoice {
    int32_t depth = -1;
    int32_t tile = 0;      // product tile edge (0: launch rule)
    int32_t wide = 1;      // wide placements (1) or those of Tables 3 and 4 (0)
    int32_t base = 0;      // 0: the base path of p; CLS_LIMB3: three int8 limbs
    double ms = 0.0;       // measured time of the choice at tuning
};

// Shape classes: base path class, ceil(log2 n), ceil(log2 k), accumulate
// form ((alpha, beta) != (1, 0)), low-memory placements requested.
bool tune_lookup(int cls, int64_t n, int64_t k, bool accumulate, bool lowmem, TuneChoice* out);
void tune_store(int cls, int64_t n, int64_t k, bool accumulate, bool lowmem, const TuneChoice& c);

// The job's flags with its depth, placements and base path made explicit
// (FFP_DEPTH, FFP_LOW_MEMORY, FFP_BASE_LIMB3) as the tuning table or the
// built-in rule chooses them now, so that its workspace figure stays valid
// whatever the table holds later.
unsigned pin_flags(const ffp_job& j, unsigned flags);

}  // namespace ffp
