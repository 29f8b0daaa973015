// Batched fsyrk_modp (grouped launches over many independent jobs).
#pragma once
#include <hip/hip_runtime.h>

#include "ffp.h"

namespace ffp {

int batched_run(int njobs, const ffp_job* jobs, unsigned flags, hipStream_t s);

}  // namespace ffp
