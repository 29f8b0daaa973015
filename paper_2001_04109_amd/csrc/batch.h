// Batched fsyrk_modp (grouped launches over many independent jobs).
#pragma once
#include <hip/hip_runtime.h>

#include "ffp.h"

namespace ffp {

// Workspace bytes that job j needs on its own inside batched_run.
int64_t job_workspace_bytes(const ffp_job& j, unsigned flags);

// job_ws: optional per-job device workspaces (job j gets job_ws[j], at least
// job_workspace_bytes(jobs[j]) bytes, 256-byte aligned); when null the
// library's per-stream workspace holds all jobs' slices.
// job_flags: optional per-job flags in place of `flags`.
int batched_run(int njobs, const ffp_job* jobs, unsigned flags, hipStream_t s,
                char* const* job_ws = nullptr, const unsigned* job_flags = nullptr);

}  // namespace ffp
