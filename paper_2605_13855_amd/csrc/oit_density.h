// Internal interface of the densification kernels (k_density.hip) for the C ABI.
#pragma once

#include "oit_internal.h"

namespace oit {

// Workspace of oit_densify_plan / oit_densify_apply for n splats: three keep flags per
// splat (original, clone copy, children), their exclusive scans, the scan's block sums
// and the three segment totals.
struct DensityBuffers {
    uint32_t *flag[3];
    uint32_t *off[3];
    uint32_t *tmp;
    uint32_t *totals;
};

size_t density_workspace_bytes(int64_t n);
DensityBuffers density_buffers(void *ws, int64_t n);

void launch_densify_stats(const Buffers &b, const RowList &rl, float *accum, float *denom, float *max_radius,
                          hipStream_t s);
void launch_densify_plan(const SplatPtrs &sp, const float *accum, const float *denom, const float *max_radius,
                         const float *uniform, const oit_density_rules &rules, int64_t *n_new,
                         const DensityBuffers &db, hipStream_t s);
void launch_densify_apply(const SplatPtrs &sp, const float *const *m, const float *const *v, const float *normals,
                          float *const *params_new, float *const *m_new, float *const *v_new, int64_t cap_new,
                          const DensityBuffers &db, hipStream_t s);
void launch_reset_opacity(float *logit, float *m, float *v, int64_t n, float max_logit, hipStream_t s);

}  // namespace oit
