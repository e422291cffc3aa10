// Densification, pruning and opacity reset of the first training phase: 3DGS's density
// control, which the paper keeps (with a random keep probability that caps the splat
// count) for the iterations before the active-set phase (Sec. 5.1 "Implementation
// Details"; Fig. "overview").  The rules are stated with the entry points in oit.h.
#include "oit_density.h"

namespace oit {

constexpr unsigned kDensityBlocks = 1024;

// ---------------------------------------------------------------------------------
// statistic: one thread per active row, its views in order (no atomics, the sums
// are reproducible).  A view counts when the record's alpha >= 1/255 box reaches a
// pixel centre; its dL/d(projected mean) is the sum of the pair's entry partials.
// ---------------------------------------------------------------------------------
struct DStatArgs {
    Buffers b;
    RowList rl;
    float *accum, *denom, *maxr;
};

__global__ __launch_bounds__(256) void k_densify_stats(DStatArgs a)
{
    int64_t na = a.rl.n_active ? (int64_t)*a.rl.n_active : a.rl.n_active_host;
    na = na < 0 ? 0 : (na > a.rl.Acap ? a.rl.Acap : na);
    int64_t nd = a.rl.n_delta ? (int64_t)*a.rl.n_delta : 0;
    nd = nd < 0 ? 0 : (nd > a.rl.Rcap - a.rl.Acap ? a.rl.Rcap - a.rl.Acap : nd);
    const int64_t nrec = na + nd;
    const int V = a.b.n_views;
    const uint64_t cap = (uint64_t)a.b.pair_cap;
    const float k = 0.5f * kLog2e;   // conic = record's scaled conic / (-k): cov = k adj / det
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < na;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = a.rl.active_idx ? (int64_t)a.rl.active_idx[t] : t;
        float acc = 0.f, den = 0.f, rmax = 0.f;
        for (int v = 0; v < V; ++v) {
            const CamDev &cam = a.b.cams[v];
            const Rec r = a.b.rec[(size_t)v * a.rl.Rcap + t];
            const float tl = r.b.y - kLog2AlphaMin;   // alpha >= 1/255 <=> scaled form <= tl
            if (!(tl >= 0.f)) continue;
            const float A = -r.a.z, B = -0.5f * r.a.w, C = -r.b.x;
            const float det = A * C - B * B;
            if (!(det > 0.f)) continue;
            const float hx = sqrtf(tl * C / det), hy = sqrtf(tl * A / det);
            const float mx = r.a.x, my = r.a.y;
            const float xl = fmaxf(ceilf(mx - hx - 0.5f), 0.f), xh = fminf(floorf(mx + hx - 0.5f), (float)(cam.W - 1));
            const float yl = fmaxf(ceilf(my - hy - 0.5f), 0.f), yh = fminf(floorf(my + hy - 0.5f), (float)(cam.H - 1));
            if (!(xl <= xh && yl <= yh)) continue;
            float gx = 0.f, gy = 0.f;
            const size_t pv = (size_t)v * nrec + t;
            const uint64_t g0 = a.b.hoff[pv], nh = a.b.nhits[pv];
            for (uint64_t e = 0; e < nh && g0 + e < cap; ++e) {
                const float2 p = *(const float2 *)(a.b.ep + (g0 + e) * kEpStride);
                gx += p.x;
                gy += p.y;
            }
            const float ux = gx * 0.5f * (float)cam.W, uy = gy * 0.5f * (float)cam.H;
            acc += sqrtf(ux * ux + uy * uy);
            den += 1.f;
            const float cxx = k * C / det, cyy = k * A / det, cxy = -k * B / det;
            const float hd = 0.5f * (cxx - cyy);
            const float lam = 0.5f * (cxx + cyy) + sqrtf(hd * hd + cxy * cxy);
            rmax = fmaxf(rmax, 3.f * sqrtf(lam));
        }
        if (den > 0.f) {
            a.accum[id] += acc;
            a.denom[id] += den;
            a.maxr[id] = fmaxf(a.maxr[id], rmax);
        }
    }
}

void launch_densify_stats(const Buffers &b, const RowList &rl, float *accum, float *denom, float *max_radius,
                          hipStream_t s)
{
    DStatArgs a{b, rl, accum, denom, max_radius};
    hipLaunchKernelGGL(k_densify_stats, dim3(kDensityBlocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------------
// plan: keep flags of every splat's possible outputs, their scans, the new size
// ---------------------------------------------------------------------------------
size_t density_workspace_bytes(int64_t n)
{
    const size_t nb = (size_t)((n + kScanBlockItems - 1) / kScanBlockItems);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return 6 * al(4 * (size_t)n) + al(4 * (nb + 1)) + al(16);
}

DensityBuffers density_buffers(void *ws, int64_t n)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *w = (char *)ws;
    size_t o = 0;
    DensityBuffers d;
    for (int k = 0; k < 3; ++k) {
        d.flag[k] = (uint32_t *)(w + o);
        o += al(4 * (size_t)n);
    }
    for (int k = 0; k < 3; ++k) {
        d.off[k] = (uint32_t *)(w + o);
        o += al(4 * (size_t)n);
    }
    d.tmp = (uint32_t *)(w + o);
    o += al(4 * ((size_t)((n + kScanBlockItems - 1) / kScanBlockItems) + 1));
    d.totals = (uint32_t *)(w + o);
    return d;
}

struct DPlanArgs {
    SplatPtrs sp;
    const float *accum, *denom, *maxr, *uniform;
    oit_density_rules r;
    DensityBuffers db;
};

__global__ __launch_bounds__(256) void k_densify_flags(DPlanArgs a)
{
    const oit_density_rules &r = a.r;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.sp.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float d = a.denom[i];
        const float avg = d > 0.f ? a.accum[i] / d : 0.f;
        const bool cand = avg >= r.grad_threshold && a.uniform[i] < r.keep_probability;
        const float smax = fmaxf(fmaxf(expf(a.sp.log_scale[3 * i]), expf(a.sp.log_scale[3 * i + 1])),
                                 expf(a.sp.log_scale[3 * i + 2]));
        const bool small = smax <= r.percent_dense * r.scene_extent;
        const bool low = 1.f / (1.f + expf(-a.sp.logit[i])) < r.min_opacity;
        const float wlim = r.max_world_frac * r.scene_extent;
        const bool world = r.max_world_frac > 0.f;
        const bool screen_big = r.max_screen_size > 0.f && a.maxr[i] > r.max_screen_size;
        const bool clone = cand && small, split = cand && !small;
        a.db.flag[0][i] = !split && !low && !screen_big && !(world && smax > wlim);
        a.db.flag[1][i] = clone && !low && !(world && smax > wlim);
        a.db.flag[2][i] = split && !low && !(world && smax / 1.6f > wlim);
    }
}

__global__ void k_densify_totals(DensityBuffers db, int64_t n, int64_t *n_new)
{
    uint32_t t[3];
    for (int k = 0; k < 3; ++k) {
        t[k] = n > 0 ? db.off[k][n - 1] + db.flag[k][n - 1] : 0u;
        db.totals[k] = t[k];
    }
    *n_new = (int64_t)t[0] + (int64_t)t[1] + 2 * (int64_t)t[2];
}

void launch_densify_plan(const SplatPtrs &sp, const float *accum, const float *denom, const float *max_radius,
                         const float *uniform, const oit_density_rules &rules, int64_t *n_new,
                         const DensityBuffers &db, hipStream_t s)
{
    DPlanArgs a{sp, accum, denom, max_radius, uniform, rules, db};
    hipLaunchKernelGGL(k_densify_flags, dim3(kDensityBlocks), dim3(256), 0, s, a);
    for (int k = 0; k < 3; ++k) launch_scan_u32(db.flag[k], db.off[k], sp.n, db.tmp, s);
    hipLaunchKernelGGL(k_densify_totals, dim3(1), dim3(1), 0, s, db, sp.n, n_new);
}

// ---------------------------------------------------------------------------------
// apply: one thread per source splat writes its surviving outputs
// ---------------------------------------------------------------------------------
struct DApplyArgs {
    SplatPtrs sp;
    const float *m[6], *v[6];
    const float *normals;
    float *p_new[6], *m_new[6], *v_new[6];
    int64_t cap_new;
    DensityBuffers db;
};

__device__ __constant__ const int kGroupWidth[6] = {3, 3, 4, 1, 48, 16};

// copies splat i's parameters to row j of the new set; moments carried or zero
__device__ void copy_row(const DApplyArgs &a, int64_t i, int64_t j, bool carry)
{
    const float *src[6] = {a.sp.mean, a.sp.log_scale, a.sp.quat, a.sp.logit, a.sp.sh, a.sp.vsh};
    for (int g = 0; g < 6; ++g) {
        const int C = kGroupWidth[g];
        for (int c = 0; c < C; ++c) {
            const size_t si = (size_t)i * C + c, dj = (size_t)j * C + c;
            a.p_new[g][dj] = src[g][si];
            a.m_new[g][dj] = carry ? a.m[g][si] : 0.f;
            a.v_new[g][dj] = carry ? a.v[g][si] : 0.f;
        }
    }
}

__global__ __launch_bounds__(256) void k_densify_apply(DApplyArgs a)
{
    const uint32_t T0 = a.db.totals[0], T1 = a.db.totals[1], T2 = a.db.totals[2];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.sp.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (a.db.flag[0][i]) {
            const int64_t j = a.db.off[0][i];
            if (j < a.cap_new) copy_row(a, i, j, true);
        }
        if (a.db.flag[1][i]) {
            const int64_t j = (int64_t)T0 + a.db.off[1][i];
            if (j < a.cap_new) copy_row(a, i, j, false);
        }
        if (a.db.flag[2][i]) {
            float q[4], Rq[9], s[3], mu[3];
            for (int c = 0; c < 4; ++c) q[c] = a.sp.quat[4 * i + c];
            const float qi = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
            quat_rot(q[0] * qi, q[1] * qi, q[2] * qi, q[3] * qi, Rq);
            for (int c = 0; c < 3; ++c) {
                s[c] = expf(a.sp.log_scale[3 * i + c]);
                mu[c] = a.sp.mean[3 * i + c];
            }
            const float ln_div = 0.47000362924573558f;   // ln 1.6
            for (int child = 0; child < 2; ++child) {
                const int64_t j = (int64_t)T0 + T1 + (int64_t)child * T2 + a.db.off[2][i];
                if (j >= a.cap_new) continue;
                copy_row(a, i, j, false);
                const float *z = a.normals + (size_t)i * 6 + 3 * child;
                const float sz[3] = {s[0] * z[0], s[1] * z[1], s[2] * z[2]};
                for (int r = 0; r < 3; ++r) {
                    a.p_new[0][3 * j + r] = mu[r] + Rq[3 * r] * sz[0] + Rq[3 * r + 1] * sz[1] + Rq[3 * r + 2] * sz[2];
                    a.p_new[1][3 * j + r] = a.sp.log_scale[3 * i + r] - ln_div;
                }
            }
        }
    }
}

void launch_densify_apply(const SplatPtrs &sp, const float *const *m, const float *const *v, const float *normals,
                          float *const *params_new, float *const *m_new, float *const *v_new, int64_t cap_new,
                          const DensityBuffers &db, hipStream_t s)
{
    DApplyArgs a;
    a.sp = sp;
    for (int g = 0; g < 6; ++g) {
        a.m[g] = m[g];
        a.v[g] = v[g];
        a.p_new[g] = params_new[g];
        a.m_new[g] = m_new[g];
        a.v_new[g] = v_new[g];
    }
    a.normals = normals;
    a.cap_new = cap_new;
    a.db = db;
    hipLaunchKernelGGL(k_densify_apply, dim3(kDensityBlocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------------
// opacity reset
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reset_opacity(float *logit, float *m, float *v, int64_t n, float max_logit)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        logit[i] = fminf(logit[i], max_logit);
        m[i] = 0.f;
        v[i] = 0.f;
    }
}

void launch_reset_opacity(float *logit, float *m, float *v, int64_t n, float max_logit, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_opacity, dim3(kDensityBlocks), dim3(256), 0, s, logit, m, v, n, max_logit);
}

}  // namespace oit
