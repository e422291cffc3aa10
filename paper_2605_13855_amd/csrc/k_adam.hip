// Adam restricted to the active rows (Sec. 4.1, Alg. "Active Set Method": only the
// active splats are updated; the optimiser is Adam, Sec. 5.1).  Rows outside the
// active set keep their values and moments.
#include "oit_internal.h"

namespace oit {

__global__ void k_step_inc(int32_t *step) { *step += 1; }

struct AdamArgs {
    AdamPtrs p;
    int64_t gstride;
    const int32_t *idx;
    const int32_t *n_active;
    int64_t n;
    int64_t rows_cap;   // compact gradient rows available (the device count is clamped to it)
    float b1, b2, eps;
    const int32_t *step;
};

// One block per tile of kRows active rows of one attribute group (grid.y = group),
// grid-stride over the tiles with a fixed grid (the row count is read on the device).
// The tile's gradients arrive component-major ([C][stride], one coalesced run per
// component) and are transposed through LDS, so that the parameters and both moments
// ([n][C]) are read and written in whole per-splat segments.
constexpr int kAdamThreads = 256;
constexpr int kRows = 64;
constexpr unsigned kAdamTiles = 1024;
constexpr int kUnroll = 4;

template <int C>
__device__ void adam_group(const AdamArgs &a, int grp, int64_t na, float bc1, float bc2, float *s_g,
                           int64_t *s_id)
{
    float *p = a.p.p[grp], *m = a.p.m[grp], *v = a.p.v[grp];
    const float *g = a.p.g[grp];
    const float lr = a.p.lr[grp];
    const int64_t ntiles = (na + kRows - 1) / kRows;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * kRows;
        const int rows = (int)min((int64_t)kRows, na - r0);
        // the element loops take kUnroll elements per thread per pass, their loads issued
        // before any is used, so that a pass waits on memory once
#pragma unroll
        for (int e0 = 0; e0 < C * kRows; e0 += kUnroll * kAdamThreads) {
            float gv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int e = e0 + u * kAdamThreads + threadIdx.x, c = e / kRows, j = e % kRows;
                gv[u] = e < C * kRows && j < rows ? g[(size_t)c * a.gstride + r0 + j] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int e = e0 + u * kAdamThreads + threadIdx.x, c = e / kRows, j = e % kRows;
                if (e < C * kRows && j < rows) s_g[c * (kRows + 1) + j] = gv[u];
            }
        }
        if (threadIdx.x < rows) s_id[threadIdx.x] = a.idx ? (int64_t)a.idx[r0 + threadIdx.x] : r0 + threadIdx.x;
        __syncthreads();
        for (int e0 = 0; e0 < rows * C; e0 += kUnroll * kAdamThreads) {
            size_t pi[kUnroll];
            float gg[kUnroll], m0[kUnroll], v0[kUnroll], p0[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int e = e0 + u * kAdamThreads + threadIdx.x;
                const bool ok = e < rows * C;
                const int j = ok ? e / C : 0, c = ok ? e % C : 0;
                pi[u] = (size_t)s_id[j] * C + c;
                gg[u] = s_g[c * (kRows + 1) + j];
                m0[u] = ok ? m[pi[u]] : 0.f;
                v0[u] = ok ? v[pi[u]] : 0.f;
                p0[u] = ok ? p[pi[u]] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (e0 + u * kAdamThreads + (int)threadIdx.x >= rows * C) continue;
                const float mm = a.b1 * m0[u] + (1.f - a.b1) * gg[u];
                const float vv = a.b2 * v0[u] + (1.f - a.b2) * gg[u] * gg[u];
                m[pi[u]] = mm;
                v[pi[u]] = vv;
                p[pi[u]] = p0[u] - lr * (mm / bc1) / (sqrtf(vv / bc2) + a.eps);
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kAdamThreads) void k_sparse_adam(AdamArgs a)
{
    __shared__ float s_g[48 * (kRows + 1)];   // the largest group (colour SH), padded rows
    __shared__ int64_t s_id[kRows];
    __shared__ float s_bc[2];                 // bias corrections of this step
    if (threadIdx.x == 0) {
        const float t = (float)*a.step;
        s_bc[0] = 1.f - powf(a.b1, t);
        s_bc[1] = 1.f - powf(a.b2, t);
    }
    __syncthreads();
    const int64_t na = a.n_active ? min((int64_t)*a.n_active, a.rows_cap) : a.n;
    const float bc1 = s_bc[0], bc2 = s_bc[1];
    switch (blockIdx.y) {
    case 0: adam_group<3>(a, 0, na, bc1, bc2, s_g, s_id); break;
    case 1: adam_group<3>(a, 1, na, bc1, bc2, s_g, s_id); break;
    case 2: adam_group<4>(a, 2, na, bc1, bc2, s_g, s_id); break;
    case 3: adam_group<1>(a, 3, na, bc1, bc2, s_g, s_id); break;
    case 4: adam_group<48>(a, 4, na, bc1, bc2, s_g, s_id); break;
    default: adam_group<16>(a, 5, na, bc1, bc2, s_g, s_id); break;
    }
}

void launch_sparse_adam(const AdamPtrs &p, int64_t gstride, const int32_t *active_idx, const int32_t *n_active,
                        int64_t n, int64_t rows_cap, float b1, float b2, float eps, int32_t *step,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, s, step);
    AdamArgs a{p, gstride, active_idx, n_active, n, rows_cap, b1, b2, eps, step};
    const int64_t tiles = (rows_cap + kRows - 1) / kRows;
    const unsigned bx = (unsigned)min((int64_t)kAdamTiles, tiles);
    if (bx) hipLaunchKernelGGL(k_sparse_adam, dim3(bx, 6), dim3(kAdamThreads), 0, s, a);
}

__global__ void k_sigma_adam(float *sigma, const double *g, float *m, float *v, float lr, float b1, float b2,
                             float eps, int32_t *step)
{
    const int32_t st = *step + 1;
    *step = st;
    const float gg = (float)*g;
    const float t = (float)st;
    const float mm = b1 * *m + (1.f - b1) * gg;
    const float vv = b2 * *v + (1.f - b2) * gg * gg;
    *m = mm;
    *v = vv;
    *sigma -= lr * (mm / (1.f - powf(b1, t))) / (sqrtf(vv / (1.f - powf(b2, t))) + eps);
}

void launch_sigma_adam(float *sigma, const double *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int32_t *step, hipStream_t s)
{
    hipLaunchKernelGGL(k_sigma_adam, dim3(1), dim3(1), 0, s, sigma, g, m, v, lr, b1, b2, eps, step);
}

}  // namespace oit
