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
    float b1, b2, eps;
    const int32_t *step;
};

__device__ __constant__ const int kGroupStart[7] = {0, 3, 6, 10, 11, 59, 75};

// grid.y = component (75), grid.x covers the active rows
__global__ __launch_bounds__(256) void k_sparse_adam(AdamArgs a)
{
    // bias corrections of this step, once per block
    __shared__ float s_bc[2];
    if (threadIdx.x == 0) {
        const float t = (float)*a.step;
        s_bc[0] = 1.f - powf(a.b1, t);
        s_bc[1] = 1.f - powf(a.b2, t);
    }
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t na = a.n_active ? (int64_t)*a.n_active : a.n;
    if (r >= na) return;
    const int c = blockIdx.y;
    int grp = 0;
#pragma unroll
    for (int k = 1; k < 6; ++k)
        if (c >= kGroupStart[k]) grp = k;
    const int sub = c - kGroupStart[grp];
    const int64_t id = a.idx ? (int64_t)a.idx[r] : r;
    const size_t pi = (size_t)sub * a.n + id;
    const float g = a.p.g[grp][(size_t)sub * a.gstride + r];
    const float bc1 = s_bc[0], bc2 = s_bc[1];
    const float m = a.b1 * a.p.m[grp][pi] + (1.f - a.b1) * g;
    const float v = a.b2 * a.p.v[grp][pi] + (1.f - a.b2) * g * g;
    a.p.m[grp][pi] = m;
    a.p.v[grp][pi] = v;
    a.p.p[grp][pi] -= a.p.lr[grp] * (m / bc1) / (sqrtf(v / bc2) + a.eps);
}

void launch_sparse_adam(const AdamPtrs &p, int64_t gstride, const int32_t *active_idx, const int32_t *n_active,
                        int64_t n, int64_t rows_cap, float b1, float b2, float eps, int32_t *step,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, s, step);
    AdamArgs a{p, gstride, active_idx, n_active, n, b1, b2, eps, step};
    const unsigned bx = (unsigned)((rows_cap + 255) / 256);
    if (bx) hipLaunchKernelGGL(k_sparse_adam, dim3(bx, 75), dim3(256), 0, s, a);
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
