// L1 + D-SSIM photometric loss of 3DGS, which the paper keeps (Sec. 5.1 "Implementation
// Details"): loss = sum_views (1 - lambda) mean|C - I| + lambda (1 - mean SSIM(C, I)).
// SSIM uses an 11 x 11 Gaussian window (std 1.5) with zero padding, C1 = 0.01^2,
// C2 = 0.03^2.  Two passes per view and channel, each on 16 x 16 pixel tiles with a
// 5-pixel halo staged in LDS and filtered separably:
//   k_ssim_stats: window means of x, y, x^2, y^2, xy -> SSIM and its partials with
//                 respect to the window mean of x, of x^2 and of xy;
//   k_ssim_grad:  the same window applied to those partial maps (the filter is its own
//                 adjoint) -> dL/dC, plus the L1 term.
#include "oit_internal.h"

namespace oit {

constexpr int kLT = 16;            // output tile edge
constexpr int kLR = 5;             // window radius
constexpr int kLH = kLT + 2 * kLR; // staged edge (26)
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

struct LossArgs2 {
    const CamDev *cams;
    int n_views, T16;              // 16 x 16 tiles over the batch (per channel)
    const float *image, *target;
    float *grad;
    float *maps;                   // [3 partials][3 ch][total_px]
    double *parts;                 // [2][blocks]: each block's share of sum |C - I| / (3HW), then of
                                   // sum SSIM / (3HW)
    int64_t total_px;
    float lambda;
    float g[11];
};

__device__ __forceinline__ void loss_tile(const LossArgs2 &a, int blk, int &v, int &ch, int &x0, int &y0)
{
    // blocks: view-major, then channel, then tile
    int rem = blk;
    v = 0;
    for (int k = 0; k < a.n_views; ++k) {
        const CamDev &c = a.cams[k];
        const int t = ((c.W + kLT - 1) / kLT) * ((c.H + kLT - 1) / kLT);
        if (rem < 3 * t) {
            v = k;
            break;
        }
        rem -= 3 * t;
    }
    const CamDev &c = a.cams[v];
    const int tx_n = (c.W + kLT - 1) / kLT;
    const int t = ((c.W + kLT - 1) / kLT) * ((c.H + kLT - 1) / kLT);
    ch = rem / t;
    const int lt = rem % t;
    x0 = (lt % tx_n) * kLT;
    y0 = (lt / tx_n) * kLT;
}

// The block's sum of v (lanes by a butterfly, waves in turn), written by thread 0 to
// *dst: each block's share is summed afterwards in a fixed order, so the loss value does
// not depend on the order in which the blocks finish.
__device__ __forceinline__ void block_share(double v, double *dst)
{
    __shared__ double s0[4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s0[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) *dst = s0[0] + s0[1] + s0[2] + s0[3];
}

// pass 1: window statistics, SSIM and its partials
__global__ __launch_bounds__(256) void k_ssim_stats(LossArgs2 a)
{
    __shared__ float sx[kLH][kLH], sy[kLH][kLH];
    __shared__ float hx[kLH][kLT], hy[kLH][kLT], hxx[kLH][kLT], hyy[kLH][kLT], hxy[kLH][kLT];
    int v, ch, x0, y0;
    loss_tile(a, blockIdx.x, v, ch, x0, y0);
    const CamDev &cam = a.cams[v];
    const size_t HW = (size_t)cam.W * cam.H;
    const float *X = a.image + 3 * (size_t)cam.pix_base + ch * HW;
    const float *Y = a.target + 3 * (size_t)cam.pix_base + ch * HW;
    for (int k = threadIdx.x; k < kLH * kLH; k += 256) {
        const int ly = k / kLH, lx = k % kLH;
        const int gx = x0 - kLR + lx, gy = y0 - kLR + ly;
        const bool in = gx >= 0 && gy >= 0 && gx < cam.W && gy < cam.H;
        sx[ly][lx] = in ? X[(size_t)gy * cam.W + gx] : 0.f;
        sy[ly][lx] = in ? Y[(size_t)gy * cam.W + gx] : 0.f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kLH * kLT; k += 256) {
        const int ly = k / kLT, lx = k % kLT;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float gx = a.g[d], xv = sx[ly][lx + d], yv = sy[ly][lx + d];
            s0 = fmaf(gx, xv, s0);
            s1 = fmaf(gx, yv, s1);
            s2 = fmaf(gx, xv * xv, s2);
            s3 = fmaf(gx, yv * yv, s3);
            s4 = fmaf(gx, xv * yv, s4);
        }
        hx[ly][lx] = s0;
        hy[ly][lx] = s1;
        hxx[ly][lx] = s2;
        hyy[ly][lx] = s3;
        hxy[ly][lx] = s4;
    }
    __syncthreads();
    const int lx = threadIdx.x % kLT, ly = threadIdx.x / kLT;
    const int px = x0 + lx, py = y0 + ly;
    double ssum = 0.0;
    if (px < cam.W && py < cam.H) {
        float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float gy = a.g[d];
            mx = fmaf(gy, hx[ly + d][lx], mx);
            my = fmaf(gy, hy[ly + d][lx], my);
            exx = fmaf(gy, hxx[ly + d][lx], exx);
            eyy = fmaf(gy, hyy[ly + d][lx], eyy);
            exy = fmaf(gy, hxy[ly + d][lx], exy);
        }
        const float A1 = 2.f * mx * my + kC1;
        const float A2 = 2.f * (exy - mx * my) + kC2;
        const float B1 = mx * mx + my * my + kC1;
        const float B2 = (exx - mx * mx) + (eyy - my * my) + kC2;
        const float S = (A1 * A2) / (B1 * B2);
        const float dmx = S * (2.f * my / A1 - 2.f * my / A2 - 2.f * mx / B1 + 2.f * mx / B2);
        const float dexx = -S / B2;
        const float dexy = 2.f * S / A2;
        const size_t pix = (size_t)cam.pix_base + (size_t)py * cam.W + px;
        const size_t plane = (size_t)a.total_px;
        a.maps[(0 * 3 + ch) * plane + pix] = dmx;
        a.maps[(1 * 3 + ch) * plane + pix] = dexx;
        a.maps[(2 * 3 + ch) * plane + pix] = dexy;
        ssum = (double)S / (3.0 * (double)HW);
    }
    block_share(ssum, a.parts + gridDim.x + blockIdx.x);
}

// pass 2: adjoint filtering of the partials, L1 term, dL/dC
__global__ __launch_bounds__(256) void k_ssim_grad(LossArgs2 a)
{
    __shared__ float sm[3][kLH][kLH];
    __shared__ float hm[3][kLH][kLT];
    int v, ch, x0, y0;
    loss_tile(a, blockIdx.x, v, ch, x0, y0);
    const CamDev &cam = a.cams[v];
    const size_t HW = (size_t)cam.W * cam.H;
    const size_t plane = (size_t)a.total_px;
    for (int k = threadIdx.x; k < kLH * kLH; k += 256) {
        const int ly = k / kLH, lx = k % kLH;
        const int gx = x0 - kLR + lx, gy = y0 - kLR + ly;
        const bool in = gx >= 0 && gy >= 0 && gx < cam.W && gy < cam.H;
        const size_t pix = (size_t)cam.pix_base + (size_t)gy * cam.W + gx;
#pragma unroll
        for (int m = 0; m < 3; ++m) sm[m][ly][lx] = in ? a.maps[(m * 3 + ch) * plane + pix] : 0.f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kLH * kLT; k += 256) {
        const int ly = k / kLT, lx = k % kLT;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float s = 0.f;
#pragma unroll
            for (int d = 0; d < 11; ++d) s = fmaf(a.g[d], sm[m][ly][lx + d], s);
            hm[m][ly][lx] = s;
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % kLT, ly = threadIdx.x / kLT;
    const int px = x0 + lx, py = y0 + ly;
    double l1 = 0.0;
    if (px < cam.W && py < cam.H) {
        float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int d = 0; d < 11; ++d) f[m] = fmaf(a.g[d], hm[m][ly + d][lx], f[m]);
        const size_t off = 3 * (size_t)cam.pix_base + ch * HW + (size_t)py * cam.W + px;
        const float x = a.image[off], y = a.target[off];
        const float inv = 1.f / (3.f * (float)HW);
        const float dl1 = x > y ? inv : (x < y ? -inv : 0.f);
        const float dssim = -(f[0] + 2.f * x * f[1] + y * f[2]) * inv;
        a.grad[off] = (1.f - a.lambda) * dl1 + a.lambda * dssim;
        l1 = fabs((double)x - (double)y) / (3.0 * (double)HW);
    }
    block_share(l1, a.parts + blockIdx.x);
}

__global__ void k_loss_combine(const double *acc, int n_views, float lambda, double *loss)
{
    // acc[1] holds sum over views of mean SSIM; D-SSIM sums (1 - mean SSIM) over views
    *loss = (1.0 - (double)lambda) * acc[0] + (double)lambda * ((double)n_views - acc[1]);
}

void launch_l1_dssim(const CamDev *cams, int n_views, int64_t total_px, int tiles16, const float *image,
                     const float *target, float lambda, float *grad, double *loss, float *maps, double *acc,
                     double *parts, hipStream_t s)
{
    LossArgs2 a;
    a.cams = cams;
    a.n_views = n_views;
    a.T16 = tiles16;
    a.image = image;
    a.target = target;
    a.grad = grad;
    a.maps = maps;
    a.parts = parts;
    a.total_px = total_px;
    a.lambda = lambda;
    double g[11], sum = 0.0;
    for (int k = 0; k < 11; ++k) {
        const double x = k - 5;
        g[k] = exp(-x * x / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < 11; ++k) a.g[k] = (float)(g[k] / sum);
    const unsigned blocks = (unsigned)(3 * tiles16);
    hipLaunchKernelGGL(k_ssim_stats, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ssim_grad, dim3(blocks), dim3(256), 0, s, a);
    launch_sum_shares(parts, (int)blocks, acc, s);
    launch_sum_shares(parts + blocks, (int)blocks, acc + 1, s);
    hipLaunchKernelGGL(k_loss_combine, dim3(1), dim3(1), 0, s, acc, n_views, lambda, loss);
}

}  // namespace oit
