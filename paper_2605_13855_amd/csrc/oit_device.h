// Device-side math of the OIT splat renderer, float32, shared by the forward and
// backward kernels so that both take bitwise-identical per-splat decisions.
//
// Screen-space model (Sec. 3.1): 3D covariance Sigma = R S S^T R^T from a quaternion
// and log-scales (Eq. "3d_gaussian"), EWA projection Sigma' = J W Sigma W^T J^T
// (Eq. "3dgs_proj") with the 3DGS low-pass +0.3 px^2 and 1.3x guard band, opacity
// alpha = o exp(-1/2 d^T Sigma'^-1 d) (Eq. "3dgs_alpha"), colour from degree-3 SH at
// the viewing direction (Eq. "3dgs_color"), weight w = max(0, 1 - d/sigma) v(r)
// (Eq. "sf_weight").  The opacity is evaluated as alpha = 2^e with
// e = log2(o) + qa dx^2 + qb dx dy + qc dy^2 (q* = the conic scaled by -log2(e)/2),
// so that the "alpha >= 1/255" test is a compare on e before any exponential.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oit {

constexpr float kAlphaMax = 0.99f;
constexpr float kLog2AlphaMax = -0.01449956969511509f;   // log2(0.99)
constexpr float kLog2AlphaMin = -7.994353436858858f;     // log2(1/255)
// A splat whose log2 opacity is below kLog2NoCap never reaches the opacity cap: the
// exponent at any pixel is at most log2(opacity) plus rounding, far below the margin.
constexpr float kLog2NoCap = kLog2AlphaMax - 1e-4f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kDilation = 0.3f;
constexpr float kGuardBand = 1.3f;
constexpr float kColorOffset = 0.5f;

// Per-view constants, in device memory (uploaded by a kernel so that graph capture
// records them by value).  128 bytes.
struct CamDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float near_z, lim_x, lim_y;
    float cc[3];      // camera centre -R^T t
    int W, H;
    int tiles_x, tiles_y;
    int tile_base;    // first tile of this view in the batch
    int pix_base;     // first pixel of this view in the batch
    int pad[2];
};

// Record of one (view, listed splat), 3 x float4 = 48 bytes used, read by the
// rasterisers, padded to 64 bytes: a record is gathered alone (its tile's list orders
// the records by tile, not by address), and at a 64-byte stride it takes one memory
// sector instead of one or two.
//   a = (mx, my, qa, qb)   b = (qc, lo, c_r, c_g)   c = (c_b, wv, dd, sgn)
// active records: wv = w,  dd = dw/dsigma (0 when d >= sigma),  sgn = 1
// label-change records: wv = v (0 when d >= sigma), dd = d, sgn = -1 (leaves pre) / +1
struct Rec {
    float4 a, b, c;
    float4 pad;   // never written or read
};

// ---------------------------------------------------------------------------------
// Spherical harmonics, degree 3, real basis in the 3DGS sign convention.
// ---------------------------------------------------------------------------------
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.4886025119029199f;
constexpr float kSH2a = 1.0925484305920792f;
constexpr float kSH2b = 0.31539156525252005f;
constexpr float kSH2c = 0.5462742152960396f;
constexpr float kSH3a = 0.5900435899266435f;
constexpr float kSH3b = 2.890611442640554f;
constexpr float kSH3c = 0.4570457994644658f;
constexpr float kSH3d = 0.3731763325901154f;
constexpr float kSH3e = 1.445305721320277f;

__device__ __forceinline__ void sh_eval(float x, float y, float z, float Y[16])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = kSH0;
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2.f * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    Y[9] = -kSH3a * y * (3.f * xx - yy);
    Y[10] = kSH3b * x * y * z;
    Y[11] = -kSH3c * y * (4.f * zz - xx - yy);
    Y[12] = kSH3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -kSH3c * x * (4.f * zz - xx - yy);
    Y[14] = kSH3e * z * (xx - yy);
    Y[15] = -kSH3a * x * (xx - 3.f * yy);
}

// Vector-Jacobian product: out = sum_k g[k] dY_k/d(x, y, z).
__device__ __forceinline__ void sh_vjp(float x, float y, float z, const float g[16], float out[3])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    gy += -kSH1 * g[1];
    gz += kSH1 * g[2];
    gx += -kSH1 * g[3];
    gx += kSH2a * y * g[4];                 gy += kSH2a * x * g[4];
    gy += -kSH2a * z * g[5];                gz += -kSH2a * y * g[5];
    gx += -2.f * kSH2b * x * g[6];          gy += -2.f * kSH2b * y * g[6];   gz += 4.f * kSH2b * z * g[6];
    gx += -kSH2a * z * g[7];                gz += -kSH2a * x * g[7];
    gx += 2.f * kSH2c * x * g[8];           gy += -2.f * kSH2c * y * g[8];
    gx += -6.f * kSH3a * x * y * g[9];      gy += -kSH3a * (3.f * xx - 3.f * yy) * g[9];
    gx += kSH3b * y * z * g[10];            gy += kSH3b * x * z * g[10];     gz += kSH3b * x * y * g[10];
    gx += 2.f * kSH3c * x * y * g[11];
    gy += -kSH3c * (4.f * zz - xx - 3.f * yy) * g[11];
    gz += -8.f * kSH3c * y * z * g[11];
    gx += -6.f * kSH3d * x * z * g[12];
    gy += -6.f * kSH3d * y * z * g[12];
    gz += kSH3d * (6.f * zz - 3.f * xx - 3.f * yy) * g[12];
    gx += -kSH3c * (4.f * zz - 3.f * xx - yy) * g[13];
    gy += 2.f * kSH3c * x * y * g[13];
    gz += -8.f * kSH3c * x * z * g[13];
    gx += 2.f * kSH3e * x * z * g[14];      gy += -2.f * kSH3e * y * z * g[14];  gz += kSH3e * (xx - yy) * g[14];
    gx += -kSH3a * (3.f * xx - 3.f * yy) * g[15];
    gy += 6.f * kSH3a * x * y * g[15];
    out[0] = gx;
    out[1] = gy;
    out[2] = gz;
}

// ---------------------------------------------------------------------------------
// Geometry of one splat in one view.
// ---------------------------------------------------------------------------------
struct Geo {
    float tc[3];        // camera-space mean
    int clamp_x, clamp_y;
    float J00, J02, J11, J12;
    float T[6];         // J W, 2x3 row-major
    float cov_a, cov_b, cov_c;   // Sigma' incl. dilation
    float det;
    float con_a, con_b, con_c;   // conic
    float mx, my;
};

// Rotation of the unit quaternion (w, x, y, z).
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float Rq[9])
{
    Rq[0] = 1.f - 2.f * (y * y + z * z);
    Rq[1] = 2.f * (x * y - w * z);
    Rq[2] = 2.f * (x * z + w * y);
    Rq[3] = 2.f * (x * y + w * z);
    Rq[4] = 1.f - 2.f * (x * x + z * z);
    Rq[5] = 2.f * (y * z - w * x);
    Rq[6] = 2.f * (x * z - w * y);
    Rq[7] = 2.f * (y * z + w * x);
    Rq[8] = 1.f - 2.f * (x * x + y * y);
}

// 3D covariance (6 unique entries xx, xy, xz, yy, yz, zz) of M M^T, M = Rq diag(s).
__device__ __forceinline__ void cov3d(const float Rq[9], const float s[3], float S6[6])
{
    float M[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * s[b];
    S6[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    S6[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    S6[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    S6[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    S6[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    S6[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
}

// Camera-space mean, EWA Jacobian, screen covariance and conic.  Returns false when
// the splat is culled (depth <= near plane or a degenerate screen covariance).
__device__ __forceinline__ bool geometry(const CamDev &cam, const float mu[3], const float S6[6], Geo &g)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
        g.tc[r] = cam.R[3 * r] * mu[0] + cam.R[3 * r + 1] * mu[1] + cam.R[3 * r + 2] * mu[2] + cam.t[r];
    const float tz = g.tc[2];
    if (!(tz > cam.near_z)) return false;
    const float itz = 1.f / tz;
    float rx = g.tc[0] * itz, ry = g.tc[1] * itz;
    g.clamp_x = rx > cam.lim_x ? 1 : (rx < -cam.lim_x ? -1 : 0);
    g.clamp_y = ry > cam.lim_y ? 1 : (ry < -cam.lim_y ? -1 : 0);
    rx = fminf(fmaxf(rx, -cam.lim_x), cam.lim_x);
    ry = fminf(fmaxf(ry, -cam.lim_y), cam.lim_y);
    // J = [[fx/tz, 0, -fx rx/tz], [0, fy/tz, -fy ry/tz]]  (rx = clamped tx/tz)
    g.J00 = cam.fx * itz;
    g.J02 = -cam.fx * rx * itz;
    g.J11 = cam.fy * itz;
    g.J12 = -cam.fy * ry * itz;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        g.T[b] = g.J00 * cam.R[b] + g.J02 * cam.R[6 + b];
        g.T[3 + b] = g.J11 * cam.R[3 + b] + g.J12 * cam.R[6 + b];
    }
    // U = T Sigma
    const float Sg[9] = {S6[0], S6[1], S6[2], S6[1], S6[3], S6[4], S6[2], S6[4], S6[5]};
    float U[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            U[3 * a + b] = g.T[3 * a] * Sg[b] + g.T[3 * a + 1] * Sg[3 + b] + g.T[3 * a + 2] * Sg[6 + b];
    g.cov_a = U[0] * g.T[0] + U[1] * g.T[1] + U[2] * g.T[2] + kDilation;
    g.cov_b = U[0] * g.T[3] + U[1] * g.T[4] + U[2] * g.T[5];
    g.cov_c = U[3] * g.T[3] + U[4] * g.T[4] + U[5] * g.T[5] + kDilation;
    g.det = g.cov_a * g.cov_c - g.cov_b * g.cov_b;
    if (!(g.det > 0.f)) return false;
    const float idet = 1.f / g.det;
    g.con_a = g.cov_c * idet;
    g.con_b = -g.cov_b * idet;
    g.con_c = g.cov_a * idet;
    g.mx = cam.fx * g.tc[0] * itz + cam.cx;
    g.my = cam.fy * g.tc[1] * itz + cam.cy;
    return true;
}

// Opacity exponent e (alpha = 2^e, see the file comment) at a pixel of a tile.  Both
// raster passes form it with the same float operations, so they take identical
// per-pair decisions:
//   dx = (x0 - mx) + col,  dy = (y0 - my) + row     (x0, y0: centre of the tile's
//                                                    first pixel; col, row: offsets)
//   e  = fma(dy, fma(qc, dy, qb dx), fma(qa dx, dx, lo)).
// The two per-column terms are exp_col_b and exp_col_c; a pixel adds two FMAs.
__device__ __forceinline__ float exp_col_b(float qb, float dx) { return qb * dx; }
__device__ __forceinline__ float exp_col_c(float qa, float lo, float dx) { return fmaf(qa * dx, dx, lo); }
__device__ __forceinline__ float exp_pix(float qc, float dy, float colb, float colc)
{
    return fmaf(dy, fmaf(qc, dy, colb), colc);
}

// Conservative test: does the ellipse {m(d) <= tau}, m = A dx^2 + 2B dx dy + C dy^2,
// reach the rectangle [x0, x1] x [y0, y1] (coordinates relative to the mean)?
// Exact minimum of the convex form over the rectangle; evaluated without
// contraction so that every caller takes the same decision for the same inputs.
__device__ __forceinline__ bool ellipse_hits_rect(float A, float B, float C, float tau,
                                                  float x0, float x1, float y0, float y1)
{
#pragma clang fp contract(off)
    if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
    float best = 3.0e38f;
    // edges x = x0, x = x1: minimise over dy
    const float xs[2] = {x0, x1};
    const float ys[2] = {y0, y1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float dx = xs[k];
        float dy = -B * dx / C;
        dy = fminf(fmaxf(dy, y0), y1);
        const float m = A * dx * dx + 2.f * B * dx * dy + C * dy * dy;
        best = fminf(best, m);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float dy = ys[k];
        float dx = -B * dy / A;
        dx = fminf(fmaxf(dx, x0), x1);
        const float m = A * dx * dx + 2.f * B * dx * dy + C * dy * dy;
        best = fminf(best, m);
    }
    return best <= tau;
}

}  // namespace oit
