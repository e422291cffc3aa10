// Backward pass: L1 loss gradient, per-pixel constants of the OIT partials, the
// per-splat raster backward and the chain rule to the splat parameters and sigma
// (App. B, Eqs. "oit_rendering_md" and "oit_rendering_detail").
#include "oit_internal.h"

namespace oit {

// Sum of a double over the block, added once to *dst.
__device__ __forceinline__ void block_add_double(double v, double *dst)
{
    __shared__ double s_part[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s_part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) t += s_part[w];
        if (t != 0.0) unsafeAtomicAdd(dst, t);
    }
}

__device__ __forceinline__ int view_of_pixel(const CamDev *cams, int n_views, int64_t gp)
{
    int v = 0;
    for (int k = 1; k < n_views; ++k)
        if (gp >= cams[k].pix_base) v = k;
    return v;
}

// ---------------------------------------------------------------------------------
// L1 loss: loss = sum_views mean |C - I|, grad = sign(C - I) / (3 H W)
// ---------------------------------------------------------------------------------
struct LossArgs {
    Buffers b;
    const float *image, *target;
    float *grad;
    double *loss;
};

__global__ __launch_bounds__(256) void k_l1_loss(LossArgs a)
{
    const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (gp < a.b.total_px) {
        const int v = view_of_pixel(a.b.cams, a.b.n_views, gp);
        const CamDev &cam = a.b.cams[v];
        const size_t HW = (size_t)cam.W * cam.H;
        const size_t local = (size_t)(gp - cam.pix_base);
        const size_t base = 3 * (size_t)cam.pix_base + local;
        const float inv = 1.f / (3.f * (float)HW);
        const double dinv = 1.0 / (3.0 * (double)HW);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = a.image[base + ch * HW] - a.target[base + ch * HW];
            a.grad[base + ch * HW] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
            acc += fabs((double)d) * dinv;
        }
    }
    block_add_double(acc, a.loss);
}

void launch_l1_loss(const Buffers &b, const float *image, const float *target, float *grad, double *loss,
                    hipStream_t s)
{
    fill_f64(loss, 1, 0.0, s);
    LossArgs a{b, image, target, grad, loss};
    const unsigned blocks = (unsigned)((b.total_px + 255) / 256);
    if (blocks) hipLaunchKernelGGL(k_l1_loss, dim3(blocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------------
// per-pixel constants of the partials:
//   A_ch = g_ch (1 - T) / Q   (0 if Q <= 0),  s1 = sum_ch A_ch F_ch,
//   B    = T sum_ch g_ch (F_ch - c0_ch)
// so that for a contributing pair  dL/dc = A alpha w,  dL/dw = alpha (A.c - s1),
//   dL/dalpha = B / (1 - alpha) + w (A.c - s1).
// The inactive set's share of dL/dsigma, sum_ch A_ch (P1_ch - F_ch Q1) / sigma^2, is
// summed here from the pre-rendered accumulators.
// ---------------------------------------------------------------------------------
struct PixArgs {
    Buffers b;
    const float *sigma;
    float bg0, bg1, bg2;
    const float *pre, *grad, *pixstate;
    double *grad_sigma;
};

__global__ __launch_bounds__(256) void k_pixconst(PixArgs a)
{
    const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (gp < a.b.total_px) {
        const int v = view_of_pixel(a.b.cams, a.b.n_views, gp);
        const CamDev &cam = a.b.cams[v];
        const size_t HW = (size_t)cam.W * cam.H;
        const size_t local = (size_t)(gp - cam.pix_base);
        const size_t pb = (size_t)cam.pix_base;
        const float *ps = a.pixstate + 5 * pb + local;
        const float *gr = a.grad + 3 * pb + local;
        const float T = ps[0], Q = ps[HW];
        const float F[3] = {ps[2 * HW], ps[3 * HW], ps[4 * HW]};
        const float g[3] = {gr[0], gr[HW], gr[2 * HW]};
        const float k = Q > 0.f ? (1.f - T) / Q : 0.f;
        const float A0 = g[0] * k, A1 = g[1] * k, A2 = g[2] * k;
        const float s1 = A0 * F[0] + A1 * F[1] + A2 * F[2];
        const float B = T * (g[0] * (F[0] - a.bg0) + g[1] * (F[1] - a.bg1) + g[2] * (F[2] - a.bg2));
        a.b.pixconst[2 * gp] = make_float4(A0, A1, A2, s1);
        a.b.pixconst[2 * gp + 1] = make_float4(B, 0.f, 0.f, 0.f);
        if (a.pre) {
            const float *pr = a.pre + 9 * pb + local;
            const float Q1 = pr[7 * HW];
            const double sig = (double)*a.sigma;
            acc = ((double)A0 * ((double)pr[3 * HW] - (double)F[0] * Q1) +
                   (double)A1 * ((double)pr[4 * HW] - (double)F[1] * Q1) +
                   (double)A2 * ((double)pr[5 * HW] - (double)F[2] * Q1)) / (sig * sig);
        }
    }
    if (a.pre) block_add_double(acc, a.grad_sigma);
}

void launch_pixconst(const Buffers &b, const float *sigma, const float bg[3], const float *pre,
                     const float *grad_image, const float *pixstate, double *grad_sigma, hipStream_t s)
{
    PixArgs a{b, sigma, bg[0], bg[1], bg[2], pre, grad_image, pixstate, grad_sigma};
    const unsigned blocks = (unsigned)((b.total_px + 255) / 256);
    if (blocks) hipLaunchKernelGGL(k_pixconst, dim3(blocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------------
// raster backward: one wave per work item = (tile, 64 active entries); one splat per
// lane.  The wave stages 64 pixels' constants in its own LDS slice (every lane
// fetches one pixel once) and then every lane walks those 64 pixels in turn, so all
// per-splat sums stay in registers; they are added to the per-(view, record)
// screen-space gradient once per work item.
// Screen-space gradient layout (10 floats): d/dmx, d/dmy, d/dqa, d/dqb, d/dqc, d/dlo,
// d/dc (rgb), d/dw — q* and lo as in the record.
// ---------------------------------------------------------------------------------
struct BwdArgs {
    Buffers b;
};

template <int S>
__global__ __launch_bounds__(256) void k_raster_bwd(BwdArgs a)
{
    __shared__ float4 s_pc[4][64][2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t total = a.b.counters[CNT_TOTAL_CHUNKS];
    const uint64_t cap = (uint64_t)a.b.pair_cap;
    constexpr int GROUPS = S * S / 64;
    constexpr int ROWS = 64 / S > 0 ? 64 / S : 1;   // tile rows per group (S >= 8)

    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(&a.b.counters[CNT_BWD_WORK], 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        int lo_t = 0, hi_t = a.b.T;
        while (hi_t - lo_t > 1) {
            const int mid = (lo_t + hi_t) >> 1;
            if (a.b.chunk_off[mid] <= item) lo_t = mid;
            else hi_t = mid;
        }
        const int tile = lo_t;
        const uint32_t chunk = item - a.b.chunk_off[tile];
        const int v = view_of_tile(a.b.cams, a.b.n_views, tile);
        const CamDev &cam = a.b.cams[v];
        const int lt = tile - cam.tile_base;
        const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
        const uint64_t off = a.b.tile_off[tile];
        uint64_t na = a.b.cnt_a[tile];
        if (off + na > cap) na = off < cap ? cap - off : 0;
        const uint64_t j = (uint64_t)chunk * 64 + lane;
        const uint32_t rj = j < na ? a.b.entries[off + j] : 0u;
        const bool valid = j < na && rj < a.b.Acap;
        uint32_t r = 0;
        float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = make_float4(0.f, -1e30f, 0.f, 0.f),
               rc = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) {
            r = rj;
            const Rec rr = a.b.rec[(size_t)v * a.b.Rcap + r];
            ra = rr.a;
            rb = rr.b;
            rc = rr.c;
        }
        const float mx = ra.x, my = ra.y, qa = ra.z, qb = ra.w, qc = rb.x, lo = rb.y;
        const float cr = rb.z, cg = rb.w, cb = rc.x, w = rc.y;
        // vertical extent of the footprint, to skip pixel groups no lane reaches
        float ylo = 1e30f, yhi = -1e30f;
        if (valid) {
            const float A = -qa, B = -0.5f * qb, C = -qc;
            const float det = A * C - B * B;
            const float tau = (lo - kLog2AlphaMin) * 1.001f + 1e-3f;
            if (tau > 0.f && det > 0.f) {
                const float hy = sqrtf(tau * A / det) + 0.01f;
                ylo = my - hy;
                yhi = my + hy;
            }
        }
        float g_mx = 0.f, g_my = 0.f, g_qa = 0.f, g_qb = 0.f, g_qc = 0.f, g_lo = 0.f;
        float g_cr = 0.f, g_cg = 0.f, g_cb = 0.f, g_w = 0.f;
        const size_t pb = (size_t)cam.pix_base;
        const int cols = min(S, cam.W - tx * S);   // in-image columns of this tile

        for (int grp = 0; grp < GROUPS; ++grp) {
            const float gy0 = (float)(ty * S + grp * ROWS) + 0.5f;
            const float gy1 = gy0 + (float)(ROWS - 1);
            const bool hit = (ylo <= gy1) && (yhi >= gy0);
            if (__ballot(hit) == 0) continue;
            // stage this group's pixel constants: lane = pixel
            {
                const int p = grp * 64 + lane;
                const int x = tx * S + p % S, y = ty * S + p / S;
                float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (x < cam.W && y < cam.H) {
                    const size_t gp = pb + (size_t)y * cam.W + x;
                    c0 = a.b.pixconst[2 * gp];
                    c1 = a.b.pixconst[2 * gp + 1];
                }
                s_pc[wave][lane][0] = c0;
                s_pc[wave][lane][1] = c1;
            }
            __builtin_amdgcn_wave_barrier();
            // walk the group row by row; per-row terms of the exponent are hoisted, and
            // the exponent is formed with the same operations as alpha_exponent() so that
            // forward and backward take identical decisions for every pair
            for (int row = 0; row < ROWS; ++row) {
                const int y = ty * S + grp * ROWS + row;
                if (y >= cam.H) break;
                const float dy = ((float)y + 0.5f) - my;
                const float qbdy = qb * dy;
                const float cterm = fmaf(qc * dy, dy, lo);
#pragma unroll
                for (int col = 0; col < S; ++col) {
                    if (col >= cols) break;
                    const float dx = ((float)(tx * S + col) + 0.5f) - mx;
                    const float e = fmaf(dx, fmaf(qa, dx, qbdy), cterm);
                    if (e >= kLog2AlphaMin) {
                        const int jj = row * S + col;
                        const float4 c0 = s_pc[wave][jj][0];
                        const bool capped = e > kLog2AlphaMax;
                        const float al = capped ? kAlphaMax : __builtin_amdgcn_exp2f(e);
                        const float diff = fmaf(c0.x, cr, fmaf(c0.y, cg, c0.z * cb)) - c0.w;
                        const float aw = al * w;
                        g_cr = fmaf(c0.x, aw, g_cr);
                        g_cg = fmaf(c0.y, aw, g_cg);
                        g_cb = fmaf(c0.z, aw, g_cb);
                        g_w = fmaf(al, diff, g_w);
                        if (!capped) {
                            const float Bc = s_pc[wave][jj][1].x;
                            // dL/dalpha = B / (1 - alpha) + w diff;  d alpha / de = alpha ln 2
                            // (the ln 2 is applied once per work item, below)
                            const float dLda = fmaf(w, diff, Bc * __builtin_amdgcn_rcpf(1.f - al));
                            const float dLde = dLda * al;
                            g_lo += dLde;
                            const float ex = dLde * dx, ey = dLde * dy;
                            g_qa = fmaf(ex, dx, g_qa);
                            g_qb = fmaf(ex, dy, g_qb);
                            g_qc = fmaf(ey, dy, g_qc);
                            // de/dmx = -(2 qa dx + qb dy), de/dmy = -(qb dx + 2 qc dy)
                            g_mx -= fmaf(2.f * qa, ex, qb * ey);
                            g_my -= fmaf(qb, ex, 2.f * qc * ey);
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (valid) {
            float *dst = a.b.sgrad + ((size_t)v * a.b.Acap + r) * 10;
            const float vals[10] = {g_mx * kLn2, g_my * kLn2, g_qa * kLn2, g_qb * kLn2, g_qc * kLn2, g_lo * kLn2,
                                    g_cr, g_cg, g_cb, g_w};
#pragma unroll
            for (int k = 0; k < 10; ++k)
                if (vals[k] != 0.f) unsafeAtomicAdd(dst + k, vals[k]);
        }
    }
}

// ---------------------------------------------------------------------------------
// raster backward, per-pixel form (the 3DGS baseline of the paper's ablation): one
// thread per pixel walks its tile's active entries (staged through LDS like the
// forward) and adds the 10 screen-space partials of every contributing pair to the
// splat with one atomic each.  Same partials as k_raster_bwd; kept for comparison.
// ---------------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(S * S < 256 ? S * S : 256) void k_raster_bwd_pixel(BwdArgs a)
{
    constexpr int NT = S * S < 256 ? S * S : 256;
    constexpr int PPT = S * S / NT;
    constexpr int B = 64;
    __shared__ float4 s_rec[B * 3];
    __shared__ uint32_t s_r[B];
    const int tile = blockIdx.x;
    const int v = view_of_tile(a.b.cams, a.b.n_views, tile);
    const CamDev &cam = a.b.cams[v];
    const int lt = tile - cam.tile_base;
    const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
    float px[PPT], py[PPT], A0[PPT], A1[PPT], A2[PPT], s1[PPT], Bc[PPT];
    bool in[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int li = threadIdx.x + p * NT;
        const int x = tx * S + li % S, y = ty * S + li / S;
        px[p] = (float)x + 0.5f;
        py[p] = (float)y + 0.5f;
        in[p] = x < cam.W && y < cam.H;
        float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (in[p]) {
            const size_t gp = (size_t)cam.pix_base + (size_t)y * cam.W + x;
            c0 = a.b.pixconst[2 * gp];
            c1 = a.b.pixconst[2 * gp + 1];
        }
        A0[p] = c0.x;
        A1[p] = c0.y;
        A2[p] = c0.z;
        s1[p] = c0.w;
        Bc[p] = c1.x;
    }
    const uint64_t cap = (uint64_t)a.b.pair_cap;
    const uint64_t off = a.b.tile_off[tile];
    uint64_t na = a.b.cnt_a[tile];
    if (off + na > cap) na = off < cap ? cap - off : 0;
    const Rec *recv = a.b.rec + (size_t)v * a.b.Rcap;
    for (uint64_t base = 0; base < na; base += B) {
        const int cnt = (int)(na - base < (uint64_t)B ? na - base : (uint64_t)B);
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += NT) {
            const uint32_t ri = a.b.entries[off + base + j];
            const bool ok = ri < a.b.Acap;
            const Rec r = ok ? recv[ri] : Rec{{0.f, 0.f, 0.f, 0.f}, {0.f, -1e30f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
            s_rec[3 * j] = r.a;
            s_rec[3 * j + 1] = r.b;
            s_rec[3 * j + 2] = r.c;
            s_r[j] = ok ? ri : 0u;
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const float4 ra = s_rec[3 * j], rb = s_rec[3 * j + 1], rc = s_rec[3 * j + 2];
            float *dst = a.b.sgrad + ((size_t)v * a.b.Acap + s_r[j]) * 10;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                if (!in[p]) continue;
                const float dx = px[p] - ra.x, dy = py[p] - ra.y;
                const float e = alpha_exponent(rb.y, ra.z, ra.w, rb.x, dx, dy);
                if (e < kLog2AlphaMin) continue;
                const bool capped = e > kLog2AlphaMax;
                const float al = capped ? kAlphaMax : __builtin_amdgcn_exp2f(e);
                const float w = rc.y;
                const float diff = fmaf(A0[p], rb.z, fmaf(A1[p], rb.w, A2[p] * rc.x)) - s1[p];
                const float aw = al * w;
                unsafeAtomicAdd(dst + 6, A0[p] * aw);
                unsafeAtomicAdd(dst + 7, A1[p] * aw);
                unsafeAtomicAdd(dst + 8, A2[p] * aw);
                unsafeAtomicAdd(dst + 9, al * diff);
                if (!capped) {
                    const float dLde = fmaf(w, diff, Bc[p] * __builtin_amdgcn_rcpf(1.f - al)) * al * kLn2;
                    const float ex = dLde * dx, ey = dLde * dy;
                    unsafeAtomicAdd(dst + 0, -fmaf(2.f * ra.z, ex, ra.w * ey));
                    unsafeAtomicAdd(dst + 1, -fmaf(ra.w, ex, 2.f * rb.x * ey));
                    unsafeAtomicAdd(dst + 2, ex * dx);
                    unsafeAtomicAdd(dst + 3, ex * dy);
                    unsafeAtomicAdd(dst + 4, ey * dy);
                    unsafeAtomicAdd(dst + 5, dLde);
                }
            }
        }
    }
}

bool launch_raster_bwd(const Buffers &b, const RowList &rl, hipStream_t s)
{
    (void)rl;
    BwdArgs a{b};
    if (b.bwd_mode == OIT_BWD_PER_PIXEL) {
        if (b.T == 0) return true;
        switch (b.tile) {
        case 8: hipLaunchKernelGGL(k_raster_bwd_pixel<8>, dim3(b.T), dim3(64), 0, s, a); return true;
        case 16: hipLaunchKernelGGL(k_raster_bwd_pixel<16>, dim3(b.T), dim3(256), 0, s, a); return true;
        case 32: hipLaunchKernelGGL(k_raster_bwd_pixel<32>, dim3(b.T), dim3(256), 0, s, a); return true;
        default: return false;
        }
    }
    const dim3 grid(1024), block(256);
    switch (b.tile) {
    case 8: hipLaunchKernelGGL(k_raster_bwd<8>, grid, block, 0, s, a); return true;
    case 16: hipLaunchKernelGGL(k_raster_bwd<16>, grid, block, 0, s, a); return true;
    case 32: hipLaunchKernelGGL(k_raster_bwd<32>, grid, block, 0, s, a); return true;
    default: return false;
    }
}

// ---------------------------------------------------------------------------------
// preprocess backward: one thread per active row; chain rule from the per-view
// screen-space gradients to every parameter (Sec. 3.1 model) and to sigma.
// ---------------------------------------------------------------------------------
struct PreBwdArgs {
    SplatPtrs sp;
    const float *sigma;
    RowList rl;
    Buffers b;
    GradPtrs g;
    double *grad_sigma;
    float *score;
    float eps[6];
};

__global__ __launch_bounds__(256) void k_preprocess_bwd(PreBwdArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double gsig = 0.0;
    const int64_t na = a.rl.n_active ? (int64_t)*a.rl.n_active : a.rl.n_active_host;
    if (t < a.rl.Acap && t < na) {
        const int64_t id = a.rl.active_idx ? (int64_t)a.rl.active_idx[t] : t;
        const int64_t n = a.sp.n;
        const float sigma = *a.sigma;
        float mu[3], s[3], q[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mu[k] = a.sp.mean[k * n + id];
            s[k] = expf(a.sp.log_scale[k * n + id]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = a.sp.quat[k * n + id];
        const float qlen = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float qi = 1.f / qlen;
        const float qn[4] = {q[0] * qi, q[1] * qi, q[2] * qi, q[3] * qi};
        float Rq[9], S6[6];
        quat_rot(qn[0], qn[1], qn[2], qn[3], Rq);
        cov3d(Rq, s, S6);
        const float lg = a.sp.logit[id];
        const float o = 1.f / (1.f + expf(-lg));

        float g_mu[3] = {0.f, 0.f, 0.f};
        float G6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float g_sh[48], g_vsh[16];
#pragma unroll
        for (int k = 0; k < 48; ++k) g_sh[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) g_vsh[k] = 0.f;
        float g_lo = 0.f;

        for (int v = 0; v < a.b.n_views; ++v) {
            const float *sg = a.b.sgrad + ((size_t)v * a.b.Acap + t) * 10;
            float gs[10];
            bool any = false;
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                gs[k] = sg[k];
                any |= gs[k] != 0.f;
            }
            if (!any) continue;
            const CamDev &cam = a.b.cams[v];
            Geo g;
            if (!geometry(cam, mu, S6, g)) continue;
            const float tz = g.tc[2], itz = 1.f / tz;
            float g_tc[3] = {0.f, 0.f, 0.f};
            g_lo += gs[5];

            // appearance: colour and view weight at the viewing direction
            float u[3] = {mu[0] - cam.cc[0], mu[1] - cam.cc[1], mu[2] - cam.cc[2]};
            const float dist = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            const float idist = 1.f / dist;
            const float dir[3] = {u[0] * idist, u[1] * idist, u[2] * idist};
            float Y[16];
            sh_eval(dir[0], dir[1], dir[2], Y);
            float gY[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) gY[k] = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float raw = kColorOffset;
#pragma unroll
                for (int k = 0; k < 16; ++k) raw += Y[k] * a.sp.sh[(3 * k + ch) * n + id];
                if (raw > 0.f) {
                    const float gc = gs[6 + ch];
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        g_sh[3 * k + ch] = fmaf(gc, Y[k], g_sh[3 * k + ch]);
                        gY[k] = fmaf(gc, a.sp.sh[(3 * k + ch) * n + id], gY[k]);
                    }
                }
            }
            {
                float raw = kColorOffset;
#pragma unroll
                for (int k = 0; k < 16; ++k) raw += Y[k] * a.sp.vsh[k * n + id];
                const float vv = fmaxf(raw, 0.f);
                const float gw = gs[9];
                if (tz < sigma) {
                    const float gv = gw * (1.f - tz / sigma);
                    g_tc[2] += -gw * vv / sigma;
                    gsig += (double)gw * (double)vv * (double)tz / ((double)sigma * (double)sigma);
                    if (raw > 0.f) {
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            g_vsh[k] = fmaf(gv, Y[k], g_vsh[k]);
                            gY[k] = fmaf(gv, a.sp.vsh[k * n + id], gY[k]);
                        }
                    }
                }
            }
            float gdir[3];
            sh_vjp(dir[0], dir[1], dir[2], gY, gdir);
            {
                const float dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
#pragma unroll
                for (int k = 0; k < 3; ++k) g_mu[k] += (gdir[k] - dir[k] * dd) * idist;
            }

            // conic (scaled): qa = h A, qb = 2 h B, qc = h C with h = -log2(e)/2
            const float h = -0.5f * kLog2e;
            const float gA = h * gs[2], gB = 2.f * h * gs[3], gC = h * gs[4];
            // conic = cov^-1: G_cov = -K G K with G = [[gA, gB/2], [gB/2, gC]]
            const float A = g.con_a, Bk = g.con_b, C = g.con_c, hb = 0.5f * gB;
            const float ga = -(A * A * gA + 2.f * A * Bk * hb + Bk * Bk * gC);
            const float gb = -2.f * (A * Bk * gA + (Bk * Bk + A * C) * hb + Bk * C * gC);
            const float gcc = -(Bk * Bk * gA + 2.f * Bk * C * hb + C * C * gC);
            // cov = T Sigma T^T + 0.3 I
            const float Sg[9] = {S6[0], S6[1], S6[2], S6[1], S6[3], S6[4], S6[2], S6[4], S6[5]};
            float V[6];
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
                    V[3 * aa + bb] = g.T[3 * aa] * Sg[bb] + g.T[3 * aa + 1] * Sg[3 + bb] + g.T[3 * aa + 2] * Sg[6 + bb];
            const float hgb = 0.5f * gb;
            float gT[6];
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                gT[bb] = 2.f * (ga * V[bb] + hgb * V[3 + bb]);
                gT[3 + bb] = 2.f * (hgb * V[bb] + gcc * V[3 + bb]);
            }
            // G_Sigma (full, symmetric) = T^T Gc T
            {
                const float *T0 = g.T, *T1 = g.T + 3;
                const int ks[6] = {0, 0, 0, 1, 1, 2}, ls[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    const int k = ks[e], l = ls[e];
                    G6[e] += ga * T0[k] * T0[l] + hgb * (T0[k] * T1[l] + T1[k] * T0[l]) + gcc * T1[k] * T1[l];
                }
            }
            // T = J W
            const float gJ00 = gT[0] * cam.R[0] + gT[1] * cam.R[1] + gT[2] * cam.R[2];
            const float gJ02 = gT[0] * cam.R[6] + gT[1] * cam.R[7] + gT[2] * cam.R[8];
            const float gJ11 = gT[3] * cam.R[3] + gT[4] * cam.R[4] + gT[5] * cam.R[5];
            const float gJ12 = gT[3] * cam.R[6] + gT[4] * cam.R[7] + gT[5] * cam.R[8];
            g_tc[2] += -gJ00 * g.J00 * itz - gJ11 * g.J11 * itz;
            if (g.clamp_x == 0) {
                g_tc[0] += gJ02 * (-cam.fx * itz * itz);
                g_tc[2] += gJ02 * (-2.f * g.J02 * itz);
            } else {
                g_tc[2] += gJ02 * (-g.J02 * itz);
            }
            if (g.clamp_y == 0) {
                g_tc[1] += gJ12 * (-cam.fy * itz * itz);
                g_tc[2] += gJ12 * (-2.f * g.J12 * itz);
            } else {
                g_tc[2] += gJ12 * (-g.J12 * itz);
            }
            // mean' = (fx tx / tz + cx, fy ty / tz + cy)
            g_tc[0] += gs[0] * cam.fx * itz;
            g_tc[1] += gs[1] * cam.fy * itz;
            g_tc[2] += -(gs[0] * cam.fx * g.tc[0] + gs[1] * cam.fy * g.tc[1]) * itz * itz;
            // tc = R mu + t
#pragma unroll
            for (int k = 0; k < 3; ++k)
                g_mu[k] += cam.R[k] * g_tc[0] + cam.R[3 + k] * g_tc[1] + cam.R[6 + k] * g_tc[2];
        }

        // Sigma = M M^T, M = Rq diag(s):  dL/dM = 2 G M
        const float Gf[9] = {G6[0], G6[1], G6[2], G6[1], G6[3], G6[4], G6[2], G6[4], G6[5]};
        float gRq[9], g_ls[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float gsj = 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                float gm = 0.f;
#pragma unroll
                for (int k = 0; k < 3; ++k) gm += Gf[3 * i + k] * Rq[3 * k + j] * s[j];
                gm *= 2.f;
                gsj += gm * Rq[3 * i + j];
                gRq[3 * i + j] = gm * s[j];
            }
            g_ls[j] = gsj * s[j];
        }
        const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
        float gq[4];
        gq[0] = -2.f * z * gRq[1] + 2.f * y * gRq[2] + 2.f * z * gRq[3] - 2.f * x * gRq[5] - 2.f * y * gRq[6] +
                2.f * x * gRq[7];
        gq[1] = 2.f * y * gRq[1] + 2.f * z * gRq[2] + 2.f * y * gRq[3] - 4.f * x * gRq[4] - 2.f * w * gRq[5] +
                2.f * z * gRq[6] + 2.f * w * gRq[7] - 4.f * x * gRq[8];
        gq[2] = -4.f * y * gRq[0] + 2.f * x * gRq[1] + 2.f * w * gRq[2] + 2.f * x * gRq[3] + 2.f * z * gRq[5] -
                2.f * w * gRq[6] + 2.f * z * gRq[7] - 4.f * y * gRq[8];
        gq[3] = -4.f * z * gRq[0] - 2.f * w * gRq[1] + 2.f * x * gRq[2] + 2.f * w * gRq[3] - 4.f * z * gRq[4] +
                2.f * y * gRq[5] + 2.f * x * gRq[6] + 2.f * y * gRq[7];
        const float dq = gq[0] * qn[0] + gq[1] * qn[1] + gq[2] * qn[2] + gq[3] * qn[3];
        float g_q[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) g_q[k] = (gq[k] - qn[k] * dq) * qi;
        // lo = log2(sigmoid(logit)): dlo/dlogit = (1 - o) / ln 2
        const float g_logit = g_lo * (1.f - o) / kLn2;

        const int64_t st = a.g.stride;
        float n2[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a.g.mean[k * st + t] = g_mu[k];
            a.g.log_scale[k * st + t] = g_ls[k];
            n2[0] += g_mu[k] * g_mu[k];
            n2[1] += g_ls[k] * g_ls[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a.g.quat[k * st + t] = g_q[k];
            n2[2] += g_q[k] * g_q[k];
        }
        a.g.logit[t] = g_logit;
        n2[3] = g_logit * g_logit;
#pragma unroll
        for (int k = 0; k < 48; ++k) {
            a.g.sh[k * st + t] = g_sh[k];
            n2[4] += g_sh[k] * g_sh[k];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            a.g.vsh[k * st + t] = g_vsh[k];
            n2[5] += g_vsh[k] * g_vsh[k];
        }
        if (a.score) {
            float sc = 0.f;
#pragma unroll
            for (int k = 0; k < 6; ++k) sc = fmaxf(sc, sqrtf(n2[k]) / a.eps[k]);
            a.score[id] = sc;
        }
    }
    block_add_double(gsig, a.grad_sigma);
}

void launch_preprocess_bwd(const SplatPtrs &sp, const float *sigma, const RowList &rl, const Buffers &b,
                           const GradPtrs &g, double *grad_sigma, float *score, const float eps[6],
                           hipStream_t s)
{
    PreBwdArgs a;
    a.sp = sp;
    a.sigma = sigma;
    a.rl = rl;
    a.b = b;
    a.g = g;
    a.grad_sigma = grad_sigma;
    a.score = score;
    for (int k = 0; k < 6; ++k) a.eps[k] = eps[k];
    const unsigned blocks = (unsigned)((rl.Acap + 255) / 256);
    if (blocks) hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks), dim3(256), 0, s, a);
}

}  // namespace oit
