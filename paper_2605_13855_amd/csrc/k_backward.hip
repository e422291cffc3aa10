// Backward pass: L1 loss gradient, per-pixel constants of the OIT partials, the
// per-splat raster backward and the chain rule to the splat parameters and sigma
// (App. B, Eqs. "oit_rendering_md" and "oit_rendering_detail").
#include <hip/hip_ext.h>

#include "oit_internal.h"

namespace oit {

// The block's sum of v, on thread 0 (fixed order: lanes by a butterfly, waves in turn).
__device__ __forceinline__ double block_sum_double(double v)
{
    __shared__ double s_sum[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s_sum[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) t += s_sum[w];
    }
    return t;
}

// A sum of per-block shares (dL/dsigma: those of the pixel constants' pass, the inactive
// set, then those of the preprocess backward; the L1 loss: those of its pass), added in a
// fixed order by one block (each thread a fixed strided subset, then a tree in LDS), so
// that the result does not depend on the order in which the blocks that wrote them
// finished.
constexpr int kSumThreads = 1024;

__global__ __launch_bounds__(kSumThreads) void k_sum_shares(const double *a, int na, const double *b, int nb,
                                                            double *dst)
{
    __shared__ double s_t[kSumThreads];
    double t = 0.0;
    for (int i = threadIdx.x; i < na; i += kSumThreads) t += a[i];
    for (int i = threadIdx.x; i < nb; i += kSumThreads) t += b[i];
    s_t[threadIdx.x] = t;
    __syncthreads();
    for (int o = kSumThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s_t[threadIdx.x] += s_t[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dst = s_t[0];
}

// The pixels gp = tid, tid + stride, ... of the batch, as a flat grid-stride loop visits
// them and in the same order, but taken view by view so that the view's pixel base and
// size are wave-uniform: f(pix_base, HW, local) with gp = pix_base + local.  The views'
// pixels are contiguous and their total fits an int (the plan checks 9 x pixels).
template <class F>
__device__ __forceinline__ void for_batch_pixels(const Buffers &b, F &&f)
{
    const int stride = (int)(gridDim.x * blockDim.x);
    const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    for (int v = 0; v < b.n_views; ++v) {
        const int pb = b.cams[v].pix_base;
        const int hw = b.cams[v].W * b.cams[v].H;
        int local = tid - pb;
        if (local < 0) local += ((stride - 1 - local) / stride) * stride;
        for (; local < hw; local += stride) f((size_t)pb, (size_t)hw, (size_t)local);
    }
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

// Grid of the per-pixel kernels: a grid-stride loop over the batch's pixels with at most
// kPixBlocks blocks, so that the one FP64 atomic per block onto a single address stays
// a few thousand operations instead of one per 256 pixels.
constexpr int64_t kPixBlocks = kSigPixParts;

static unsigned pixel_blocks(int64_t total_px)
{
    const int64_t b = (total_px + 255) / 256;
    return (unsigned)(b < kPixBlocks ? b : kPixBlocks);
}

__global__ __launch_bounds__(256) void k_l1_loss(LossArgs a)
{
    double acc = 0.0;
    const float *__restrict__ image = a.image;
    const float *__restrict__ target = a.target;
    float *__restrict__ grad = a.grad;
    for_batch_pixels(a.b, [&](size_t pb, size_t HW, size_t local) {
        const size_t base = 3 * pb + local;
        const float inv = 1.f / (3.f * (float)HW);
        const double dinv = 1.0 / (3.0 * (double)HW);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = image[base + ch * HW] - target[base + ch * HW];
            grad[base + ch * HW] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
            acc += fabs((double)d) * dinv;
        }
    });
    const double t = block_sum_double(acc);
    if (threadIdx.x == 0) a.b.loss_part[blockIdx.x] = t;
}

void launch_sum_shares(const double *parts, int n, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_shares, dim3(1), dim3(kSumThreads), 0, s, parts, n, (const double *)nullptr, 0, dst);
}

void launch_l1_loss(const Buffers &b, const float *image, const float *target, float *grad, double *loss,
                    hipStream_t s)
{
    LossArgs a{b, image, target, grad, loss};
    const unsigned blocks = pixel_blocks(b.total_px);
    if (blocks) hipLaunchKernelGGL(k_l1_loss, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sum_shares, dim3(1), dim3(kSumThreads), 0, s, (const double *)b.loss_part, (int)blocks,
                       (const double *)nullptr, 0, loss);
}

// ---------------------------------------------------------------------------------
// per-pixel constants of the partials:
//   A_ch = g_ch (1 - T) / Q   (0 if Q <= 0),  s1 = sum_ch A_ch F_ch,
//   B    = T sum_ch g_ch (F_ch - c0_ch),  lambda = (dQ/dsigma) / Q  (0 if Q <= 0)
// so that for a contributing pair  dL/dc = A alpha w,  dL/dw = alpha (A.c - s1),
//   dL/dalpha = B / (1 - alpha) + w (A.c - s1).
//
// dL/dsigma.  F is the alpha w weighted mean of the colours, so at every pixel
// sum_i alpha_i w_i (c_i - F) = 0 exactly.  Hence
//   dL/dsigma = sum_p sum_i A . (c_i - F) alpha_i (dw_i/dsigma - lambda_p w_i)
// for any per-pixel lambda_p, and lambda_p = (dQ/dsigma) / Q (dQ/dsigma = sum_i alpha_i
// dw_i/dsigma) makes the sum insensitive, to first order, to an error in F: an error
// dF moves it by -A.dF sum_i alpha_i (dw_i/dsigma - lambda_p w_i) = 0.  Without the
// lambda term the float32 rounding of the forward's sums P and Q over ~10^3 splats
// per pixel enters dL/dsigma amplified by its cancellation (Sec. 1 Eq. "sf_weight";
// App. B, the dC/dw term).  Each splat therefore also sums lambda alpha (A.c - s1).
// The inactive set's share, sum_ch A_ch [(P1_ch - F_ch Q1) / sigma^2
//   - lambda (P0_ch - P1_ch / sigma - F_ch (Q0 - Q1 / sigma))]
//   = sum_ch A_ch [u P1'_ch - lambda P0'_ch + (1/2 - F_ch) (u Q1 - lambda Q0)],
// u = 1 / sigma^2 + lambda / sigma, is summed here from the pre-rendered accumulators,
// whose colour sums P0', P1' are stored centred on the colour offset 1/2.
// ---------------------------------------------------------------------------------
struct PixArgs {
    Buffers b;
    const float *sigma;
    float bg0, bg1, bg2;
    const float *pre, *grad, *pixstate;
    double *grad_sigma;
};

// PRE: a pre-rendered inactive set is given (its loads are issued with the others).
template <bool PRE>
__global__ __launch_bounds__(256) void k_pixconst(PixArgs a)
{
    double acc = 0.0;
    const float *__restrict__ pixstate = a.pixstate;
    const float *__restrict__ grad = a.grad;
    const float *__restrict__ pre = a.pre;
    float4 *__restrict__ pixconst = a.b.pixconst;
    float2 *__restrict__ pixB = a.b.pixB;
    const double sig = (double)*a.sigma, isig = 1.0 / sig, isig2 = isig * isig;
    for_batch_pixels(a.b, [&](size_t pb, size_t HW, size_t local) {
        const float *ps = pixstate + kPixStatePlanes * pb + local;
        const float *gr = grad + 3 * pb + local;
        const float T = ps[0], Q = ps[HW], Qs = ps[5 * HW];
        const float F[3] = {ps[2 * HW], ps[3 * HW], ps[4 * HW]};
        const float g[3] = {gr[0], gr[HW], gr[2 * HW]};
        float P0[3] = {0.f, 0.f, 0.f}, P1[3] = {0.f, 0.f, 0.f}, Q0 = 0.f, Q1 = 0.f;
        if constexpr (PRE) {
            const float *pr = pre + 9 * pb + local;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                P0[ch] = pr[ch * HW];
                P1[ch] = pr[(3 + ch) * HW];
            }
            Q0 = pr[6 * HW];
            Q1 = pr[7 * HW];
        }
        const float k = Q > 0.f ? (1.f - T) / Q : 0.f;
        const float lam = Q > 0.f ? Qs / Q : 0.f;
        const float A0 = g[0] * k, A1 = g[1] * k, A2 = g[2] * k;
        const float s1 = A0 * F[0] + A1 * F[1] + A2 * F[2];
        const float B = T * (g[0] * (F[0] - a.bg0) + g[1] * (F[1] - a.bg1) + g[2] * (F[2] - a.bg2));
        pixconst[pb + local] = make_float4(A0, A1, A2, -s1);
        pixB[pb + local] = make_float2(B, lam);
        if constexpr (PRE) {
            const double A[3] = {A0, A1, A2};
            const double ld = (double)lam, u = isig2 + ld * isig;
            const double qt = u * (double)Q1 - ld * (double)Q0;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                acc += A[ch] * (u * (double)P1[ch] - ld * (double)P0[ch] + ((double)kColorOffset - (double)F[ch]) * qt);
        }
    });
    const double t = block_sum_double(acc);
    if (threadIdx.x == 0) a.b.sig_part[blockIdx.x] = PRE ? t : 0.0;
}

void launch_pixconst(const Buffers &b, const float *sigma, const float bg[3], const float *pre,
                     const float *grad_image, const float *pixstate, double *grad_sigma, hipStream_t s)
{
    PixArgs a{b, sigma, bg[0], bg[1], bg[2], pre, grad_image, pixstate, grad_sigma};
    const unsigned blocks = pixel_blocks(b.total_px);
    if (!blocks) return;
    if (pre)
        hipLaunchKernelGGL(k_pixconst<true>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_pixconst<false>, dim3(blocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------------
// raster backward (the paper's per-splat backward, Sec. 4.2): one wave per work item
// = (tile, 64 active entries), one splat per lane.  The tile is cut into 8 x 8 pixel
// groups and a group that no lane's footprint box reaches is skipped.  The reached
// groups are taken four at a time: the wave stages their pixels' constants in its LDS
// slice, lists the (splat, group) pairs of the four (a splat and a group its box
// reaches) and deals them 64 per round to its lanes, so that a lane walks a group only
// for a splat that reaches it (items whose boxes are all small walk each lane's own box
// instead, and items whose splats nearly all reach all their groups are walked group by
// group by the whole wave).  Per splat, the colour and weight sums and the moments of dL/de over the
// pixel offsets end in the splat's own lane; they give the 10 screen-space partials
// once per work item, stored with plain stores in the entry's own row at its unsorted
// slot (no atomics: a (record, view) pair's slots are contiguous, and the preprocess
// backward sums them in a fixed order).
//
// Work items go to the XCDs in blocks of consecutive items (block b to XCD b mod 8), so
// that each XCD gets a mix of the batch and the waves working on one tile share an L2;
// a block holds about ten tiles' items (64 items when tiles have few, up to 1024).  The waves of an XCD take its items in order from the XCD's own queue, one device
// ticket per item; a wave stops when its queue is drained.  Same-address device atomics
// serialise at the memory side, so no wave polls the other XCDs' queues.
//
// Screen-space gradient layout (10 floats): d/dmx, d/dmy, d/dqa, d/dqb, d/dqc, d/dlo,
// d/dc (rgb), d/dw, and sum lambda alpha (A.c - s1) for dL/dsigma -- q* and lo as in
// the record.
// ---------------------------------------------------------------------------------
struct BwdArgs {
    Buffers b;
};

constexpr int kGroup = 8;   // pixel group edge of the backward

// tile of every backward work item (a chunk of 64 active entries of one tile)
__global__ __launch_bounds__(256) void k_chunk_map(Buffers b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.T) return;
    const uint32_t c1 = min(b.chunk_off[t + 1], b.max_chunks);
    for (uint32_t c = b.chunk_off[t]; c < c1; ++c) b.chunk_tile[c] = (uint32_t)t;
}

// Per-lane sums of the backward over the pixels of its tile entry.  g_c* hold
// sum A_ch alpha; dL/dc_ch = w times that (w is the lane's), taken once at the end.
// g_w = dL/dw; g_h = the same sum weighted by the pixel's lambda (for dL/dsigma).
struct BwdSums {
    float g_cr, g_cg, g_cb, g_w, g_h;
    // moments of dL/de (without the ln 2 of d alpha / de) over the pixel offsets
    float m0, m_x, m_y, m_xx, m_xy, m_yy;
};

// One staged 8 x 8 group for one lane's splat, column by column.  CAP: some splat of
// the work item may reach the opacity cap, so alpha is clamped to 0.99 and its
// derivative cut where it is; otherwise every alpha stays below 0.99 (the splats'
// opacities are below it with a margin) and neither step is needed.
template <bool CAP>
__device__ __forceinline__ void bwd_group(const float4 *pcs, const float2 *pBs, int gxp, int gyp, float dx0, float dy0,
                                          float qa, float qb, float qc, float lo, float cr, float cg, float cb,
                                          float w, BwdSums &o)
{
    float dy[kGroup];
#pragma unroll
    for (int r = 0; r < kGroup; ++r) dy[r] = dy0 + (float)(gyp + r);
    // the column's moments over dy = yb + r are taken from sums over the row index r
    // (c0 = sum dL/de, c1 = sum r dL/de, c2 = sum r^2 dL/de: r and r^2 are constants of
    // the unrolled rows) and shifted by yb once per column
    const float yb = dy0 + (float)gyp;
    // columns stay a loop: unrolled, the per-column moment updates are deferred and
    // every column's partial sums stay live
#pragma unroll 1
    for (int c = 0; c < kGroup; ++c) {
        const float dx = dx0 + (float)(gxp + c);
        const float kb = exp_col_b(qb, dx), kc = exp_col_c(qa, lo, dx);
        float c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
            const float e = exp_pix(qc, dy[r], kb, kc);
            if (e >= kLog2AlphaMin) {
                const float4 pc = pcs[r * kGroup + c];
                const float2 Bl = pBs[r * kGroup + c];
                const float ex = __builtin_amdgcn_exp2f(e);
                const float al = CAP ? fminf(ex, kAlphaMax) : ex;
                // A . c - s1 (pc.w holds -s1)
                const float diff = fmaf(pc.x, cr, fmaf(pc.y, cg, fmaf(pc.z, cb, pc.w)));
                o.g_cr = fmaf(pc.x, al, o.g_cr);
                o.g_cg = fmaf(pc.y, al, o.g_cg);
                o.g_cb = fmaf(pc.z, al, o.g_cb);
                const float ad = al * diff;
                o.g_w += ad;
                o.g_h = fmaf(ad, Bl.y, o.g_h);
                // dL/de / ln 2 = alpha (B / (1 - alpha) + w diff); zero where alpha is capped
                const float dLda = fmaf(w, diff, Bl.x * __builtin_amdgcn_rcpf(1.f - al));
                const float dLde = (CAP ? (al < kAlphaMax ? al : 0.f) : al) * dLda;
                c0 += dLde;
                if (r > 0) {
                    c1 = fmaf(dLde, (float)r, c1);
                    c2 = fmaf(dLde, (float)(r * r), c2);
                }
            }
        }
        // sum dL/de dy = yb c0 + c1, sum dL/de dy^2 = yb^2 c0 + 2 yb c1 + c2
        const float cy = fmaf(yb, c0, c1);
        const float cyy = fmaf(yb, cy + c1, c2);
        o.m0 += c0;
        o.m_x = fmaf(dx, c0, o.m_x);
        o.m_xx = fmaf(dx * dx, c0, o.m_xx);
        o.m_y += cy;
        o.m_xy = fmaf(dx, cy, o.m_xy);
        o.m_yy += cyy;
    }
}

// Box mode is taken when the largest footprint box is at most kBoxPerGroup pixels per
// reached group.  A box pixel costs several group pixel slots (its own exponent terms, a
// memory read of the constants, the full moments); with the groups' pairs dealt to the
// lanes a group costs only the lanes that reach it, and a sweep at configs 4 and 5 and
// the sub-pixel scene put the best threshold near 5 (it was 21 for the walk of every
// reached group by the whole wave).
constexpr int kBoxPerGroup = 5;

// Groups of a pair window: their pixel constants are staged together in a wave's slice,
// kSlot entries apart (one more than a group's 64 pixels), so that lanes reading the
// same pixel of different groups hit different LDS banks.
constexpr int kWin = 4;
constexpr int kSlot = 65;

// The entry's 10 screen-space partials from the lane's sums:
// de/dlo = 1, de/dqa = dx^2, de/dqb = dx dy, de/dqc = dy^2,
// de/dmx = -(2 qa dx + qb dy), de/dmy = -(qb dx + 2 qc dy); the ln 2 of d alpha / de.
__device__ __forceinline__ void write_partials(float *dst, float qa, float qb, float qc, float w, const BwdSums &o)
{
    ((float4 *)dst)[0] = make_float4(-(2.f * qa * o.m_x + qb * o.m_y) * kLn2, -(qb * o.m_x + 2.f * qc * o.m_y) * kLn2,
                                     o.m_xx * kLn2, o.m_xy * kLn2);
    ((float4 *)dst)[1] = make_float4(o.m_yy * kLn2, o.m0 * kLn2, w * o.g_cr, w * o.g_cg);
    ((float4 *)dst)[2] = make_float4(w * o.g_cb, o.g_w, o.g_h, 0.f);
}

template <int S>
// walks: the wave's counts of items walked box by box (low 16 bits) and group by group by
// the whole wave (high 16 bits), for the counters
__device__ __forceinline__ void bwd_item(const Buffers &b, uint32_t item, int wave, int lane,
                                         float4 (*s_c)[kWin * kSlot], float2 (*s_B)[kWin * kSlot],
                                         uint8_t (*s_pair)[kWin * 64], uint32_t &walks)
{
    constexpr int GX = S / kGroup;   // groups per tile edge
    const uint64_t cap = (uint64_t)b.pair_cap;
    const int tile = (int)b.chunk_tile[item];
    const uint32_t chunk = item - b.chunk_off[tile];
    const int v = view_of_tile(b.cams, b.n_views, tile);
    const CamDev &cam = b.cams[v];
    const int lt = tile - cam.tile_base;
    const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
    const float x0 = (float)(tx * S) + 0.5f, y0 = (float)(ty * S) + 0.5f;
    const uint64_t off = b.tile_off[tile];
    uint64_t na = b.cnt_a[tile];
    if (off + na > cap) na = off < cap ? cap - off : 0;
    const uint64_t j = (uint64_t)chunk * 64 + lane;
    const uint32_t rj = j < na ? b.entries[off + j] : 0u;
    const bool valid = j < na && rj < b.Acap;
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = make_float4(0.f, -1e30f, 0.f, 0.f),
           rc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
        const Rec rr = b.rec[(size_t)v * b.Rcap + rj];
        ra = rr.a;
        rb = rr.b;
        rc = rr.c;
    }
    const float dx0 = x0 - ra.x, dy0 = y0 - ra.y;
    const float qa = ra.z, qb = ra.w, qc = rb.x, lo = rb.y;
    const float cr = rb.z, cg = rb.w, cb = rc.x, w = rc.y;

    // footprint half-extents of the (widened) alpha >= 1/255 level set, in pixels
    float hx = -1.f, hy = -1.f;
    if (valid) {
        const float A = -qa, B = -0.5f * qb, C = -qc;
        const float det = A * C - B * B;
        const float tau = (lo - kLog2AlphaMin) * 1.001f + 1e-3f;
        if (tau > 0.f && det > 0.f) {
            hx = sqrtf(tau * C / det) + 0.01f;
            hy = sqrtf(tau * A / det) + 0.01f;
        }
    }
    // this entry's row of screen-space partials, at its unsorted slot (written for every
    // valid lane)
    float *dst = b.ep + (size_t)(valid ? b.orig[off + j] : 0u) * kEpStride;
    // bit g of mask: some lane's footprint box reaches group g (pixel offsets [g0, g0 + 7]);
    // bit g of my: this lane's box does
    uint32_t mask = 0, my = 0;
#pragma unroll
    for (int g = 0; g < GX * GX; ++g) {
        const float gx0 = dx0 + (float)((g % GX) * kGroup), gy0 = dy0 + (float)((g / GX) * kGroup);
        const bool hit = hx >= 0.f && gx0 <= hx && gx0 + (float)(kGroup - 1) >= -hx && gy0 <= hy &&
                         gy0 + (float)(kGroup - 1) >= -hy;
        if (hit) my |= 1u << g;
        if (__ballot(hit)) mask |= 1u << g;
    }
    if (mask == 0) {
        if (valid) {
            ((float4 *)dst)[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            ((float4 *)dst)[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            ((float4 *)dst)[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return;
    }

    const size_t pb = (size_t)cam.pix_base;
    const bool may_cap = __ballot(valid && lo > kLog2NoCap) != 0;

    // Small footprints (typical of sub-pixel splats): each lane walks its own box,
    // reading the pixel constants it needs from memory, instead of the whole wave
    // walking every reached group.  The box holds every pixel whose exponent can pass
    // the threshold (same widened extents).
    {
        int bc0 = 0, bc1 = -1, br0 = 0, br1 = -1;   // tile-local columns / rows of the box
        if (hx >= 0.f) {
            const float lim = 1e6f;
            bc0 = max(0, (int)ceilf(fmaxf(-hx - dx0, -lim)));
            bc1 = min(min(S, cam.W - tx * S) - 1, (int)floorf(fminf(hx - dx0, lim)));
            br0 = max(0, (int)ceilf(fmaxf(-hy - dy0, -lim)));
            br1 = min(min(S, cam.H - ty * S) - 1, (int)floorf(fminf(hy - dy0, lim)));
        }
        const int area = (bc1 >= bc0 && br1 >= br0) ? (bc1 - bc0 + 1) * (br1 - br0 + 1) : 0;
        int amax = area;
        for (int m = 32; m > 0; m >>= 1) amax = max(amax, __shfl_xor(amax, m));
        if (amax <= kBoxPerGroup * __builtin_popcount(mask)) {
            ++walks;
            BwdSums o = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            int c = bc0, r = br0;
            // the constants of the lane's next box pixel are fetched one pixel ahead
            const size_t row0 = pb + (size_t)(ty * S) * cam.W + (size_t)(tx * S);
            float4 npc = make_float4(0.f, 0.f, 0.f, 0.f);
            float2 nBc = make_float2(0.f, 0.f);
            if (area > 0) {
                npc = b.pixconst[row0 + (size_t)r * cam.W + c];
                nBc = b.pixB[row0 + (size_t)r * cam.W + c];
            }
            for (int k = 0; k < amax; ++k) {
                if (k < area) {
                    const float4 pc = npc;
                    const float2 Bl = nBc;
                    const float dx = dx0 + (float)c, dy = dy0 + (float)r;
                    if (++c > bc1) {
                        c = bc0;
                        ++r;
                    }
                    if (k + 1 < area) {
                        npc = b.pixconst[row0 + (size_t)r * cam.W + c];
                        nBc = b.pixB[row0 + (size_t)r * cam.W + c];
                    }
                    const float e = exp_pix(qc, dy, exp_col_b(qb, dx), exp_col_c(qa, lo, dx));
                    if (e >= kLog2AlphaMin) {
                        const float ex = __builtin_amdgcn_exp2f(e);
                        const float al = may_cap ? fminf(ex, kAlphaMax) : ex;
                        const float diff = fmaf(pc.x, cr, fmaf(pc.y, cg, fmaf(pc.z, cb, pc.w)));
                        o.g_cr = fmaf(pc.x, al, o.g_cr);
                        o.g_cg = fmaf(pc.y, al, o.g_cg);
                        o.g_cb = fmaf(pc.z, al, o.g_cb);
                        const float ad = al * diff;
                        o.g_w += ad;
                        o.g_h = fmaf(ad, Bl.y, o.g_h);
                        const float dLda = fmaf(w, diff, Bl.x * __builtin_amdgcn_rcpf(1.f - al));
                        const float dLde = (al < kAlphaMax ? al : 0.f) * dLda;
                        const float exx = dLde * dx, eyy = dLde * dy;
                        o.m0 += dLde;
                        o.m_x += exx;
                        o.m_y += eyy;
                        o.m_xx = fmaf(exx, dx, o.m_xx);
                        o.m_xy = fmaf(exx, dy, o.m_xy);
                        o.m_yy = fmaf(eyy, dy, o.m_yy);
                    }
                }
            }
            if (valid) write_partials(dst, qa, qb, qc, w, o);
            return;
        }
    }

    // this lane's pixel when staging a group's constants
    const int sx = lane % kGroup, sy = lane / kGroup;
    auto fetch = [&](int g, float4 &c, float2 &Bv) {
        const int x = tx * S + (g % GX) * kGroup + sx, y = ty * S + (g / GX) * kGroup + sy;
        c = make_float4(0.f, 0.f, 0.f, 0.f);
        Bv = make_float2(0.f, 0.f);
        if (x < cam.W && y < cam.H) {
            const size_t gp = pb + (size_t)y * cam.W + x;
            c = b.pixconst[gp];
            Bv = b.pixB[gp];
        }
    };

    BwdSums o = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float4 *const wc = s_c[wave];
    float2 *const wB = s_B[wave];
    uint8_t *const wp = s_pair[wave];

    // Where the dealt rounds would be nearly as many as the reached groups (most splats of
    // the item reach most of its groups), the whole wave walks every reached group with
    // a uniform LDS broadcast of each pixel's constants instead (the next group's are
    // fetched while the current one is walked): no shuffles, no window staging.
    int rounds = 0;
    {
        uint32_t r = mask;
        while (r) {
            int pw = 0;
            for (int k = 0; k < kWin && r; ++k) {
                const int g = __builtin_ctz(r);
                r &= r - 1;
                pw += (int)__builtin_popcountll(__ballot((my >> g) & 1u));
            }
            rounds += (pw + 63) >> 6;
        }
    }
    if (10 * rounds >= 9 * __builtin_popcount(mask)) {
        walks += 1u << 16;
        uint32_t rest = mask;
        int g = __builtin_ctz(rest);
        rest &= rest - 1;
        float4 nc;
        float2 nB;
        fetch(g, nc, nB);
        for (;;) {
            wc[lane] = nc;
            wB[lane] = nB;
            int gn = -1;
            if (rest) {
                gn = __builtin_ctz(rest);
                rest &= rest - 1;
                fetch(gn, nc, nB);
            }
            __builtin_amdgcn_wave_barrier();
            const int gxp = (g % GX) * kGroup, gyp = (g / GX) * kGroup;
            if (may_cap)
                bwd_group<true>(wc, wB, gxp, gyp, dx0, dy0, qa, qb, qc, lo, cr, cg, cb, w, o);
            else
                bwd_group<false>(wc, wB, gxp, gyp, dx0, dy0, qa, qb, qc, lo, cr, cg, cb, w, o);
            __builtin_amdgcn_wave_barrier();
            if (gn < 0) break;
            g = gn;
        }
        if (valid) write_partials(dst, qa, qb, qc, w, o);
        return;
    }

    // (splat, group) pairs dealt to the lanes.  The reached groups are taken kWin at a
    // time; the window's pixel constants are staged in the wave's LDS slice (slot k holds
    // the window's k-th group, one pixel per lane).  The window's pairs -- a lane's splat
    // and a group of the window that its box reaches -- are listed splat by splat and
    // dealt 64 per round, one per lane; each lane walks its pair's group for the pair's
    // splat, whose parameters it reads from the owning lane.  A splat's consecutive pairs
    // in a round (at most kWin) are then summed at the first of them and added into the
    // owning lane's sums.  Lanes thus walk pixels for splats that reach them, instead of
    // every lane walking every group that some lane reaches.
    uint32_t rest = mask;
    while (rest) {
        uint32_t wpack = 0;   // the window's groups, 4 bits each
        int nw = 0;
        while (rest && nw < kWin) {
            wpack |= (uint32_t)__builtin_ctz(rest) << (4 * nw);
            rest &= rest - 1;
            ++nw;
        }
        uint32_t slots = 0;   // window slots of this lane's pairs
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            if (k < nw) {
                const int g = (int)((wpack >> (4 * k)) & 15u);
                float4 c;
                float2 Bv;
                fetch(g, c, Bv);
                wc[k * kSlot + lane] = c;
                wB[k * kSlot + lane] = Bv;
                if ((my >> g) & 1u) slots |= 1u << k;
            }
        }
        // the lane's first pair in the window's list (exclusive prefix over the wave)
        const int cnt = __builtin_popcount(slots);
        int incl = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        const int pfx = incl - cnt;
        const int P = __builtin_amdgcn_readfirstlane(__shfl(incl, 63));   // pairs in the window
        {
            int q = pfx;
#pragma unroll
            for (int k = 0; k < kWin; ++k)
                if ((slots >> k) & 1u) wp[q++] = (uint8_t)((lane << 2) | k);
        }
        __builtin_amdgcn_wave_barrier();
        for (int base = 0; base < P; base += 64) {
            const int t = base + lane;
            const bool on = t < P;
            const int e = on ? (int)wp[t] : 0;
            const int owner = e >> 2, slot = e & 3;
            const int g = (int)((wpack >> (4 * slot)) & 15u);
            // the pair's splat (a lane past the last pair evaluates nothing: lo = -1e30).
            // Every lane takes part in every shuffle: a lane left out of one (a shuffle
            // under a branch) does not supply its value to the others.
            const float pdx0 = __shfl(dx0, owner), pdy0 = __shfl(dy0, owner);
            const float pqa = __shfl(qa, owner), pqb = __shfl(qb, owner), pqc = __shfl(qc, owner);
            const float slo = __shfl(lo, owner);
            const float plo = on ? slo : -1e30f;
            const float pcr = __shfl(cr, owner), pcg = __shfl(cg, owner), pcb = __shfl(cb, owner);
            const float pw = __shfl(w, owner);
            BwdSums p = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const int gxp = (g % GX) * kGroup, gyp = (g / GX) * kGroup;
            if (may_cap)
                bwd_group<true>(wc + slot * kSlot, wB + slot * kSlot, gxp, gyp, pdx0, pdy0, pqa, pqb, pqc, plo, pcr, pcg, pcb,
                                pw, p);
            else
                bwd_group<false>(wc + slot * kSlot, wB + slot * kSlot, gxp, gyp, pdx0, pdy0, pqa, pqb, pqc, plo, pcr, pcg, pcb,
                                 pw, p);
            // segments of at most kWin lanes with one owner: two steps sum each at its head
            const int own1 = __shfl_down(owner, 1), own2 = __shfl_down(owner, 2);
            const bool s1 = lane + 1 < 64 && t + 1 < P && own1 == owner;
            const bool s2 = lane + 2 < 64 && t + 2 < P && own2 == owner;
            // this lane as owner: its pairs in the round start at lane `head`
            const bool mine = cnt > 0 && pfx < base + 64 && pfx + cnt > base;
            const int head = (pfx > base ? pfx : base) - base;
            auto add = [&](float v, float &sum) {
                const float a1 = __shfl_down(v, 1);
                v += s1 ? a1 : 0.f;
                const float a2 = __shfl_down(v, 2);
                v += s2 ? a2 : 0.f;
                const float h = __shfl(v, head);
                if (mine) sum += h;
            };
            add(p.g_cr, o.g_cr);
            add(p.g_cg, o.g_cg);
            add(p.g_cb, o.g_cb);
            add(p.g_w, o.g_w);
            add(p.g_h, o.g_h);
            add(p.m0, o.m0);
            add(p.m_x, o.m_x);
            add(p.m_y, o.m_y);
            add(p.m_xx, o.m_xx);
            add(p.m_xy, o.m_xy);
            add(p.m_yy, o.m_yy);
        }
        // the window's slices are rewritten by the next window
        __builtin_amdgcn_wave_barrier();
    }
    if (valid) write_partials(dst, qa, qb, qc, w, o);
}

// Five waves per SIMD: 96 registers, with 48 bytes per lane of scratch used per item, per
// window and per group of the whole-wave walk, none inside the rounds or the columns.
// At config 4 (5% active) four waves keep everything in registers and ran 4% slower;
// six waves spilled 92 bytes per lane inside the walks and ran 15% slower.
template <int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_raster_bwd(BwdArgs a)
{
    __shared__ float4 s_c[4][kWin * kSlot];
    __shared__ float2 s_B[4][kWin * kSlot];
    __shared__ uint8_t s_pair[4][kWin * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t total = a.b.counters[CNT_TOTAL_CHUNKS];
    if (total > a.b.max_chunks) total = a.b.max_chunks;
    const int xcd = (int)(blockIdx.x % kXcds);
    // block size: 64 items per six items of the average tile, a power of two up to 1024
    const uint32_t per_tile = total / (uint32_t)(a.b.T > 0 ? a.b.T : 1);
    const uint32_t want = 64u * ((per_tile + 5u) / 6u);
    int lb = 6;
    while ((1u << lb) < want && lb < 10) ++lb;
    uint32_t walks = 0;   // a wave takes far fewer than 2^16 items
    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(&a.b.counters[CNT_XQUEUE + xcd], 1u);
        ticket = __builtin_amdgcn_readfirstlane(ticket);
        // the ticket-th item of this XCD: block xcd + 8 (ticket / B), offset ticket % B
        const uint64_t item = (((uint64_t)xcd + (uint64_t)kXcds * (ticket >> lb)) << lb) + (ticket & ((1u << lb) - 1u));
        if (item >= total) break;   // items grow with the ticket: the queue is drained
        bwd_item<S>(a.b, (uint32_t)item, wave, lane, s_c, s_B, s_pair, walks);
    }
    // one atomic per block for each walk counter
    __shared__ uint32_t s_walks[4];
    if (lane == 0) s_walks[wave] = walks;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t nb = 0, nw = 0;
        for (int k = 0; k < 4; ++k) {
            nb += s_walks[k] & 0xffffu;
            nw += s_walks[k] >> 16;
        }
        if (nb) atomicAdd(&a.b.counters[CNT_BOX_ITEMS], nb);
        if (nw) atomicAdd(&a.b.counters[CNT_WAVE_ITEMS], nw);
    }
}

// ---------------------------------------------------------------------------------
// raster backward, per-pixel form (the 3DGS baseline of the paper's ablation): one
// thread per pixel walks its tile's active entries (staged through LDS like the
// forward) and adds the 10 screen-space partials of every contributing pair to the
// entry's row with one atomic each.  Same partials as k_raster_bwd; kept for
// comparison.
// ---------------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(S * S < 256 ? S * S : 256) void k_raster_bwd_pixel(BwdArgs a)
{
    constexpr int NT = S * S < 256 ? S * S : 256;
    constexpr int PPT = S * S / NT;
    constexpr int RSTEP = NT / S;
    constexpr int B = 64;
    __shared__ float4 s_rec[B * 3];
    __shared__ uint32_t s_r[B];
    const int tile = blockIdx.x;
    const int v = view_of_tile(a.b.cams, a.b.n_views, tile);
    const CamDev &cam = a.b.cams[v];
    const int lt = tile - cam.tile_base;
    const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
    const float x0 = (float)(tx * S) + 0.5f, y0 = (float)(ty * S) + 0.5f;
    const int col = threadIdx.x % S, row0 = threadIdx.x / S;
    const float colf = (float)col;
    float rowf[PPT], A0[PPT], A1[PPT], A2[PPT], ns1[PPT], Bc[PPT], Lc[PPT];
    bool in[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int x = tx * S + col, y = ty * S + row0 + p * RSTEP;
        rowf[p] = (float)(row0 + p * RSTEP);
        in[p] = x < cam.W && y < cam.H;
        float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 cB = make_float2(0.f, 0.f);
        if (in[p]) {
            const size_t gp = (size_t)cam.pix_base + (size_t)y * cam.W + x;
            c0 = a.b.pixconst[gp];
            cB = a.b.pixB[gp];
        }
        A0[p] = c0.x;
        A1[p] = c0.y;
        A2[p] = c0.z;
        ns1[p] = c0.w;
        Bc[p] = cB.x;
        Lc[p] = cB.y;
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
            s_rec[3 * j] = make_float4(x0 - r.a.x, y0 - r.a.y, r.a.z, r.a.w);
            s_rec[3 * j + 1] = r.b;
            s_rec[3 * j + 2] = r.c;
            s_r[j] = ok ? 1u : 0u;
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const float4 ra = s_rec[3 * j], rb = s_rec[3 * j + 1], rc = s_rec[3 * j + 2];
            if (!s_r[j]) continue;
            // the entry's row at its unsorted slot, zeroed when the list was written
            float *dst = a.b.ep + (size_t)a.b.orig[off + base + j] * kEpStride;
            const float dx = ra.x + colf;
            const float kb = exp_col_b(ra.w, dx), kc = exp_col_c(ra.z, rb.y, dx);
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                if (!in[p]) continue;
                const float dy = ra.y + rowf[p];
                const float e = exp_pix(rb.x, dy, kb, kc);
                if (e < kLog2AlphaMin) continue;
                const float al = fminf(__builtin_amdgcn_exp2f(e), kAlphaMax);
                const float w = rc.y;
                const float diff = fmaf(A0[p], rb.z, fmaf(A1[p], rb.w, fmaf(A2[p], rc.x, ns1[p])));
                const float aw = al * w;
                unsafeAtomicAdd(dst + 6, A0[p] * aw);
                unsafeAtomicAdd(dst + 7, A1[p] * aw);
                unsafeAtomicAdd(dst + 8, A2[p] * aw);
                unsafeAtomicAdd(dst + 9, al * diff);
                unsafeAtomicAdd(dst + 10, Lc[p] * (al * diff));
                if (al < kAlphaMax) {
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

// Persistent grid of the per-splat backward: 8 workgroups of 4 waves per CU of the
// largest device (256 CUs); a multiple of the 8 XCDs, so that every XCD's queue is served.
constexpr unsigned kBwdBlocks = 2048;
static_assert(kBwdBlocks % kXcds == 0, "every XCD queue needs workgroups");

template <int S>
static void launch_bwd_pixel_s(const BwdArgs &a, dim3 block, hipStream_t s, const KTimer *t)
{
    const dim3 grid((unsigned)a.b.T);
    if (t)
        hipExtLaunchKernelGGL(k_raster_bwd_pixel<S>, grid, block, 0, s, t->start, t->stop, 0, a);
    else
        hipLaunchKernelGGL(k_raster_bwd_pixel<S>, grid, block, 0, s, a);
}

template <int S>
static void launch_bwd_s(const BwdArgs &a, hipStream_t s, const KTimer *t)
{
    const dim3 grid(kBwdBlocks), block(256);
    if (t)
        hipExtLaunchKernelGGL(k_raster_bwd<S>, grid, block, 0, s, t->start, t->stop, 0, a);
    else
        hipLaunchKernelGGL(k_raster_bwd<S>, grid, block, 0, s, a);
}

bool launch_raster_bwd(const Buffers &b, const RowList &rl, hipStream_t s, const KTimer *t)
{
    (void)rl;
    BwdArgs a{b};
    if (b.T == 0) return true;
    if (b.bwd_mode == OIT_BWD_PER_PIXEL) {
        switch (b.tile) {
        case 8: launch_bwd_pixel_s<8>(a, dim3(64), s, t); return true;
        case 16: launch_bwd_pixel_s<16>(a, dim3(256), s, t); return true;
        case 32: launch_bwd_pixel_s<32>(a, dim3(256), s, t); return true;
        default: return false;
        }
    }
    hipLaunchKernelGGL(k_chunk_map, dim3((unsigned)((b.T + 255) / 256)), dim3(256), 0, s, b);
    switch (b.tile) {
    case 8: launch_bwd_s<8>(a, s, t); return true;
    case 16: launch_bwd_s<16>(a, s, t); return true;
    case 32: launch_bwd_s<32>(a, s, t); return true;
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
    int vlanes;   // lanes per row: the view count rounded up to a power of two (<= 64)
};

// Per-view share of one active row's parameter gradient: everything the views sum.
struct ViewPart {
    float g_mu[3];   // mean (geometry and the viewing direction)
    float G6[6];     // 3D covariance (upper triangle of the symmetric gradient)
    float g_lo;      // log2 opacity
    float gcm[3];    // colour gradient where the channel is not clamped
    float gvm;       // view-weight gradient where v(r) is not clamped and d < sigma
    float Y[16];     // SH basis at the viewing direction
    double gsig;     // sigma
};

// Chain rule of one view, from the record's 10 screen-space partials to the splat's
// parameters (Sec. 3.1 model; the inverse of the forward projection step by step).
__device__ void view_partials(const PreBwdArgs &a, int64_t nrec, int64_t t, int64_t id, int v, const float mu[3],
                              const float S6[6], float sigma, ViewPart &o)
{
    const float *sh = a.sp.sh + 48 * id;    // [16][3] of this splat
    const float *vsh = a.sp.vsh + 16 * id;
#pragma unroll
    for (int k = 0; k < 3; ++k) o.g_mu[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) o.G6[k] = 0.f;
    o.g_lo = 0.f;
    o.gcm[0] = o.gcm[1] = o.gcm[2] = 0.f;
    o.gvm = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) o.Y[k] = 0.f;
    o.gsig = 0.0;

    // screen-space partials of this (record, view): the sum of its tile entries' rows
    float gs[kEpUsed];
#pragma unroll
    for (int k = 0; k < kEpUsed; ++k) gs[k] = 0.f;
    {
        // the pair's entries hold the contiguous slots [hoff, hoff + nhits); active rows
        // are the first listed records, so the pair index is view * nrec + t
        const size_t pv = (size_t)v * nrec + t;
        const uint64_t cap = (uint64_t)a.b.pair_cap;
        const uint64_t g0 = a.b.hoff[pv], nh = a.b.nhits[pv];
        const uint64_t n = g0 >= cap ? 0 : (nh < cap - g0 ? nh : cap - g0);
        // rows four at a time: the loads are issued together, the sums stay in row order
        for (uint64_t k = 0; k < n; k += 4) {
            float4 e0[4], e1[4];
            float3 e2[4];   // the row's last three partials (the fourth float is padding)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (k + j < n) {
                    const float *e = a.b.ep + (g0 + k + j) * kEpStride;
                    e0[j] = ((const float4 *)e)[0];
                    e1[j] = ((const float4 *)e)[1];
                    e2[j] = make_float3(e[8], e[9], e[10]);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (k + j < n) {
                    gs[0] += e0[j].x;
                    gs[1] += e0[j].y;
                    gs[2] += e0[j].z;
                    gs[3] += e0[j].w;
                    gs[4] += e1[j].x;
                    gs[5] += e1[j].y;
                    gs[6] += e1[j].z;
                    gs[7] += e1[j].w;
                    gs[8] += e2[j].x;
                    gs[9] += e2[j].y;
                    gs[10] += e2[j].z;
                }
            }
        }
    }
    bool any = false;
#pragma unroll
    for (int k = 0; k < kEpUsed; ++k) any |= gs[k] != 0.f;
    if (!any) return;
    const CamDev &cam = a.b.cams[v];
    Geo g;
    if (!geometry(cam, mu, S6, g)) return;
    const float tz = g.tc[2], itz = 1.f / tz;
    float g_tc[3] = {0.f, 0.f, 0.f};
    o.g_lo = gs[5];

    // appearance: colour and view weight at the viewing direction
    float u[3] = {mu[0] - cam.cc[0], mu[1] - cam.cc[1], mu[2] - cam.cc[2]};
    const float dist = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const float idist = 1.f / dist;
    const float dir[3] = {u[0] * idist, u[1] * idist, u[2] * idist};
    sh_eval(dir[0], dir[1], dir[2], o.Y);
    float gY[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gY[k] = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float raw = kColorOffset;
#pragma unroll
        for (int k = 0; k < 16; ++k) raw += o.Y[k] * sh[3 * k + ch];
        if (raw > 0.f) {
            const float gc = gs[6 + ch];
            o.gcm[ch] = gc;
#pragma unroll
            for (int k = 0; k < 16; ++k) gY[k] = fmaf(gc, sh[3 * k + ch], gY[k]);
        }
    }
    {
        float raw = kColorOffset;
#pragma unroll
        for (int k = 0; k < 16; ++k) raw += o.Y[k] * vsh[k];
        const float vv = fmaxf(raw, 0.f);
        const float gw = gs[9];
        if (tz < sigma) {
            const float gv = gw * (1.f - tz / sigma);
            g_tc[2] += -gw * vv / sigma;
            // sum over the pixels of alpha (A.c - s1) (dw/dsigma - lambda w): dw/dsigma and
            // w in float, as the forward pass forms them; the difference in double
            const float dw = vv * tz / (sigma * sigma), wv = (1.f - tz / sigma) * vv;
            o.gsig = fma((double)gw, (double)dw, -(double)gs[10] * (double)wv);
            if (raw > 0.f) {
                o.gvm = gv;
#pragma unroll
                for (int k = 0; k < 16; ++k) gY[k] = fmaf(gv, vsh[k], gY[k]);
            }
        }
    }
    float gdir[3];
    sh_vjp(dir[0], dir[1], dir[2], gY, gdir);
    {
        const float dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) o.g_mu[k] += (gdir[k] - dir[k] * dd) * idist;
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
    float Vm[6];
#pragma unroll
    for (int aa = 0; aa < 2; ++aa)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
            Vm[3 * aa + bb] = g.T[3 * aa] * Sg[bb] + g.T[3 * aa + 1] * Sg[3 + bb] + g.T[3 * aa + 2] * Sg[6 + bb];
    const float hgb = 0.5f * gb;
    float gT[6];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
        gT[bb] = 2.f * (ga * Vm[bb] + hgb * Vm[3 + bb]);
        gT[3 + bb] = 2.f * (hgb * Vm[bb] + gcc * Vm[3 + bb]);
    }
    // G_Sigma (full, symmetric) = T^T Gc T
    {
        const float *T0 = g.T, *T1 = g.T + 3;
        const int ks[6] = {0, 0, 0, 1, 1, 2}, ls[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int k = ks[e], l = ls[e];
            o.G6[e] = ga * T0[k] * T0[l] + hgb * (T0[k] * T1[l] + T1[k] * T0[l]) + gcc * T1[k] * T1[l];
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
    for (int k = 0; k < 3; ++k) o.g_mu[k] += cam.R[k] * g_tc[0] + cam.R[3 + k] * g_tc[1] + cam.R[6 + k] * g_tc[2];
}

// ---------------------------------------------------------------------------------
// preprocess backward: a group of `vlanes` lanes per active row, one lane per view.
// Each lane forms its view's share of the parameter gradient (view_partials); the
// shares meet in LDS, where the row's lanes sum them: lane 0 finishes the geometric
// chain (covariance -> log-scales and quaternion, opacity), every lane a quarter of
// the 64 SH outputs.  Also the activeness score (Sec. 4.1) and dL/dsigma (FP64).
// ---------------------------------------------------------------------------------
constexpr int kPbThreads = 256;
constexpr unsigned kPbBlocks = kSigPreParts;

__global__ __launch_bounds__(kPbThreads) void k_preprocess_bwd(PreBwdArgs a)
{
    __shared__ float s_geo[kPbThreads][10];   // g_mu, G6, g_lo
    __shared__ float s_app[kPbThreads][20];   // gcm (3), gvm, Y (16)
    const int P = a.vlanes, V = a.b.n_views;
    const int rows_per_block = kPbThreads / P;
    const int lr = threadIdx.x / P, vl = threadIdx.x % P;
    const int64_t st = a.g.stride;
    int64_t na = a.rl.n_active ? (int64_t)*a.rl.n_active : a.rl.n_active_host;
    na = na < 0 ? 0 : (na > a.rl.Acap ? a.rl.Acap : na);
    int64_t nd = a.rl.n_delta ? (int64_t)*a.rl.n_delta : 0;
    nd = nd < 0 ? 0 : (nd > a.rl.Rcap - a.rl.Acap ? a.rl.Rcap - a.rl.Acap : nd);
    const int64_t nrec = na + nd;   // listed records: pair index = view * nrec + listed index
    const float sigma = *a.sigma;
    double gsig = 0.0;

    for (int64_t base = (int64_t)blockIdx.x * rows_per_block; base < na;
         base += (int64_t)gridDim.x * rows_per_block) {
        const int64_t t = base + lr;
        const bool row_ok = t < na;
        const int64_t id = row_ok ? (a.rl.active_idx ? (int64_t)a.rl.active_idx[t] : t) : 0;
        float mu[3], s3[3], qn[4], Rq[9], S6[6], qi = 1.f;
        if (row_ok) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                mu[k] = a.sp.mean[3 * id + k];
                s3[k] = expf(a.sp.log_scale[3 * id + k]);
            }
            float q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = a.sp.quat[4 * id + k];
            qi = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
            for (int k = 0; k < 4; ++k) qn[k] = q[k] * qi;
            quat_rot(qn[0], qn[1], qn[2], qn[3], Rq);
            cov3d(Rq, s3, S6);
        }
        {
            ViewPart o;
            if (row_ok && vl < V) {
                view_partials(a, nrec, t, id, vl, mu, S6, sigma, o);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) o.g_mu[k] = 0.f;
#pragma unroll
                for (int k = 0; k < 6; ++k) o.G6[k] = 0.f;
                o.g_lo = 0.f;
                o.gcm[0] = o.gcm[1] = o.gcm[2] = 0.f;
                o.gvm = 0.f;
#pragma unroll
                for (int k = 0; k < 16; ++k) o.Y[k] = 0.f;
                o.gsig = 0.0;
            }
            gsig += o.gsig;
#pragma unroll
            for (int k = 0; k < 3; ++k) s_geo[threadIdx.x][k] = o.g_mu[k];
#pragma unroll
            for (int k = 0; k < 6; ++k) s_geo[threadIdx.x][3 + k] = o.G6[k];
            s_geo[threadIdx.x][9] = o.g_lo;
#pragma unroll
            for (int k = 0; k < 3; ++k) s_app[threadIdx.x][k] = o.gcm[k];
            s_app[threadIdx.x][3] = o.gvm;
#pragma unroll
            for (int k = 0; k < 16; ++k) s_app[threadIdx.x][4 + k] = o.Y[k];
        }
        __syncthreads();
        const int g0 = lr * P;   // first lane of this row's group
        // SH outputs: j < 48 -> sh[j] (basis j / 3, channel j % 3); j >= 48 -> vsh[j - 48]
        float nsh = 0.f, nvsh = 0.f;
        for (int j = vl; j < 64; j += P) {
            float acc = 0.f;
            if (j < 48) {
                const int k = j / 3, ch = j % 3;
                for (int u = 0; u < V; ++u) acc = fmaf(s_app[g0 + u][ch], s_app[g0 + u][4 + k], acc);
                if (row_ok) a.g.sh[j * st + t] = acc;
                nsh += acc * acc;
            } else {
                const int k = j - 48;
                for (int u = 0; u < V; ++u) acc = fmaf(s_app[g0 + u][3], s_app[g0 + u][4 + k], acc);
                if (row_ok) a.g.vsh[k * st + t] = acc;
                nvsh += acc * acc;
            }
        }
        // the row's squared norms of the sh / vsh outputs: a butterfly over its P lanes
        // (P divides 64, so a row's lanes are within one wave)
        for (int o = 1; o < P; o <<= 1) {
            nsh += __shfl_xor(nsh, o);
            nvsh += __shfl_xor(nvsh, o);
        }
        if (row_ok && vl == 0) {
            float g_mu[3] = {0.f, 0.f, 0.f}, G6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, g_lo = 0.f;
            float n2[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int u = 0; u < V; ++u) {
#pragma unroll
                for (int k = 0; k < 3; ++k) g_mu[k] += s_geo[g0 + u][k];
#pragma unroll
                for (int k = 0; k < 6; ++k) G6[k] += s_geo[g0 + u][3 + k];
                g_lo += s_geo[g0 + u][9];
            }
            n2[4] = nsh;
            n2[5] = nvsh;
            // Sigma = M M^T, M = Rq diag(s):  dL/dM = 2 G M
            const float Gf[9] = {G6[0], G6[1], G6[2], G6[1], G6[3], G6[4], G6[2], G6[4], G6[5]};
            float gRq[9], g_ls[3];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                float gsj = 0.f;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    float gm = 0.f;
#pragma unroll
                    for (int k = 0; k < 3; ++k) gm += Gf[3 * i + k] * Rq[3 * k + jj] * s3[jj];
                    gm *= 2.f;
                    gsj += gm * Rq[3 * i + jj];
                    gRq[3 * i + jj] = gm * s3[jj];
                }
                g_ls[jj] = gsj * s3[jj];
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
            const float o = 1.f / (1.f + expf(-a.sp.logit[id]));
            const float g_logit = g_lo * (1.f - o) / kLn2;
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
            if (a.score) {
                float sc = 0.f;
#pragma unroll
                for (int k = 0; k < 6; ++k) sc = fmaxf(sc, sqrtf(n2[k]) / a.eps[k]);
                a.score[id] = sc;
            }
        }
        __syncthreads();
    }
    const double t = block_sum_double(gsig);
    if (threadIdx.x == 0) a.b.sig_part[kSigPixParts + blockIdx.x] = t;
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
    int P = 1;
    while (P < b.n_views) P *= 2;
    a.vlanes = P;
    const int64_t rows_per_block = kPbThreads / P;
    int64_t blocks = (rl.Acap + rows_per_block - 1) / rows_per_block;
    if (blocks > kPbBlocks) blocks = kPbBlocks;
    if (blocks > 0) hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)blocks), dim3(kPbThreads), 0, s, a);
    hipLaunchKernelGGL(k_sum_shares, dim3(1), dim3(kSumThreads), 0, s, (const double *)b.sig_part,
                       (int)pixel_blocks(b.total_px), (const double *)(b.sig_part + kSigPixParts), (int)blocks,
                       grad_sigma);
}

}  // namespace oit
