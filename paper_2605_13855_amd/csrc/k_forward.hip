// Forward pass: projection, tile binning without depth order, and the per-pixel
// blend-and-normalise / blend-and-update pass (App. A, Alg. "rasterize").
#include <hip/hip_ext.h>


#include "oit_internal.h"

namespace oit {

// ---------------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------------
// Cameras travel as kernel arguments (graph capture records them by value); 24 of
// them (2.9 KB) per launch, below the kernel-argument limit.
constexpr int kCamChunk = 24;
struct CamChunk {
    CamDev c[kCamChunk];
};
static_assert(sizeof(CamChunk) <= 3584, "cameras of one upload fit the kernel arguments");

__global__ void k_upload_cams(CamChunk chunk, int n, CamDev *dst)
{
    const int i = threadIdx.x;
    if (i < n) dst[i] = chunk.c[i];
}

void upload_cams(const CamDev *host, int n_views, CamDev *dst, hipStream_t s)
{
    for (int base = 0; base < n_views; base += kCamChunk) {
        CamChunk ch;
        const int k = n_views - base < kCamChunk ? n_views - base : kCamChunk;
        for (int i = 0; i < k; ++i) ch.c[i] = host[base + i];
        hipLaunchKernelGGL(k_upload_cams, dim3(1), dim3(64), 0, s, ch, k, dst + base);
    }
}

template <typename T>
__global__ void k_fill(T *p, size_t n, T v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T>
static void fill_any(T *p, size_t n, T v, hipStream_t s)
{
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

void fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) { fill_any(p, n, v, s); }
void fill_f32(float *p, size_t n, float v, hipStream_t s) { fill_any(p, n, v, s); }
void fill_f64(double *p, size_t n, double v, hipStream_t s) { fill_any(p, n, v, s); }

// ---------------------------------------------------------------------------------
// row lookup shared by the per-record kernels
// ---------------------------------------------------------------------------------
// Returns the splat id of record t, or -1 if the record is unused in this call.
// sign: 0 for an active record, -1 / +1 for a label change.
__device__ __forceinline__ int64_t record_row(const RowList &rl, int64_t t, int &sign)
{
    if (t < rl.Acap) {
        const int64_t na = rl.n_active ? (int64_t)*rl.n_active : rl.n_active_host;
        if (t >= na) return -1;
        sign = 0;
        return rl.active_idx ? (int64_t)rl.active_idx[t] : t;
    }
    const int64_t k = t - rl.Acap;
    const int64_t nd = rl.n_delta ? (int64_t)*rl.n_delta : 0;
    if (k >= nd) return -1;
    sign = rl.delta_sign[k] < 0 ? -1 : 1;
    return (int64_t)rl.delta_idx[k];
}

// Tile test of the record in the rasteriser's own units: the record's exponent is
// e = lo - m' with m' = A dx^2 + 2 B dx dy + C dy^2, A = -qa, B = -qb / 2, C = -qc;
// a pair contributes iff m' <= lo + log2(255).  The bound is widened slightly so that
// a tile is never dropped for a pair the per-pixel float test would keep.
__device__ __forceinline__ float tile_tau(float lo) { return (lo - kLog2AlphaMin) * 1.0001f + 1e-4f; }

__device__ __forceinline__ bool tile_hit(const Rec &r, float tau, const CamDev &cam, int S, int tx, int ty)
{
    const float px0 = (float)(tx * S) + 0.5f;
    const float px1 = (float)min(tx * S + S, cam.W) - 0.5f;
    const float py0 = (float)(ty * S) + 0.5f;
    const float py1 = (float)min(ty * S + S, cam.H) - 0.5f;
    return ellipse_hits_rect(-r.a.z, -0.5f * r.a.w, -r.b.x, tau, px0 - r.a.x, px1 - r.a.x, py0 - r.a.y,
                             py1 - r.a.y);
}

// ---------------------------------------------------------------------------------
// Work items of the per-record kernels: one (listed record, view) pair per item, the
// records being the call's active rows and then its label changes.  The counts live
// on the device, so the grid is fixed and strides over them.
// ---------------------------------------------------------------------------------
constexpr unsigned kRecBlocks = 2048;

struct RecItems {
    int64_t na, nrec, total;   // listed active rows; listed records (na + n_delta); items = nrec * views
};

__device__ __forceinline__ RecItems rec_items(const RowList &rl, int n_views)
{
    int64_t na = rl.n_active ? (int64_t)*rl.n_active : rl.n_active_host;
    na = na < 0 ? 0 : (na > rl.Acap ? rl.Acap : na);
    int64_t nd = rl.n_delta ? (int64_t)*rl.n_delta : 0;
    const int64_t dcap = rl.Rcap - rl.Acap;
    nd = nd < 0 ? 0 : (nd > dcap ? dcap : nd);
    return RecItems{na, na + nd, (na + nd) * n_views};
}

// record index of listed record k (active rows first, then label changes)
__device__ __forceinline__ int64_t rec_of(const RowList &rl, int64_t na, int64_t k)
{
    return k < na ? k : rl.Acap + (k - na);
}

// ---------------------------------------------------------------------------------
// preprocess: one thread per (listed record, view); projects the splat, writes the
// record and its tile rectangle and counts the tiles it reaches.
// ---------------------------------------------------------------------------------
struct PreArgs {
    SplatPtrs sp;    // active rows
    SplatPtrs dsp;   // label-change rows
    const float *sigma;
    RowList rl;
    Buffers b;
};

// What the tile count of one (record, view) pair takes: the record's exponent form
// (mx, my, qa, qb, qc of the record), the test's bound, the tile rectangle and the view.
struct CountItem {
    float mx, my, qa, qb, qc, tau, lo;
    int org;    // rectangle origin: x | y << 16
    int wv;     // rectangle width | view << 16
    int area;   // tiles of the rectangle (0: nothing to count)
};

// t: record index; v: view.  Writes the record and its tile rectangle; returns false
// if the record is unused in this call.
__device__ bool preprocess_one(const PreArgs &a, int64_t t, int v, CountItem &ci)
{
    int sign = 0;
    const int64_t id = record_row(a.rl, t, sign);
    if (id < 0) return false;
    const SplatPtrs &sp = sign == 0 ? a.sp : a.dsp;
    const CamDev &cam = a.b.cams[v];
    const size_t ri = (size_t)v * a.rl.Rcap + t;

    float mu[3], s3[3], q[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mu[k] = sp.mean[3 * id + k];
        s3[k] = expf(sp.log_scale[3 * id + k]);
    }
    {
        const float4 q4 = ((const float4 *)sp.quat)[id];
        q[0] = q4.x;
        q[1] = q4.y;
        q[2] = q4.z;
        q[3] = q4.w;
    }
    const float qi = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    float Rq[9], S6[6];
    quat_rot(q[0] * qi, q[1] * qi, q[2] * qi, q[3] * qi, Rq);
    cov3d(Rq, s3, S6);

    Rec r;
    short4 rect = make_short4(0, 0, 0, 0);
    Geo g;
    if (geometry(cam, mu, S6, g)) {
        const float lo = -log2f(1.f + expf(-sp.logit[id]));   // log2(sigmoid(logit))
        float dir[3] = {mu[0] - cam.cc[0], mu[1] - cam.cc[1], mu[2] - cam.cc[2]};
        const float di = rsqrtf(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        dir[0] *= di;
        dir[1] *= di;
        dir[2] *= di;
        float Y[16];
        sh_eval(dir[0], dir[1], dir[2], Y);
        float col[3] = {kColorOffset, kColorOffset, kColorOffset};
        float vr = kColorOffset;
        // the splat's 48 colour and 16 view-weight coefficients: 16 contiguous float4
        const float4 *sh4 = (const float4 *)sp.sh + 12 * id;
        const float4 *vsh4 = (const float4 *)sp.vsh + 4 * id;
#pragma unroll
        for (int j = 0; j < 12; ++j) {   // float4 j holds coefficients 4j .. 4j+3 of [16][3]
            const float4 c4 = sh4[j];
            const float cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) col[(4 * j + e) % 3] += Y[(4 * j + e) / 3] * cv[e];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 c4 = vsh4[j];
            vr += Y[4 * j] * c4.x;
            vr += Y[4 * j + 1] * c4.y;
            vr += Y[4 * j + 2] * c4.z;
            vr += Y[4 * j + 3] * c4.w;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] = fmaxf(col[ch], 0.f);
        const float vv = fmaxf(vr, 0.f);
        const float sigma = *a.sigma;
        const float d = g.tc[2];
        const bool w_on = d < sigma;
        const float w = w_on ? (1.f - d / sigma) * vv : 0.f;
        const float h = -0.5f * kLog2e;
        r.a = make_float4(g.mx, g.my, h * g.con_a, 2.f * h * g.con_b);
        r.b = make_float4(h * g.con_c, lo, col[0], col[1]);
        // an active record carries dw/dsigma = v d / sigma^2 (0 where d >= sigma) for
        // the pixel sum dQ/dsigma of the forward pass
        if (sign == 0)
            r.c = make_float4(col[2], w, w_on ? vv * d / (sigma * sigma) : 0.f, 1.f);
        else
            r.c = make_float4(col[2], w_on ? vv : 0.f, d, (float)sign);

        const float tau = tile_tau(lo);
        if (tau > 0.f) {
            // footprint box of the (slightly widened) level set, in pixels, +1 px
            const float tau_px = tau * 2.f * kLn2;   // back to units of the unscaled form
            const float hx = sqrtf(tau_px * g.cov_a), hy = sqrtf(tau_px * g.cov_c);
            const float xl = fminf(fmaxf(g.mx - hx - 0.5f, -1e7f), 1e7f);
            const float xh = fminf(fmaxf(g.mx + hx - 0.5f, -1e7f), 1e7f);
            const float yl = fminf(fmaxf(g.my - hy - 0.5f, -1e7f), 1e7f);
            const float yh = fminf(fmaxf(g.my + hy - 0.5f, -1e7f), 1e7f);
            int x0 = (int)floorf(xl) - 1, x1 = (int)ceilf(xh) + 1;
            int y0 = (int)floorf(yl) - 1, y1 = (int)ceilf(yh) + 1;
            x0 = max(x0, 0);
            y0 = max(y0, 0);
            x1 = min(x1, cam.W - 1);
            y1 = min(y1, cam.H - 1);
            if (x0 <= x1 && y0 <= y1) {
                const int S = a.b.tile;
                rect = make_short4((short)(x0 / S), (short)(x1 / S + 1), (short)(y0 / S), (short)(y1 / S + 1));
                const int rw = rect.y - rect.x;
                ci = CountItem{r.a.x, r.a.y, r.a.z, r.a.w, r.b.x, tau, lo, (int)rect.x | ((int)rect.z << 16),
                               rw | (v << 16), rw * (rect.w - rect.z)};
            }
        }
    } else {
        r.a = make_float4(0.f, 0.f, 0.f, 0.f);
        r.b = make_float4(0.f, -1e30f, 0.f, 0.f);
        r.c = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    Rec &dst = a.b.rec[ri];   // the padding is left unwritten
    dst.a = r.a;
    dst.b = r.b;
    dst.c = r.c;
    a.b.rect[ri] = rect;
    return true;
}

// Tiles of each lane's rectangle that its record reaches (tile_hit), counted by the
// whole wave: the 64 rectangles are laid end to end (lane order, tile rows within a
// rectangle) and the wave tests 64 consecutive tiles of that sequence per round, each
// lane taking the values of the tile's owner from the owner's lane; an owner adds the
// round's hits in its own stretch of the sequence.  (The rectangles differ widely in
// size, so a lane walking its own would keep the wave as long as its largest.)
__device__ uint32_t wave_count_hits(const CountItem &ci, const CamDev *cams, int S)
{
    const int lane = threadIdx.x & 63;
    int incl = ci.area;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int excl = incl - ci.area, total = __shfl(incl, 63);
    uint32_t hits = 0;
    for (int f0 = 0; f0 < total; f0 += 64) {
        const int f = f0 + lane;
        // owner of position f: the last lane whose rectangle starts at or before f
        int p = 0;
        for (int step = 32; step > 0; step >>= 1) {
            const int e = __shfl(excl, p + step);
            if (e <= f) p += step;
        }
        const int j = f - __shfl(excl, p);
        const int porg = __shfl(ci.org, p), pwv = __shfl(ci.wv, p);
        Rec r{};
        r.a = make_float4(__shfl(ci.mx, p), __shfl(ci.my, p), __shfl(ci.qa, p), __shfl(ci.qb, p));
        r.b.x = __shfl(ci.qc, p);
        const float ptau = __shfl(ci.tau, p);
        bool hit = false;
        if (f < total) {
            const uint32_t w = (uint32_t)(pwv & 0xffff);
            const int ty = (porg >> 16) + (int)((uint32_t)j / w), tx = (porg & 0xffff) + (int)((uint32_t)j % w);
            hit = tile_hit(r, ptau, cams[pwv >> 16], S, tx, ty);
        }
        const uint64_t hb = __ballot(hit);
        const int s0 = max(excl - f0, 0), s1 = min(excl + ci.area - f0, 64);
        if (s1 > s0) {
            const uint64_t m = s1 - s0 == 64 ? ~0ull : ((1ull << (s1 - s0)) - 1ull) << s0;
            hits += (uint32_t)__builtin_popcountll(hb & m);
        }
    }
    return hits;
}

// Four waves per SIMD: the projection and colour terms fit in 128 registers without spills.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_preprocess_count(PreArgs a)
{
    const int V = a.b.n_views;
    const RecItems it = rec_items(a.rl, V);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t sk = stride / V, sv = stride % V;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t k = i / V;
    int v = (int)(i % V);
    // a wave's 64 items are consecutive, so the loop is uniform over the wave
    for (; i - (threadIdx.x & 63) < it.total; i += stride) {
        CountItem ci{};
        const bool listed = i < it.total && preprocess_one(a, rec_of(a.rl, it.na, k), v, ci);
        const uint32_t hits = wave_count_hits(ci, a.b.cams, a.b.tile);
        if (listed) {
            a.b.nhits[(size_t)v * it.nrec + k] = hits;
            // the raster forward clamps alpha at the cap only if some listed record can reach it
            if (hits && ci.lo > kLog2NoCap) atomicOr(&a.b.counters[CNT_CAP], 1u);
        }
        k += sk;
        v += (int)sv;
        if (v >= V) {
            v -= V;
            ++k;
        }
    }
}

void launch_preprocess_count(const SplatPtrs &sp, const SplatPtrs &dsp, const float *sigma, const RowList &rl,
                             const Buffers &b, hipStream_t s)
{
    PreArgs a{sp, dsp, sigma, rl, b};
    if (rl.Rcap > 0) hipLaunchKernelGGL(k_preprocess_count, dim3(kRecBlocks), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------------
// exclusive scans of per-tile entry counts and backward chunk counts (one block)
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(Buffers b)
{
    __shared__ unsigned long long s_e[kScanThreads / 64];
    __shared__ unsigned long long s_c[kScanThreads / 64];
    const int T = b.T;
    const int tid = threadIdx.x;
    const int seg = (T + kScanThreads - 1) / kScanThreads;
    const int t0 = min(tid * seg, T), t1 = min(t0 + seg, T);
    // a thread's counts are loaded all at once when they fit in registers (one memory
    // latency for the segment instead of one per tile)
    constexpr int kRegs = 32;
    const bool in_regs = seg <= kRegs;
    uint32_t ra[kRegs], rd[kRegs];
    unsigned long long se = 0, sc = 0;
    if (in_regs) {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            const bool ok = t0 + j < t1;
            ra[j] = ok ? b.cnt_a[t0 + j] : 0u;
            rd[j] = ok ? b.cnt_d[t0 + j] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            se += ra[j] + rd[j];
            sc += (ra[j] + kBwdLanes - 1) / kBwdLanes;
        }
    } else {
        for (int t = t0; t < t1; ++t) {
            const uint32_t na = b.cnt_a[t];
            se += na + b.cnt_d[t];
            sc += (na + kBwdLanes - 1) / kBwdLanes;
        }
    }
    // inclusive scans over each wave by shuffles, then the 16 wave totals in LDS
    const int lane = tid & 63, wave = tid >> 6;
    unsigned long long xe = se, xc = sc;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long ye = __shfl_up(xe, o), yc = __shfl_up(xc, o);
        if (lane >= o) {
            xe += ye;
            xc += yc;
        }
    }
    if (lane == 63) {
        s_e[wave] = xe;
        s_c[wave] = xc;
    }
    __syncthreads();
    unsigned long long be = 0, bc = 0;
    for (int w = 0; w < wave; ++w) {
        be += s_e[w];
        bc += s_c[w];
    }
    unsigned long long pe = be + xe - se, pc = bc + xc - sc;
    const unsigned long long cap = (unsigned long long)b.pair_cap;
    if (in_regs) {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            if (t0 + j < t1) {
                b.tile_off[t0 + j] = (uint32_t)(pe < cap ? pe : cap);
                b.chunk_off[t0 + j] = (uint32_t)pc;
            }
            pe += ra[j] + rd[j];
            pc += (ra[j] + kBwdLanes - 1) / kBwdLanes;
        }
    } else {
        for (int t = t0; t < t1; ++t) {
            b.tile_off[t] = (uint32_t)(pe < cap ? pe : cap);
            b.chunk_off[t] = (uint32_t)pc;
            const uint32_t na = b.cnt_a[t];
            pe += na + b.cnt_d[t];
            pc += (na + kBwdLanes - 1) / kBwdLanes;
        }
    }
    if (tid == kScanThreads - 1) {
        const unsigned long long te = be + xe, tc = bc + xc;
        b.tile_off[T] = (uint32_t)(te < cap ? te : cap);
        b.chunk_off[T] = (uint32_t)tc;
        b.counters[CNT_TOTAL_CHUNKS] = (uint32_t)tc;
    }
}

// The forward's launch order: the tiles by decreasing entry count (a quarter-octave
// bucket of the count; any order within a bucket), so that the heaviest tiles start
// first and the launch ends on light ones (longest-first list scheduling; the largest
// tile holds about 2.7 times the mean at config 4).  One block; the order within a
// bucket follows LDS atomics and changes no result (each tile is independent).
// It also resets the forward's work-queue ticket, which the raster forward launched
// after it on the same stream takes tiles from.
constexpr int kOrderBuckets = 128;

__global__ __launch_bounds__(1024) void k_tile_order(Buffers b)
{
    __shared__ uint32_t s_n[kOrderBuckets], s_pos[kOrderBuckets];
    const int T = b.T;
    if (threadIdx.x == 0) b.counters[CNT_FQUEUE] = 0u;
    auto bucket = [&](int t) {
        const uint32_t w = b.cnt_a[t] + b.cnt_d[t];
        const int q = (int)(4.f * __builtin_amdgcn_logf((float)w + 1.f));   // log2 of the count, x 4
        return kOrderBuckets - 1 - min(q, kOrderBuckets - 1);                // heaviest first
    };
    for (int k = threadIdx.x; k < kOrderBuckets; k += blockDim.x) s_n[k] = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += blockDim.x) atomicAdd(&s_n[bucket(t)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < kOrderBuckets; ++k) {
            s_pos[k] = acc;
            acc += s_n[k];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += blockDim.x) b.tile_order[atomicAdd(&s_pos[bucket(t)], 1u)] = (uint32_t)t;
}

void launch_scan_tiles(const Buffers &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, b);
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, b);
}

// ---------------------------------------------------------------------------------
// device-wide exclusive scan of n uint32 values in three launches: the sum of every
// block of kScanBlockItems values, an exclusive scan of those sums by one block, and
// a rescan of each block's values from its offset
// ---------------------------------------------------------------------------------
constexpr int kScanPer = kScanBlockItems / 256;   // values per thread

__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t s_v[256];
    s_v[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t t = threadIdx.x >= (unsigned)off ? s_v[threadIdx.x - off] : 0u;
        __syncthreads();
        s_v[threadIdx.x] += t;
        __syncthreads();
    }
    const uint32_t incl = s_v[threadIdx.x];
    if (total) *total = s_v[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t *in, int64_t n, uint32_t *bsum)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlockItems;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + (int64_t)k * 256 + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot = 0;
    block_excl_scan256(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_block_sums(uint32_t *bsum, int64_t nb)
{
    __shared__ uint32_t s_v[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t seg = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = (int64_t)tid * seg < nb ? (int64_t)tid * seg : nb;
    const int64_t b1 = b0 + seg < nb ? b0 + seg : nb;
    uint32_t acc = 0;
    for (int64_t i = b0; i < b1; ++i) acc += bsum[i];
    s_v[tid] = acc;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t t = tid >= off ? s_v[tid - off] : 0u;
        __syncthreads();
        s_v[tid] += t;
        __syncthreads();
    }
    uint32_t pre = s_v[tid] - acc;
    for (int64_t i = b0; i < b1; ++i) {
        const uint32_t x = bsum[i];
        bsum[i] = pre;
        pre += x;
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *in, int64_t n, const uint32_t *bsum,
                                                    uint32_t *out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlockItems + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        acc += v[k];
    }
    uint32_t pre = block_excl_scan256(acc, nullptr) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = pre;
        pre += v[k];
    }
}

// the same scan for a count that lives on the device: a fixed grid of kScanGrid blocks,
// each scanning a contiguous range of whole kScanBlockItems tiles.  The sums are formed
// in 64 bits and stored saturated at 2^32 - 1: a prefix at or past that value is past
// every pair capacity (which is below 2^32 - 1), so its entries are dropped and the
// overflow is reported instead of the offsets wrapping round.
constexpr unsigned kScanGrid = kScanThreads;   // the workspace holds this many block sums
constexpr uint64_t kSat32 = 0xffffffffull;

__device__ __forceinline__ uint32_t sat32(uint64_t x) { return (uint32_t)(x < kSat32 ? x : kSat32); }

__device__ __forceinline__ uint64_t block_excl_scan256_u64(uint64_t v, uint64_t *total)
{
    __shared__ uint64_t s_w[256];
    s_w[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t t = threadIdx.x >= (unsigned)off ? s_w[threadIdx.x - off] : 0ull;
        __syncthreads();
        s_w[threadIdx.x] += t;
        __syncthreads();
    }
    const uint64_t incl = s_w[threadIdx.x];
    if (total) *total = s_w[255];
    __syncthreads();
    return incl - v;
}

// exclusive scan of the kScanGrid block sums in place, saturated (one block)
__global__ __launch_bounds__(kScanThreads) void k_scan_block_sums_sat(uint32_t *bsum)
{
    __shared__ uint64_t s_v[kScanThreads];
    static_assert(kScanGrid == kScanThreads, "one block sum per thread");
    const int tid = threadIdx.x;
    const uint64_t x = bsum[tid];
    s_v[tid] = x;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint64_t t = tid >= off ? s_v[tid - off] : 0ull;
        __syncthreads();
        s_v[tid] += t;
        __syncthreads();
    }
    bsum[tid] = sat32(s_v[tid] - x);
}

__device__ __forceinline__ void scan_range(uint64_t n, uint64_t &lo, uint64_t &hi)
{
    uint64_t chunk = (n + kScanGrid - 1) / kScanGrid;
    chunk = (chunk + kScanBlockItems - 1) / kScanBlockItems * kScanBlockItems;
    lo = (uint64_t)blockIdx.x * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
    if (lo > hi) lo = hi;
}

__global__ __launch_bounds__(256) void k_scan_sums_dev(const uint32_t *in, const uint32_t *nptr, uint32_t *bsum)
{
    uint64_t lo, hi;
    scan_range(*nptr, lo, hi);
    uint64_t acc = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) acc += in[i];
    uint64_t tot = 0;
    block_excl_scan256_u64(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = sat32(tot);
}

__global__ __launch_bounds__(256) void k_scan_apply_dev(const uint32_t *in, const uint32_t *nptr,
                                                        const uint32_t *bsum, uint32_t *out)
{
    uint64_t lo, hi;
    scan_range(*nptr, lo, hi);
    uint64_t carry = bsum[blockIdx.x];
    for (uint64_t base = lo; base < hi; base += kScanBlockItems) {
        const uint64_t t0 = base + (uint64_t)threadIdx.x * kScanPer;
        uint32_t v[kScanPer];
        uint64_t acc = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = t0 + k < hi ? in[t0 + k] : 0u;
            acc += v[k];
        }
        uint64_t tot = 0;
        uint64_t pre = block_excl_scan256_u64(acc, &tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (t0 + k < hi) out[t0 + k] = sat32(pre);
            pre += v[k];
        }
        carry += tot;
    }
}

// exclusive scan of n (device count) uint32 values, saturated at 2^32 - 1
void launch_scan_u32_dev(const uint32_t *in, uint32_t *out, const uint32_t *nptr, uint32_t *tmp, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_sums_dev, dim3(kScanGrid), dim3(256), 0, s, in, nptr, tmp);
    hipLaunchKernelGGL(k_scan_block_sums_sat, dim3(1), dim3(kScanThreads), 0, s, tmp);
    hipLaunchKernelGGL(k_scan_apply_dev, dim3(kScanGrid), dim3(256), 0, s, in, nptr, (const uint32_t *)tmp, out);
}

void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t nb = (n + kScanBlockItems - 1) / kScanBlockItems;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_block_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, n, (const uint32_t *)tmp, out);
}

// ---------------------------------------------------------------------------------
// Binning without depth order and without atomics (App. A: tiles are the only sort
// key).  The scan of the per-pair tile counts gives every (record, view) pair its slots
// [hoff, hoff + nhits) of an unsorted entry list, in pair order; a list pass writes
// each slot's key (tile, class: active 0, label change 1) and record; a stable LSD radix
// sort orders the list by key, so that within a tile the active entries come first and
// both classes keep pair order (the forward's sums are then reproducible run to run);
// binary searches in the sorted keys give each tile's range.
// ---------------------------------------------------------------------------------
struct ListArgs {
    RowList rl;
    Buffers b;
};

// number of (listed record, view) pairs of the call, for the scan of their tile counts
__global__ void k_pair_count(ListArgs a)
{
    const RecItems it = rec_items(a.rl, a.b.n_views);
    a.b.counters[CNT_NPAIRS] = (uint32_t)it.total;
}

// total tile entries E (saturated at 2^32 - 1: the scan saturates), the sorted list's
// length min(E, capacity), overflow status
__global__ void k_list_total(ListArgs a)
{
    const uint32_t np = a.b.counters[CNT_NPAIRS];
    const uint64_t E = np ? (uint64_t)a.b.hoff[np - 1] + a.b.nhits[np - 1] : 0;
    const uint64_t cap = (uint64_t)a.b.pair_cap;
    a.b.counters[CNT_TOTAL_ENTRIES] = (uint32_t)(E < 0xffffffffull ? E : 0xffffffffull);
    a.b.counters[CNT_SORT_N] = (uint32_t)(E < cap ? E : cap);
    if (E > cap) atomicOr(a.b.status, OIT_STATUS_PAIR_OVERFLOW);
}

// Sort key of a tile entry: (tile, class) and a size class, 3 log2 of the pixel count of
// the footprint box (half-extents hx, hy around the mean mx, my; hx < 0: none) inside the
// tile, so that a 64-entry backward chunk holds footprints of similar size.
__device__ __forceinline__ uint32_t entry_key(const CamDev &cam, int S, int tx, int ty, uint32_t cls, float mx,
                                              float my, float hx, float hy)
{
    const uint32_t tile = (uint32_t)(cam.tile_base + ty * cam.tiles_x + tx);
    uint32_t sc = 0;
    if (hx >= 0.f) {
        const float dx0 = (float)(tx * S) + 0.5f - mx, dy0 = (float)(ty * S) + 0.5f - my;
        const float lim = 1e6f;
        const int c0 = max(0, (int)ceilf(fmaxf(-hx - dx0, -lim)));
        const int c1 = min(min(S, cam.W - tx * S) - 1, (int)floorf(fminf(hx - dx0, lim)));
        const int r0 = max(0, (int)ceilf(fmaxf(-hy - dy0, -lim)));
        const int r1 = min(min(S, cam.H - ty * S) - 1, (int)floorf(fminf(hy - dy0, lim)));
        const int area = (c1 >= c0 && r1 >= r0) ? (c1 - c0 + 1) * (r1 - r0 + 1) : 0;
        if (area > 1) sc = min((1u << kSizeBits) - 1u, (uint32_t)(3.f * log2f((float)area)));
    }
    return ((tile * 2u + cls) << kSizeBits) | sc;
}

// View-major items: a wave takes 64 consecutive (record, view) pairs, whose slots form
// one contiguous range.  Their tile rectangles differ widely in size (at the benchmark
// scenes a wave's largest is about three times their mean), so the lanes do not walk
// their own rectangles: the wave lays the 64 rectangles end to end (pair order, tile
// rows within a rectangle, the count's order) and tests 64 consecutive tiles of that
// sequence per round, each lane taking the pair values of the tile's owner from the
// owner's lane.  A hit's slot is the wave's first slot plus the hits before it in the
// sequence, so a round stores its hits as one contiguous run.
__global__ __launch_bounds__(256) void k_list(ListArgs a)
{
    const int V = a.b.n_views;
    const RecItems it = rec_items(a.rl, V);
    const int lane = threadIdx.x & 63;
    const int S = a.b.tile;
    const uint64_t cap = (uint64_t)a.b.pair_cap;
    const bool per_pixel = a.b.bwd_mode == OIT_BWD_PER_PIXEL;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; i0 < it.total;
         i0 += (int64_t)gridDim.x * 256) {
        const int64_t i = i0 + lane;
        // the lane's own pair: rectangle origin (x | y << 16), width | class << 15 |
        // view << 16, record, tile-test form and footprint box
        int area = 0, org = 0, wcv = 0;
        uint32_t rec = 0;
        float mx = 0.f, my = 0.f, qa = 0.f, qb = 0.f, qc = 0.f, tau = 0.f, hx = -1.f, hy = -1.f;
        if (i < it.total) {
            const int v = (int)(i / it.nrec);
            const int64_t t = rec_of(a.rl, it.na, i - (int64_t)v * it.nrec);
            int sign = 0;
            if (record_row(a.rl, t, sign) >= 0 && a.b.nhits[i] != 0) {
                const size_t ri = (size_t)v * a.rl.Rcap + t;
                const short4 rect = a.b.rect[ri];
                const Rec r = a.b.rec[ri];
                mx = r.a.x;
                my = r.a.y;
                qa = r.a.z;
                qb = r.a.w;
                qc = r.b.x;
                tau = tile_tau(r.b.y);
                // half-extents of the widened alpha >= 1/255 box (the backward's, same formulas)
                const float A = -qa, B = -0.5f * qb, C = -qc;
                const float det = A * C - B * B;
                const float tb = (r.b.y - kLog2AlphaMin) * 1.001f + 1e-3f;
                if (tb > 0.f && det > 0.f) {
                    hx = sqrtf(tb * C / det) + 0.01f;
                    hy = sqrtf(tb * A / det) + 0.01f;
                }
                const int w = rect.y - rect.x;
                area = w * (rect.w - rect.z);
                org = (int)rect.x | ((int)rect.z << 16);
                wcv = w | ((sign == 0 ? 0 : 1) << 15) | (v << 16);
                rec = (uint32_t)t;
            }
        }
        // the lane's rectangle starts at position excl of the wave's sequence
        int incl = area;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const int excl = incl - area, total = __shfl(incl, 63);
        uint64_t slot = a.b.hoff[i0];
        for (int f0 = 0; f0 < total; f0 += 64) {
            const int f = f0 + lane;
            // owner of position f: the last lane whose rectangle starts at or before f
            // (it has a nonempty rectangle when f < total)
            int p = 0;
            for (int step = 32; step > 0; step >>= 1) {
                const int e = __shfl(excl, p + step);
                if (e <= f) p += step;
            }
            const int j = f - __shfl(excl, p);
            const int porg = __shfl(org, p), pwcv = __shfl(wcv, p);
            const uint32_t prec = (uint32_t)__shfl((int)rec, p);
            Rec r{};
            r.a = make_float4(__shfl(mx, p), __shfl(my, p), __shfl(qa, p), __shfl(qb, p));
            r.b.x = __shfl(qc, p);
            const float ptau = __shfl(tau, p), phx = __shfl(hx, p), phy = __shfl(hy, p);
            bool hit = false;
            uint32_t key = 0, cls = 0;
            if (f < total) {
                const uint32_t w = (uint32_t)(pwcv & 0x7fff);
                cls = (uint32_t)(pwcv >> 15) & 1u;
                const CamDev &cam = a.b.cams[pwcv >> 16];
                const int ty = (porg >> 16) + (int)((uint32_t)j / w), tx = (porg & 0xffff) + (int)((uint32_t)j % w);
                hit = tile_hit(r, ptau, cam, S, tx, ty);
                if (hit) key = entry_key(cam, S, tx, ty, cls, r.a.x, r.a.y, phx, phy);
            }
            const uint64_t hb = __ballot(hit);
            if (hit) {
                const uint64_t o = slot + (uint64_t)__builtin_popcountll(hb & lt);
                if (o < cap) {
                    a.b.keys[0][o] = key;
                    a.b.vals[0][o] = (uint32_t)o;
                    a.b.recs[0][o] = prec;
                    if (per_pixel && cls == 0u) {
                        float4 *ep = (float4 *)(a.b.ep + o * kEpStride);
                        ep[0] = ep[1] = ep[2] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
            }
            slot += (uint64_t)__builtin_popcountll(hb);
        }
    }
}

// --- stable LSD radix sort of (key, value, record) triples, kRadixBits-bit digits ---
// A fixed grid of kSortGrid blocks; block b sorts the contiguous range of the n keys
// (n on the device) that sort_range gives it, so the work follows n, not the capacity,
// and the block order is the key order (stability).  The digit is narrow on purpose:
// every (block, digit) pair has a partly written output line per array, and with 32
// digits those lines (about 1.6 MB per XCD) stay in L2 until they are complete, where
// 256 digits would have them evicted half written.
__device__ __forceinline__ void sort_range(uint64_t n, uint64_t &lo, uint64_t &hi)
{
    uint64_t chunk = (n + kSortGrid - 1) / kSortGrid;
    chunk = (chunk + 255) & ~255ull;
    lo = (uint64_t)blockIdx.x * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
    if (lo > hi) lo = hi;
}

// Exclusive scan of the digit histograms (kRadixBuckets x kSortGrid values) in one
// block: each thread scans 32 consecutive counts in registers, the waves' totals meet
// in LDS (one launch instead of the three of the general scan).
constexpr int kHistScanPer = kRadixBuckets * kSortGrid / 1024;
static_assert(kHistScanPer == 32, "32 counts per thread");

__global__ __launch_bounds__(1024) void k_scan_hist(const uint32_t *in, uint32_t *out)
{
    __shared__ uint32_t s_w[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint4 *src = (const uint4 *)(in + (size_t)tid * kHistScanPer);
    uint32_t v[kHistScanPer];
#pragma unroll
    for (int k = 0; k < kHistScanPer / 4; ++k) {
        const uint4 q = src[k];
        v[4 * k] = q.x;
        v[4 * k + 1] = q.y;
        v[4 * k + 2] = q.z;
        v[4 * k + 3] = q.w;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kHistScanPer; ++k) sum += v[k];
    uint32_t x = sum;   // inclusive scan over the wave
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += s_w[w];
    uint32_t pre = base + x - sum;
    uint4 *dst = (uint4 *)(out + (size_t)tid * kHistScanPer);
#pragma unroll
    for (int k = 0; k < kHistScanPer / 4; ++k) {
        uint4 q;
        q.x = pre;
        pre += v[4 * k];
        q.y = pre;
        pre += v[4 * k + 1];
        q.z = pre;
        pre += v[4 * k + 2];
        q.w = pre;
        pre += v[4 * k + 3];
        dst[k] = q;
    }
}

// digit histogram of each block's range, digit-major: hist[d][block]
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *keys, const uint32_t *nptr, int shift,
                                                    uint32_t *hist)
{
    __shared__ uint32_t h[kRadixBuckets];
    if (threadIdx.x < kRadixBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t lo, hi;
    sort_range(*nptr, lo, hi);
    // four keys per thread in flight before their counts
    for (uint64_t b0 = lo; b0 < hi; b0 += 1024) {
        uint32_t k[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t i = b0 + u * 256 + threadIdx.x;
            k[u] = i < hi ? keys[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (b0 + u * 256 + threadIdx.x < hi) atomicAdd(&h[(k[u] >> shift) & (kRadixBuckets - 1u)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kRadixBuckets) hist[(size_t)threadIdx.x * kSortGrid + blockIdx.x] = h[threadIdx.x];
}

// Scatter each block's keys to their digit's range in key order, in rounds of 1024
// keys in index order (four per thread, loaded together so that a round's loads are in
// flight at once).  A key's rank among the equal digits of its wave comes from ballots
// over the digit's bits, the first position of each (key of the thread, wave) group per
// digit from a scan of the groups' counts in LDS.  The round is first ordered by digit
// in LDS and then written out by consecutive threads in that order, so that a store
// covers a few contiguous runs of its digits' ranges instead of up to one per digit.
// The counts have an array of their own that the scan clears after reading it.
constexpr int kScatterPer = 4;
constexpr int kScatterRound = kScatterPer * 256;

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *keys_in, const uint32_t *vals_in,
                                                       const uint32_t *recs_in, uint32_t *keys_out,
                                                       uint32_t *vals_out, uint32_t *recs_out, const uint32_t *nptr,
                                                       int shift, const uint32_t *hist_off)
{
    constexpr int kSub = kScatterPer * 4;   // groups of a round, in index order: (u, wave)
    __shared__ uint32_t run[kRadixBuckets];       // the digit's next output position
    __shared__ uint32_t gbase[kRadixBuckets];     // output position minus round slot, per digit
    __shared__ uint32_t cnt[kSub][kRadixBuckets], first[kSub][kRadixBuckets];
    __shared__ uint32_t s_key[kScatterRound], s_val[kScatterRound], s_rec[kScatterRound];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid < kRadixBuckets) run[tid] = hist_off[(size_t)tid * kSortGrid + blockIdx.x];
    for (int e = tid; e < kSub * kRadixBuckets; e += 256) (&cnt[0][0])[e] = 0;
    __syncthreads();
    uint64_t lo, hi;
    sort_range(*nptr, lo, hi);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint64_t base = lo; base < hi; base += kScatterRound) {
        uint32_t key[kScatterPer], val[kScatterPer], rec[kScatterPer], d[kScatterPer], rank[kScatterPer];
        bool valid[kScatterPer];
#pragma unroll
        for (int u = 0; u < kScatterPer; ++u) {
            const uint64_t i = base + u * 256 + tid;
            valid[u] = i < hi;
            key[u] = valid[u] ? keys_in[i] : 0u;
            val[u] = valid[u] ? vals_in[i] : 0u;
            rec[u] = valid[u] ? recs_in[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kScatterPer; ++u) {
            d[u] = (key[u] >> shift) & (kRadixBuckets - 1u);
            uint64_t peers = __ballot(valid[u]);
#pragma unroll
            for (int bit = 0; bit < kRadixBits; ++bit) {
                const bool set = (d[u] >> bit) & 1u;
                const uint64_t bb = __ballot(set);
                peers &= set ? bb : ~bb;
            }
            rank[u] = (uint32_t)__builtin_popcountll(peers & lt);
            if (valid[u] && rank[u] == 0) cnt[u * 4 + wave][d[u]] = (uint32_t)__builtin_popcountll(peers);
        }
        __syncthreads();
        if (wave == 0) {
            // lane dg < 32 scans digit dg's groups; the round's digit totals are then
            // scanned across those lanes for the digit's first slot of the round
            const int dg = lane & (kRadixBuckets - 1);
            uint32_t tot = 0;
            uint32_t c[kSub];
#pragma unroll
            for (int g = 0; g < kSub; ++g) {
                c[g] = cnt[g][dg];
                tot += c[g];
            }
            uint32_t x = lane < kRadixBuckets ? tot : 0u;   // inclusive scan over the digits
            for (int o = 1; o < kRadixBuckets; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane < kRadixBuckets) {
                uint32_t slot = x - tot;
                gbase[dg] = run[dg] - slot;
                run[dg] += tot;
#pragma unroll
                for (int g = 0; g < kSub; ++g) {
                    cnt[g][dg] = 0;
                    first[g][dg] = slot;
                    slot += c[g];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kScatterPer; ++u)
            if (valid[u]) {
                const uint32_t e = first[u * 4 + wave][d[u]] + rank[u];
                s_key[e] = key[u];
                s_val[e] = val[u];
                s_rec[e] = rec[u];
            }
        __syncthreads();
        const uint64_t nr = hi - base < (uint64_t)kScatterRound ? hi - base : (uint64_t)kScatterRound;
#pragma unroll
        for (int u = 0; u < kScatterPer; ++u) {
            const int e = u * 256 + tid;
            if ((uint64_t)e < nr) {
                const uint32_t k = s_key[e];
                const uint32_t pos = gbase[(k >> shift) & (kRadixBuckets - 1u)] + (uint32_t)e;
                keys_out[pos] = k;
                vals_out[pos] = s_val[e];
                recs_out[pos] = s_rec[e];
            }
        }
    }
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *a, uint32_t n, uint32_t x)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// per-tile entry counts from the sorted keys
__global__ __launch_bounds__(256) void k_tile_counts(const uint32_t *keys, const uint32_t *nptr, Buffers b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.T) return;
    const uint32_t n = *nptr;
    const uint32_t k0 = (2u * t) << kSizeBits, k1 = (2u * t + 1u) << kSizeBits, k2 = (2u * t + 2u) << kSizeBits;
    const uint32_t s0 = lower_bound_u32(keys, n, k0), s1 = lower_bound_u32(keys, n, k1),
                   s2 = lower_bound_u32(keys, n, k2);
    b.cnt_a[t] = s1 - s0;
    b.cnt_d[t] = s2 - s1;
}

void launch_binning(const RowList &rl, const Buffers &b, hipStream_t s)
{
    if ((int64_t)b.n_views * rl.Rcap <= 0) return;
    ListArgs la{rl, b};
    hipLaunchKernelGGL(k_pair_count, dim3(1), dim3(1), 0, s, la);
    launch_scan_u32_dev(b.nhits, b.hoff, b.counters + CNT_NPAIRS, b.scan_tmp, s);
    hipLaunchKernelGGL(k_list_total, dim3(1), dim3(1), 0, s, la);
    hipLaunchKernelGGL(k_list, dim3(kRecBlocks), dim3(256), 0, s, la);
    // keys are (tile * 2 + class) * 2^kSizeBits + size class < 2 T 2^kSizeBits: as many
    // kRadixBits-bit digits as that needs (>= 1); the last pass writes the unsorted
    // slots to `orig` and the records to `entries`
    const uint32_t kmax = (2u * (uint32_t)b.T) << kSizeBits;
    int bits = 0;
    while (bits < 32 && (kmax >> bits) != 0) ++bits;
    const int passes = bits == 0 ? 1 : (bits + kRadixBits - 1) / kRadixBits;
    const uint32_t *nptr = b.counters + CNT_SORT_N;
    int cur = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const bool last = ps == passes - 1;
        hipLaunchKernelGGL(k_radix_hist, dim3(kSortGrid), dim3(256), 0, s, (const uint32_t *)b.keys[cur], nptr,
                           kRadixBits * ps, b.hist);
        hipLaunchKernelGGL(k_scan_hist, dim3(1), dim3(1024), 0, s, (const uint32_t *)b.hist, b.hist_off);
        hipLaunchKernelGGL(k_radix_scatter, dim3(kSortGrid), dim3(256), 0, s, (const uint32_t *)b.keys[cur],
                           (const uint32_t *)b.vals[cur], (const uint32_t *)b.recs[cur], b.keys[cur ^ 1],
                           last ? b.orig : b.vals[cur ^ 1], last ? b.entries : b.recs[cur ^ 1], nptr,
                           kRadixBits * ps, (const uint32_t *)b.hist_off);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_tile_counts, dim3((unsigned)((b.T + 255) / 256)), dim3(256), 0, s,
                       (const uint32_t *)b.keys[cur], nptr, b);
    launch_scan_tiles(b, s);
}

// ---------------------------------------------------------------------------------
// raster forward: a tile is one workgroup's work (all views of the batch in one
// persistent launch, tiles dealt from a device queue heaviest first).
// Records of the tile's entries are staged through LDS in batches; every thread
// blends them into its pixels in list order (no depth order).  Each wave owns a
// compact block of the tile (16 x 16 pixels for 32-pixel tiles, else 8 x 8), and the
// staging step marks which blocks a record's footprint box reaches, so a wave skips
// the records that cannot touch its pixels.  A thread's pixels share one column, so
// the per-column exponent terms are formed once per record.
// ---------------------------------------------------------------------------------
// The tile at position k of the heavy-first order (k_tile_order).
__device__ __forceinline__ void fwd_tile_at(const Buffers &b, uint32_t k, int &v, int &tx, int &ty)
{
    const int tile = (int)b.tile_order[k];
    v = view_of_tile(b.cams, b.n_views, tile);
    const CamDev &cam = b.cams[v];
    const int lt = tile - cam.tile_base;
    tx = lt % cam.tiles_x;
    ty = lt / cam.tiles_x;
}

struct FwdArgs {
    Buffers b;
    const float *sigma;
    float bg0, bg1, bg2;
    float *pre, *image, *pixstate;
};

// A record that contributes nothing (its exponent is always below the threshold);
// stands in for any tile-list entry outside its class's record range.
__device__ const Rec kNoRec = {{0.f, 0.f, 0.f, 0.f}, {0.f, -1e30f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};

// Stage record r for a tile whose first pixel centre is (x0, y0): the mean is
// replaced by the offsets x0 - mx, y0 - my of the exponent form.  Returns the mask of
// the row strips that the footprint box of the record's (slightly widened) alpha >=
// 1/255 level set reaches: bit w * PPT + p for strip p of the tile's pixel block w (BW x
// BW blocks, WPR per row, NW in all; strip p holds rows [p RSTEP, (p + 1) RSTEP) of the
// block, the rows of a thread's pixel p).
template <int BW, int WPR, int NW, int PPT>
__device__ __forceinline__ int stage_rec(float4 *dst, const Rec &r, float x0, float y0)
{
    constexpr int RSTEP = BW / PPT;
    const float dx0 = x0 - r.a.x, dy0 = y0 - r.a.y;
    dst[0] = make_float4(dx0, dy0, r.a.z, r.a.w);
    dst[1] = r.b;
    dst[2] = r.c;
    const float A = -r.a.z, B = -0.5f * r.a.w, C = -r.b.x;
    const float det = A * C - B * B;
    const float tau = (r.b.y - kLog2AlphaMin) * 1.001f + 1e-3f;
    if (!(tau > 0.f && det > 0.f)) return 0;
    const float hx = sqrtf(tau * C / det) + 0.01f, hy = sqrtf(tau * A / det) + 0.01f;
    int mask = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const float bx = dx0 + (float)((w % WPR) * BW), by = dy0 + (float)((w / WPR) * BW);
        if (!(bx <= hx && bx + (float)(BW - 1) >= -hx)) continue;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const float sy = by + (float)(p * RSTEP);
            if (sy <= hy && sy + (float)(RSTEP - 1) >= -hy) mask |= 1 << (w * PPT + p);
        }
    }
    return mask;
}

// Does the footprint box of a staged record (st[0] = (x0 - mx, y0 - my, qa, qb),
// st[1] = (qc, lo, ...)) reach the rectangle [bx, bx + w - 1] x [by, by + h - 1] of the
// tile's pixel offsets?
__device__ __forceinline__ bool staged_hits_rect(const float4 &s0, const float4 &s1, int bx, int by, int w, int h)
{
    const float A = -s0.z, B = -0.5f * s0.w, C = -s1.x;
    const float det = A * C - B * B;
    const float tau = (s1.y - kLog2AlphaMin) * 1.001f + 1e-3f;
    if (!(tau > 0.f && det > 0.f)) return false;
    const float hx = sqrtf(tau * C / det) + 0.01f, hy = sqrtf(tau * A / det) + 0.01f;
    const float rx = s0.x + (float)bx, ry = s0.y + (float)by;
    return rx <= hx && rx + (float)(w - 1) >= -hx && ry <= hy && ry + (float)(h - 1) >= -hy;
}

// Blend-and-update one label-change record (staged at r) into a thread's PPT pixels:
// sign-weighted, sigma-free sums (sign * alpha * v and the same times d, by colour),
// and the factors (1 - alpha) into the product T of the record's sign.  CAP: some
// record of the call may reach the opacity cap (else alpha is not clamped).
template <int PPT, bool CAP>
__device__ __forceinline__ void bau_record(const float4 *r, float colf, const float (&rowf)[PPT], float sign,
                                           float (&dP0)[PPT][3], float (&dP1)[PPT][3], float (&dQ0)[PPT],
                                           float (&dQ1)[PPT], float (&T)[PPT])
{
    const float4 ra = r[0], rb = r[1], rc = r[2];
    const float dx = ra.x + colf;
    const float cb = exp_col_b(ra.w, dx), cc = exp_col_c(ra.z, rb.y, dx);
    const float sv = sign * rc.y;   // sign * v
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const float e = exp_pix(rb.x, ra.y + rowf[p], cb, cc);
        if (e >= kLog2AlphaMin) {
            const float ex = __builtin_amdgcn_exp2f(e);
            const float al = CAP ? fminf(ex, kAlphaMax) : ex;
            const float sav = al * sv;        // sign * alpha * v
            const float savd = sav * rc.z;    // ... * d
            dP0[p][0] = fmaf(rb.z, sav, dP0[p][0]);
            dP0[p][1] = fmaf(rb.w, sav, dP0[p][1]);
            dP0[p][2] = fmaf(rc.x, sav, dP0[p][2]);
            dP1[p][0] = fmaf(rb.z, savd, dP1[p][0]);
            dP1[p][1] = fmaf(rb.w, savd, dP1[p][1]);
            dP1[p][2] = fmaf(rc.x, savd, dP1[p][2]);
            dQ0[p] += sav;
            dQ1[p] += savd;
            T[p] = fmaf(-al, T[p], T[p]);   // T (1 - alpha)
        }
    }
}

// log T changes by ln Tp - ln Tm; the products restart at 1
template <int PPT>
__device__ __forceinline__ void fold_log_t(float (&dL)[PPT], float (&Tp)[PPT], float (&Tm)[PPT])
{
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        dL[p] += (__builtin_amdgcn_logf(Tp[p]) - __builtin_amdgcn_logf(Tm[p])) * kLn2;
        Tp[p] = Tm[p] = 1.f;
    }
}

// Blend one active record into a thread's PPT pixels (BAN accumulators, and Qs =
// dQ/dsigma, which the backward pass uses to take dL/dsigma in a form that the float
// rounding of F does not disturb).  Only the pixels p whose bit is set in the
// wave-uniform strip mask sp are evaluated (the record's footprint box misses the
// others).  CAP: some record of the call may reach the opacity cap; otherwise every
// alpha stays below it (e <= lo < log2 of the cap) and is not clamped.
template <int PPT, bool CAP>
__device__ __forceinline__ void blend_active(const float4 &ra, const float4 &rb, const float4 &rc, float cb,
                                             float cc, const float (&rowf)[PPT], const uint64_t (&inmask)[PPT],
                                             uint32_t sp, unsigned long long &npair, float (&P)[PPT][3],
                                             float (&Q)[PPT], float (&Qs)[PPT], float (&T)[PPT])
{
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        if (!((sp >> p) & 1u)) continue;
        const float e = exp_pix(rb.x, ra.y + rowf[p], cb, cc);
        const bool hit = e >= kLog2AlphaMin;
        npair += (unsigned long long)__builtin_popcountll(__ballot(hit) & inmask[p]);
        if (hit) {
            const float ex = __builtin_amdgcn_exp2f(e);
            const float al = CAP ? fminf(ex, kAlphaMax) : ex;
            const float aw = al * rc.y;
            P[p][0] = fmaf(rb.z, aw, P[p][0]);
            P[p][1] = fmaf(rb.w, aw, P[p][1]);
            P[p][2] = fmaf(rc.x, aw, P[p][2]);
            Q[p] += aw;
            Qs[p] = fmaf(al, rc.z, Qs[p]);
            T[p] = fmaf(-al, T[p], T[p]);   // T (1 - alpha)
        }
    }
}

// One tile, by the whole workgroup.  PRE (a pre-rendered buffer is given): the label
// changes (BAU, when the call lists them) are first blended into the pre-rendered
// buffer (each pixel's sign-weighted deltas are added to its stored accumulators, in
// passes over half of a thread's pixels at tile 32), then every pixel reads the
// inactive set's terms from it and blends the active entries on top (BAN), and the
// image and the pixel state are written.  Without PRE the active entries are the whole
// set.
// The forward's LDS: staged records (the active entries BATCH per block, the label
// changes 64 per wave), their strip masks, the waves' pair counts and the ticket.  One
// instance per workgroup, whichever variant of the tile loop runs.
template <int S, int BATCH, bool BAU>
struct FwdShared {
    static constexpr int NT = S * S < 256 ? S * S : 256;
    static constexpr int NW = NT / 64;
    static constexpr int kStage = BAU && NW * 64 > BATCH ? NW * 64 : BATCH;
    float4 rec[kStage * 3];
    int mask[BATCH];
    unsigned long long cnt[NW > 0 ? NW : 1];
    uint32_t ticket;
};

template <int S, int BATCH, bool PRE, bool BAU, bool CAP>
__device__ __forceinline__ void fwd_tile(const FwdArgs &a, uint32_t ticket, int tid, FwdShared<S, BATCH, BAU> &sh)
{
    static_assert(PRE || !BAU, "label changes go into a pre-rendered buffer");
    constexpr int NT = S * S < 256 ? S * S : 256;
    constexpr int PPT = S * S / NT;
    constexpr int BW = S == 32 ? 16 : 8;   // edge of a wave's pixel block
    constexpr int WPR = S / BW;            // blocks per tile row
    constexpr int NW = NT / 64;            // waves (= blocks)
    constexpr int RSTEP = 64 / BW;         // rows between one thread's pixels
    static_assert(NW == WPR * WPR && PPT * RSTEP == BW, "wave blocks must tile the tile");
    float4 *const s_rec = sh.rec;
    int *const s_mask = sh.mask;

    int v, tx, ty;
    fwd_tile_at(a.b, ticket, v, tx, ty);
    const CamDev &cam = a.b.cams[v];
    const int tile = cam.tile_base + ty * cam.tiles_x + tx;
    const float x0 = (float)(tx * S) + 0.5f, y0 = (float)(ty * S) + 0.5f;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int col = (wave % WPR) * BW + lane % BW, row0 = (wave / WPR) * BW + lane / BW;
    const float colf = (float)col;
    const bool col_in = tx * S + col < cam.W;
    const size_t HW = (size_t)cam.W * cam.H;
    const size_t pb = (size_t)cam.pix_base;

    float rowf[PPT];
    bool in[PPT];
    uint64_t inmask[PPT];   // lanes whose pixel p lies in the image
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int row = row0 + p * RSTEP;
        rowf[p] = (float)row;
        in[p] = col_in && ty * S + row < cam.H;
        inmask[p] = __ballot(in[p]);
    }

    const uint64_t cap = (uint64_t)a.b.pair_cap;
    const uint64_t off = a.b.tile_off[tile];
    uint64_t na = a.b.cnt_a[tile], nd = a.b.cnt_d[tile];
    if (off + na > cap) na = off < cap ? cap - off : 0;
    if (off + na + nd > cap) nd = off + na < cap ? cap - off - na : 0;
    const Rec *recv = a.b.rec + (size_t)v * a.b.Rcap;

    const float sigma = *a.sigma;
    const float isig = 1.f / sigma;
    // The pixel's composite sums P, Q, T and dQ/dsigma.  With a pre-rendered buffer they
    // start from the inactive set's terms -- P0 - P1 / sigma + Q / 2 (the colour sums are
    // stored centred on the colour offset), Q0 - Q1 / sigma, exp(log T), Q1 / sigma^2 --
    // read before the active entries (with BAU once the label changes are added), and
    // the active entries are blended on top: no register holds the inactive terms apart.
    float P[PPT][3], Q[PPT], T[PPT], Qs[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        P[p][0] = P[p][1] = P[p][2] = 0.f;
        Q[p] = 0.f;
        T[p] = 1.f;
        Qs[p] = 0.f;
    }
    auto take_pre = [&](int p, const float (&pv)[9]) {
        Q[p] = pv[6] - pv[7] * isig;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) P[p][ch] = fmaf(kColorOffset, Q[p], pv[ch] - pv[3 + ch] * isig);
        T[p] = expf(pv[8]);
        Qs[p] = pv[7] * (isig * isig);
    };
    // label changes: BAU accumulators (sign-weighted, sigma-free), added to the
    // pre-rendered buffer.  A thread's PPT pixels are taken NPASS at a time in passes
    // over the tile's label changes (two passes of two pixels at tile 32): eleven
    // accumulators per pixel for all four would not fit the registers of six waves per
    // SIMD.  Pass h covers rows [h BW / NPASS, (h + 1) BW / NPASS) of the wave's block,
    // and a record that misses those rows is skipped in that pass.
    if (BAU && nd > 0) {
        constexpr int NPASS = PPT >= 4 ? 2 : 1;
        constexpr int PB = PPT / NPASS;
        // log T changes by sum sign * ln(1 - alpha): the factors of each sign are
        // multiplied (Tp: +1, Tm: -1) and folded into dL every kFold records, before
        // a product of factors >= 1 - kAlphaMax can underflow
        constexpr int kFold = 16;
        // Each wave stages the tile's label changes itself, 64 at a time (one per lane),
        // in its own LDS slice, and keeps those that reach its pixels: the waves of a
        // tile never wait for one another, and a wave whose pixels the changes miss
        // ends early.
        // The loads are pipelined: a batch's entry indices are read two batches ahead and
        // its records one batch ahead, so both latencies overlap the work on a batch.
        float4 *wrec = s_rec + wave * 64 * 3;
        const uint32_t *ent = a.b.entries + off + na;
        auto rec_of_entry = [&](uint32_t ri) { return (ri >= a.b.Acap && ri < a.b.Rcap) ? recv[ri] : kNoRec; };
        // the colours of label changes enter the stored sums centred on the colour
        // offset (c - 1/2): those sums then carry both signs, and their float rounding
        // stays small against the differences that dL/dsigma takes of them
        auto rec_of_entry_c = [&](uint32_t ri) {
            Rec r = rec_of_entry(ri);
            r.b.z -= kColorOffset;
            r.b.w -= kColorOffset;
            r.c.x -= kColorOffset;
            return r;
        };
        const int bx = (wave % WPR) * BW, by = (wave / WPR) * BW;
        // unrolled: the passes index the pixel arrays with compile-time indices
#pragma unroll
        for (int h = 0; h < NPASS; ++h) {
            float rows[PB];
#pragma unroll
            for (int j = 0; j < PB; ++j) rows[j] = rowf[h * PB + j];
            float dP0[PB][3], dP1[PB][3], dQ0[PB], dQ1[PB], dL[PB], Tp[PB], Tm[PB];
#pragma unroll
            for (int p = 0; p < PB; ++p) {
                dP0[p][0] = dP0[p][1] = dP0[p][2] = 0.f;
                dP1[p][0] = dP1[p][1] = dP1[p][2] = 0.f;
                dQ0[p] = dQ1[p] = dL[p] = 0.f;
                Tp[p] = Tm[p] = 1.f;
            }
            int since_fold = 0;
            // a tile's label changes that fit one batch stay staged for the second pass
            const bool stage = h == 0 || nd > 64;
            Rec cur = kNoRec;
            uint32_t ri_next = 0xffffffffu;
            if (stage) {
                if (lane < nd) cur = rec_of_entry_c(ent[lane]);
                if (64 + lane < nd) ri_next = ent[64 + lane];
            }
            for (uint64_t base = 0; base < nd; base += 64) {
                const int cnt = (int)(nd - base < 64 ? nd - base : 64);
                if (stage) {
                    if (lane < cnt) {
                        wrec[3 * lane] = make_float4(x0 - cur.a.x, y0 - cur.a.y, cur.a.z, cur.a.w);
                        wrec[3 * lane + 1] = cur.b;
                        wrec[3 * lane + 2] = cur.c;
                    }
                    __builtin_amdgcn_wave_barrier();
                    // next batch's records (their indices are here), the batch after's indices
                    cur = kNoRec;
                    if (base + 64 + lane < nd) cur = rec_of_entry_c(ri_next);
                    ri_next = 0xffffffffu;
                    if (base + 128 + lane < nd) ri_next = ent[base + 128 + lane];
                }
                bool mine = false, minus = false;
                if (lane < cnt) {
                    const float4 s0 = wrec[3 * lane], s1 = wrec[3 * lane + 1];
                    mine = staged_hits_rect(s0, s1, bx, by + h * (BW / NPASS), BW, BW / NPASS);
                    // sign -1: the record leaves the pre-rendered set's complement
                    minus = wrec[3 * lane + 2].w < 0.f;
                }
                uint64_t todo_p = __ballot(mine && !minus), todo_m = __ballot(mine && minus);
                // sign +1: the factors (1 - alpha) go to Tp; sign -1: to Tm and v enters negated
                while (todo_p) {
                    const int j = (int)__builtin_ctzll(todo_p);
                    todo_p &= todo_p - 1;
                    bau_record<PB, CAP>(wrec + 3 * j, colf, rows, 1.f, dP0, dP1, dQ0, dQ1, Tp);
                    if (++since_fold == kFold) {
                        since_fold = 0;
                        fold_log_t<PB>(dL, Tp, Tm);
                    }
                }
                while (todo_m) {
                    const int j = (int)__builtin_ctzll(todo_m);
                    todo_m &= todo_m - 1;
                    bau_record<PB, CAP>(wrec + 3 * j, colf, rows, -1.f, dP0, dP1, dQ0, dQ1, Tm);
                    if (++since_fold == kFold) {
                        since_fold = 0;
                        fold_log_t<PB>(dL, Tp, Tm);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
            fold_log_t<PB>(dL, Tp, Tm);
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const int p = h * PB + j;
                if (!in[p]) continue;
                const size_t pix = (size_t)(ty * S + row0 + p * RSTEP) * cam.W + tx * S + col;
                float *pr = a.pre + 9 * pb + pix;
                const float add[9] = {dP0[j][0], dP0[j][1], dP0[j][2], dP1[j][0], dP1[j][1],
                                      dP1[j][2], dQ0[j],    dQ1[j],    dL[j]};
#pragma unroll
                for (int k = 0; k < 9; ++k) pr[k * HW] += add[k];
            }
        }
    }
    if (PRE) {
        // the inactive set's terms, read back after the label changes (this thread has
        // just written them), so that none is live during the passes (holding the last
        // pass's in registers instead spilled 12 bytes per lane)
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            if (!in[p]) continue;
            const size_t pix = (size_t)(ty * S + row0 + p * RSTEP) * cam.W + tx * S + col;
            const float *pr = a.pre + 9 * pb + pix;
            float pv[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) pv[k] = pr[k * HW];
            take_pre(p, pv);
        }
    }

    // active entries: BAN accumulators
    unsigned long long npair = 0;   // contributing in-image active pairs of this wave (counter)
    for (uint64_t base = 0; base < na; base += BATCH) {
        const int cnt = (int)(na - base < (uint64_t)BATCH ? na - base : (uint64_t)BATCH);
        __syncthreads();
        for (int j = tid; j < cnt; j += NT) {
            const uint32_t ri = a.b.entries[off + base + j];
            s_mask[j] = stage_rec<BW, WPR, NW, PPT>(&s_rec[3 * j], ri < a.b.Acap ? recv[ri] : kNoRec, x0, y0);
        }
        __syncthreads();
        for (int sb = 0; sb < cnt; sb += 64) {
          // lane k holds record sb + k's strips of this wave; todo: records reaching any
          const int m = sb + lane < cnt ? (s_mask[sb + lane] >> (wave * PPT)) & ((1 << PPT) - 1) : 0;
          uint64_t todo = __ballot(m != 0);
          while (todo) {
            const int k = (int)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t sp = (uint32_t)__builtin_amdgcn_readlane(m, k);
            const int j = sb + k;
            const float4 ra = s_rec[3 * j], rb = s_rec[3 * j + 1], rc = s_rec[3 * j + 2];
            const float dx = ra.x + colf;
            const float cb = exp_col_b(ra.w, dx), cc = exp_col_c(ra.z, rb.y, dx);
            blend_active<PPT, CAP>(ra, rb, rc, cb, cc, rowf, inmask, sp, npair, P, Q, Qs, T);
          }
        }
    }

    // throughput counters: contributing active pairs and evaluated (in-image) pairs
    {
        unsigned long long *const s_cnt = sh.cnt;
        if ((tid & 63) == 0) s_cnt[tid >> 6] = npair;
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < (NT + 63) / 64; ++w) t += s_cnt[w];
            const int inside = min(S, cam.W - tx * S) * min(S, cam.H - ty * S);
            // the tile's counts; k_pair_totals adds them (no device atomics per tile)
            a.b.tile_cnt[2 * (size_t)tile] = t;
            a.b.tile_cnt[2 * (size_t)tile + 1] = (unsigned long long)na * inside;
        }
    }

#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        if (!in[p]) continue;
        const size_t pix = (size_t)(ty * S + row0 + p * RSTEP) * cam.W + tx * S + col;
        const float Pt[3] = {P[p][0], P[p][1], P[p][2]};
        const float Qt = Q[p], Tt = T[p];
        const float iq = Qt > 0.f ? 1.f / Qt : 0.f;
        const float F0 = Pt[0] * iq, F1 = Pt[1] * iq, F2 = Pt[2] * iq;
        float *im = a.image + 3 * pb;
        im[pix] = Tt * a.bg0 + (1.f - Tt) * F0;
        im[HW + pix] = Tt * a.bg1 + (1.f - Tt) * F1;
        im[2 * HW + pix] = Tt * a.bg2 + (1.f - Tt) * F2;
        float *ps = a.pixstate + kPixStatePlanes * pb;
        ps[pix] = Tt;
        ps[HW + pix] = Qt;
        ps[2 * HW + pix] = F0;
        ps[3 * HW + pix] = F1;
        ps[4 * HW + pix] = F2;
        ps[5 * HW + pix] = Qs[p];
    }
}

// The persistent loop: tiles from the ticket until the heavy-first order is exhausted.
template <int S, int BATCH, bool PRE, bool BAU, bool CAP>
__device__ __forceinline__ void fwd_tiles(const FwdArgs &a, FwdShared<S, BATCH, BAU> &sh)
{
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = atomicAdd(&a.b.counters[CNT_FQUEUE], 1u);
        __syncthreads();
        const uint32_t ticket = sh.ticket;
        if (ticket >= (uint32_t)a.b.T) break;
        // Nothing derived from the thread index or the arguments is kept across tiles
        // (it would hold registers through the blending loops): both are taken afresh
        // for every tile, the arguments by scalar loads from their segment (k_raster_fwd
        // takes one argument, the FwdArgs, which therefore starts the segment).
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        typedef const __attribute__((address_space(4))) char *KernArg;
        KernArg ka = (KernArg)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(ka));
        fwd_tile<S, BATCH, PRE, BAU, CAP>(*(const FwdArgs *)ka, ticket, tid, sh);
        // every thread has read the ticket and is done with the LDS staging
        __syncthreads();
    }
}

// Persistent over (view, tile): as many workgroups as the device holds at once, each
// taking the next position of the heavy-first tile order from one device ticket until
// the order is exhausted (every workgroup reaches the end; k_tile_order reset the
// ticket).  The tiles of 10^2 to 10^4 entries are thus dealt longest first to whichever
// workgroup frees up, on any XCD.  At tile 32 the variant with BAU runs at seven waves
// per SIMD (72 registers; 24-28 bytes per lane go to scratch once per tile, outside the
// blending loops; held to eight waves it spills inside them) and the others at eight
// (the dense one with 8 bytes per lane of scratch, also once per tile).
template <int S, int BATCH, bool PRE, bool BAU>
__global__ __launch_bounds__(S * S < 256 ? S * S : 256)
__attribute__((amdgpu_waves_per_eu(S == 32 ? (BAU ? 7 : 8) : 1))) void k_raster_fwd(FwdArgs a)
{
    __shared__ FwdShared<S, BATCH, BAU> sh;
    // the opacity clamp is compiled in only if a record of the call can reach the cap
    if (a.b.counters[CNT_CAP])
        fwd_tiles<S, BATCH, PRE, BAU, true>(a, sh);
    else
        fwd_tiles<S, BATCH, PRE, BAU, false>(a, sh);
}

template <typename K>
static void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, const KTimer *t, const FwdArgs &a)
{
    if (t)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t->start, t->stop, 0, a);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, a);
}

// Workgroups of a persistent launch: as many as the current device runs at once (its
// CUs times the kernel's resident workgroups per CU), at most one per work item.
template <typename K>
static unsigned persistent_grid(K kernel, int threads, unsigned items)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || cus <= 0 || per_cu <= 0)
        return items;   // one workgroup per item is always enough
    const unsigned n = (unsigned)cus * (unsigned)per_cu;
    return n < items ? n : items;
}

template <int S, int BATCH, bool PRE, bool BAU>
static void raster_fwd_launch(const FwdArgs &a, hipStream_t s, const KTimer *t)
{
    constexpr int NT = S * S < 256 ? S * S : 256;
    const auto kernel = k_raster_fwd<S, BATCH, PRE, BAU>;
    launch_timed(kernel, dim3(persistent_grid(kernel, NT, (unsigned)a.b.T)), dim3(NT), s, t, a);
}

template <int S, bool PRE, bool BAU>
static bool raster_fwd_s(const FwdArgs &a, int batch, hipStream_t s, const KTimer *t)
{
    switch (batch) {
    case 32: raster_fwd_launch<S, 32, PRE, BAU>(a, s, t); return true;
    case 64: raster_fwd_launch<S, 64, PRE, BAU>(a, s, t); return true;
    case 128: raster_fwd_launch<S, 128, PRE, BAU>(a, s, t); return true;
    case 256: raster_fwd_launch<S, 256, PRE, BAU>(a, s, t); return true;
    default: return false;
    }
}

// Throughput counters of the active pass: the per-tile counts summed by one block.
__global__ __launch_bounds__(1024) void k_pair_totals(Buffers b)
{
    __shared__ unsigned long long s_p[1024], s_e[1024];
    unsigned long long p = 0, e = 0;
    for (int t = threadIdx.x; t < b.T; t += 1024) {
        p += b.tile_cnt[2 * (size_t)t];
        e += b.tile_cnt[2 * (size_t)t + 1];
    }
    s_p[threadIdx.x] = p;
    s_e[threadIdx.x] = e;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_p[threadIdx.x] += s_p[threadIdx.x + off];
            s_e[threadIdx.x] += s_e[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *(unsigned long long *)(b.counters + CNT_PAIRS) = s_p[0];
        *(unsigned long long *)(b.counters + CNT_EVAL) = s_e[0];
    }
}

template <int S>
static bool raster_fwd_both(const FwdArgs &a, bool deltas, int batch, hipStream_t s, const KTimer *fwd_t)
{
    const bool ok = !a.pre   ? raster_fwd_s<S, false, false>(a, batch, s, fwd_t)
                    : deltas ? raster_fwd_s<S, true, true>(a, batch, s, fwd_t)
                             : raster_fwd_s<S, true, false>(a, batch, s, fwd_t);
    if (!ok) return false;
    hipLaunchKernelGGL(k_pair_totals, dim3(1), dim3(1024), 0, s, a.b);
    return true;
}

bool launch_raster_fwd(const Buffers &b, const float *sigma, const float bg[3], float *pre, bool deltas,
                       float *image, float *pixstate, int batch, hipStream_t s, const KTimer *fwd_t)
{
    FwdArgs a{b, sigma, bg[0], bg[1], bg[2], pre, image, pixstate};
    if (b.T == 0) return true;
    switch (b.tile) {
    case 8: return raster_fwd_both<8>(a, deltas, batch, s, fwd_t);
    case 16: return raster_fwd_both<16>(a, deltas, batch, s, fwd_t);
    case 32: return raster_fwd_both<32>(a, deltas, batch, s, fwd_t);
    default: return false;
    }
}

}  // namespace oit
