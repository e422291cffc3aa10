// C ABI of liboit: argument validation on the host, the workspace plan and the
// launch sequence of each entry point.  No allocation, no synchronisation (except
// oit_read_status, which exists to synchronise).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "oit_density.h"
#include "oit_internal.h"

using namespace oit;

namespace {

thread_local char g_err[512] = "";

// optional timing (see oit_timing_enable): start/stop events of the forward and of the
// backward raster kernel (0-3), then events at the stage boundaries of the forward
// (4-7: before the preprocess, after it, after the binning, after the raster stage) and
// of the backward (8-11: before the pixel constants, after them, after the raster
// stage, after the preprocess backward)
constexpr int kTimingEvents = 12;
hipEvent_t g_ev[kTimingEvents];
bool g_timing_ready = false;
bool g_timing_on = false;


oit_status fail(oit_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

oit_status ok()
{
    g_err[0] = 0;
    return OIT_OK;
}

// Timing is for eager launches: refuse a capturing stream while it is on.
oit_status timing_guard(hipStream_t s, const char *what)
{
    if (!g_timing_on) return OIT_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return fail(OIT_ERR_INVALID, "%s: kernel timing is on while the stream is being captured", what);
    return OIT_OK;
}

oit_status check_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OIT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

struct Plan {
    size_t status, cams, counters, tiles, tile_off, chunk_off, chunk_tile, tile_order, entries, orig, keys0, keys1, vals0,
        vals1, recs0, recs1, hist, hist_off, rec, rect, nhits, hoff, scan_tmp, ep, pixconst, pixB, sig_part, loss_part,
        tile_cnt, total;
    uint32_t max_chunks;
    int T;
    int64_t total_px, Acap, Rcap;
    CamDev cams_host[kMaxViews];
};

oit_status check_cams(const oit_camera *cams, int32_t n_views)
{
    if (!cams) return fail(OIT_ERR_INVALID, "cams is NULL");
    if (n_views < 1 || n_views > OIT_MAX_VIEWS)
        return fail(OIT_ERR_INVALID, "n_views = %d outside [1, %d]", n_views, OIT_MAX_VIEWS);
    for (int v = 0; v < n_views; ++v) {
        const oit_camera &c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 32768 || c.height > 32768)
            return fail(OIT_ERR_INVALID, "camera %d: bad size %dx%d", v, c.width, c.height);
        if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
            return fail(OIT_ERR_INVALID, "camera %d: bad intrinsics", v);
        for (int k = 0; k < 9; ++k)
            if (!std::isfinite(c.R[k])) return fail(OIT_ERR_INVALID, "camera %d: non-finite R", v);
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(c.t[k])) return fail(OIT_ERR_INVALID, "camera %d: non-finite t", v);
        if (!(c.near_z > 0.f)) return fail(OIT_ERR_INVALID, "camera %d: near_z must be > 0", v);
    }
    return OIT_OK;
}

oit_status check_tuning(const oit_tuning *tu)
{
    if (!tu) return fail(OIT_ERR_INVALID, "tuning is NULL");
    if (tu->tile != 8 && tu->tile != 16 && tu->tile != 32)
        return fail(OIT_ERR_INVALID, "tuning.tile = %d not in {8, 16, 32}", tu->tile);
    if (tu->batch != 32 && tu->batch != 64 && tu->batch != 128 && tu->batch != 256)
        return fail(OIT_ERR_INVALID, "tuning.batch = %d not in {32, 64, 128, 256}", tu->batch);
    if (tu->bwd_mode != OIT_BWD_PER_SPLAT && tu->bwd_mode != OIT_BWD_PER_PIXEL)
        return fail(OIT_ERR_INVALID, "tuning.bwd_mode = %d unknown", tu->bwd_mode);
    if (tu->pair_capacity <= 0 || tu->pair_capacity >= 0xffffffffLL)
        return fail(OIT_ERR_INVALID, "tuning.pair_capacity = %lld outside [1, 2^32 - 1)",
                    (long long)tu->pair_capacity);
    return OIT_OK;
}

oit_status check_cap(const oit_capacity *cap)
{
    if (!cap) return fail(OIT_ERR_INVALID, "capacity is NULL");
    if (cap->n <= 0 || cap->n > 0x7fffffffLL) return fail(OIT_ERR_INVALID, "n = %lld outside [1, 2^31)", (long long)cap->n);
    if (cap->active_capacity <= 0 || cap->active_capacity > cap->n)
        return fail(OIT_ERR_INVALID, "active_capacity = %lld outside [1, n]", (long long)cap->active_capacity);
    if (cap->delta_capacity < 0 || cap->delta_capacity > cap->n)
        return fail(OIT_ERR_INVALID, "delta_capacity = %lld outside [0, n]", (long long)cap->delta_capacity);
    return OIT_OK;
}

oit_status make_plan(const oit_capacity *cap, const oit_camera *cams, int32_t n_views, const oit_tuning *tu,
                     Plan &p)
{
    oit_status st;
    if ((st = check_cap(cap)) != OIT_OK) return st;
    if ((st = check_cams(cams, n_views)) != OIT_OK) return st;
    if ((st = check_tuning(tu)) != OIT_OK) return st;
    const int S = tu->tile;
    int64_t tiles = 0, px = 0;
    for (int v = 0; v < n_views; ++v) {
        const oit_camera &c = cams[v];
        CamDev &d = p.cams_host[v];
        memset(&d, 0, sizeof(d));
        for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
        for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
        d.fx = c.fx;
        d.fy = c.fy;
        d.cx = c.cx;
        d.cy = c.cy;
        d.near_z = c.near_z;
        d.lim_x = kGuardBand * (0.5f * (float)c.width / c.fx);
        d.lim_y = kGuardBand * (0.5f * (float)c.height / c.fy);
        for (int r = 0; r < 3; ++r)
            d.cc[r] = (float)(-((double)c.R[r] * c.t[0] + (double)c.R[3 + r] * c.t[1] + (double)c.R[6 + r] * c.t[2]));
        d.W = c.width;
        d.H = c.height;
        d.tiles_x = (c.width + S - 1) / S;
        d.tiles_y = (c.height + S - 1) / S;
        d.tile_base = (int)tiles;
        d.pix_base = (int)px;
        tiles += (int64_t)d.tiles_x * d.tiles_y;
        px += (int64_t)c.width * c.height;
        if (tiles > (0xffffffffLL >> (kSizeBits + 1)) || px > 0x7fffffffLL / 9)
            return fail(OIT_ERR_INVALID, "batch too large: %lld tiles, %lld pixels", (long long)tiles, (long long)px);
    }
    p.T = (int)tiles;
    p.total_px = px;
    p.Acap = cap->active_capacity;
    p.Rcap = cap->active_capacity + cap->delta_capacity;
    size_t o = 0;
    // head shared with oit_l1_loss's layout: status word, camera table, loss shares
    p.status = o; o = align256(o + 4);
    p.cams = o; o = align256(o + sizeof(CamDev) * kMaxViews);
    p.loss_part = o; o = align256(o + 8 * (size_t)kSigPixParts);
    p.counters = o; o = align256(o + 4 * CNT_SLOTS);
    p.tiles = o; o = align256(o + 4 * 2 * (size_t)p.T);
    p.tile_off = o; o = align256(o + 4 * ((size_t)p.T + 1));
    p.chunk_off = o; o = align256(o + 4 * ((size_t)p.T + 1));
    p.tile_order = o; o = align256(o + 4 * (size_t)p.T);
    // every tile adds at most one partial chunk to the pair capacity's full ones
    const uint64_t mc = (uint64_t)tu->pair_capacity / kBwdLanes + (uint64_t)p.T + 1;
    p.max_chunks = (uint32_t)(mc < 0xffffffffull ? mc : 0xffffffffull);
    p.chunk_tile = o; o = align256(o + 4 * (size_t)p.max_chunks);
    const size_t pc = (size_t)tu->pair_capacity;
    p.entries = o; o = align256(o + 4 * pc);
    p.orig = o; o = align256(o + 4 * pc);
    p.keys0 = o; o = align256(o + 4 * pc);
    p.keys1 = o; o = align256(o + 4 * pc);
    p.vals0 = o; o = align256(o + 4 * pc);
    p.vals1 = o; o = align256(o + 4 * pc);
    p.recs0 = o; o = align256(o + 4 * pc);
    p.recs1 = o; o = align256(o + 4 * pc);
    p.hist = o; o = align256(o + 4 * kRadixBuckets * (size_t)kSortGrid);
    p.hist_off = o; o = align256(o + 4 * kRadixBuckets * (size_t)kSortGrid);
    p.rec = o; o = align256(o + sizeof(Rec) * (size_t)n_views * p.Rcap);
    p.rect = o; o = align256(o + sizeof(short4) * (size_t)n_views * p.Rcap);
    const size_t npairs = (size_t)n_views * p.Rcap;
    p.nhits = o; o = align256(o + 4 * npairs);
    p.hoff = o; o = align256(o + 4 * npairs);
    // block sums of the scans: the host-sized scan of the radix histograms, and the
    // device-count scan of the pairs' tile counts, which always uses kScanThreads blocks
    const size_t nscan = npairs > kRadixBuckets * (size_t)kSortGrid ? npairs : kRadixBuckets * (size_t)kSortGrid;
    const size_t nsums = nscan / kScanBlockItems + 2 > (size_t)kScanThreads ? nscan / kScanBlockItems + 2
                                                                             : (size_t)kScanThreads;
    p.scan_tmp = o; o = align256(o + 4 * nsums);
    p.ep = o; o = align256(o + 4 * kEpStride * pc);
    p.pixconst = o; o = align256(o + 16 * (size_t)p.total_px);
    p.pixB = o; o = align256(o + 8 * (size_t)p.total_px);
    p.sig_part = o; o = align256(o + 8 * (size_t)(kSigPixParts + kSigPreParts));
    p.tile_cnt = o; o = align256(o + 16 * (size_t)p.T);
    p.total = o;
    return OIT_OK;
}

Buffers buffers(const Plan &p, void *ws, int n_views, const oit_tuning *tu)
{
    char *w = (char *)ws;
    Buffers b;
    b.status = (int32_t *)(w + p.status);
    b.cams = (CamDev *)(w + p.cams);
    b.counters = (uint32_t *)(w + p.counters);
    b.cnt_a = (uint32_t *)(w + p.tiles);
    b.cnt_d = b.cnt_a + p.T;
    b.tile_off = (uint32_t *)(w + p.tile_off);
    b.chunk_off = (uint32_t *)(w + p.chunk_off);
    b.chunk_tile = (uint32_t *)(w + p.chunk_tile);
    b.tile_order = (uint32_t *)(w + p.tile_order);
    b.max_chunks = p.max_chunks;
    b.entries = (uint32_t *)(w + p.entries);
    b.orig = (uint32_t *)(w + p.orig);
    b.keys[0] = (uint32_t *)(w + p.keys0);
    b.keys[1] = (uint32_t *)(w + p.keys1);
    b.vals[0] = (uint32_t *)(w + p.vals0);
    b.vals[1] = (uint32_t *)(w + p.vals1);
    b.recs[0] = (uint32_t *)(w + p.recs0);
    b.recs[1] = (uint32_t *)(w + p.recs1);
    b.hist = (uint32_t *)(w + p.hist);
    b.hist_off = (uint32_t *)(w + p.hist_off);
    b.rec = (Rec *)(w + p.rec);
    b.rect = (short4 *)(w + p.rect);
    b.nhits = (uint32_t *)(w + p.nhits);
    b.hoff = (uint32_t *)(w + p.hoff);
    b.scan_tmp = (uint32_t *)(w + p.scan_tmp);
    b.ep = (float *)(w + p.ep);
    b.pixconst = (float4 *)(w + p.pixconst);
    b.pixB = (float2 *)(w + p.pixB);
    b.sig_part = (double *)(w + p.sig_part);
    b.loss_part = (double *)(w + p.loss_part);
    b.tile_cnt = (unsigned long long *)(w + p.tile_cnt);
    b.n_views = n_views;
    b.T = p.T;
    b.tile = tu->tile;
    b.bwd_mode = tu->bwd_mode;
    b.total_px = p.total_px;
    b.pair_cap = tu->pair_capacity;
    b.Acap = p.Acap;
    b.Rcap = p.Rcap;
    return b;
}

oit_status check_splats(const oit_splats *s, const oit_capacity *cap)
{
    if (!s) return fail(OIT_ERR_INVALID, "splats is NULL");
    if (s->n != cap->n) return fail(OIT_ERR_INVALID, "splats.n = %lld differs from capacity.n = %lld",
                                    (long long)s->n, (long long)cap->n);
    const void *ptrs[6] = {s->mean, s->log_scale, s->quat, s->opacity_logit, s->sh, s->vsh};
    const char *names[6] = {"mean", "log_scale", "quat", "opacity_logit", "sh", "vsh"};
    for (int k = 0; k < 6; ++k) {
        if (!ptrs[k]) return fail(OIT_ERR_INVALID, "splats.%s is NULL", names[k]);
        const size_t al = (k == 2 || k >= 4) ? 16 : 4;   // quat, sh and vsh rows are read as float4
        if (!aligned(ptrs[k], al))
            return fail(OIT_ERR_INVALID, "splats.%s is not %zu-byte aligned", names[k], al);
    }
    return OIT_OK;
}

oit_status check_rows(const oit_capacity *cap, const int32_t *active_idx, const int32_t *n_active,
                      const int32_t *delta_idx, const int8_t *delta_sign, const int32_t *n_delta, const void *pre)
{
    if (!active_idx) {
        if (n_active || delta_idx || delta_sign || n_delta)
            return fail(OIT_ERR_INVALID, "dense mode (active_idx NULL) takes no n_active or label changes");
        if (cap->active_capacity != cap->n)
            return fail(OIT_ERR_INVALID, "dense mode needs active_capacity == n");
        return OIT_OK;
    }
    if (!n_active) return fail(OIT_ERR_INVALID, "active_idx given without n_active");
    const bool any = delta_idx || delta_sign || n_delta;
    const bool all = delta_idx && delta_sign && n_delta;
    if (any && !all) return fail(OIT_ERR_INVALID, "delta_idx, delta_sign and n_delta go together");
    if (all && !pre) return fail(OIT_ERR_INVALID, "label changes need the pre-rendered buffer");
    if (all && cap->delta_capacity <= 0) return fail(OIT_ERR_INVALID, "label changes need delta_capacity > 0");
    return OIT_OK;
}

RowList rows(const oit_capacity *cap, const int32_t *active_idx, const int32_t *n_active, const int32_t *delta_idx,
             const int8_t *delta_sign, const int32_t *n_delta, const Plan &p)
{
    RowList r;
    r.active_idx = active_idx;
    r.n_active = n_active;
    r.n_active_host = active_idx ? 0 : cap->n;
    r.delta_idx = delta_idx;
    r.delta_sign = delta_sign;
    r.n_delta = n_delta;
    r.Acap = p.Acap;
    r.Rcap = p.Rcap;
    return r;
}

SplatPtrs splat_ptrs(const oit_splats *s)
{
    return SplatPtrs{s->mean, s->log_scale, s->quat, s->opacity_logit, s->sh, s->vsh, s->n};
}

// Layout of the selection workspace; sizes as in oit_select_workspace_bytes.
SelectBuffers select_buffers(void *ws, int64_t n)
{
    const int64_t nblk = (n + 1023) / 1024;
    char *w = (char *)ws;
    size_t o = 0;
    SelectBuffers sb;
    sb.status = (int32_t *)(w + o);
    o = align256(o + 4);
    sb.state = (uint32_t *)(w + o);
    o = align256(o + 4 * 8);
    sb.hist = (uint32_t *)(w + o);
    o = align256(o + 4 * 2048);
    sb.blk_a = (uint32_t *)(w + o);
    sb.blk_b = sb.blk_a + (nblk + 1);
    sb.blk_c = sb.blk_b + (nblk + 1);
    o = align256(o + 4 * 3 * (size_t)(nblk + 1));
    sb.flags = (uint8_t *)(w + o);
    sb.nblk = nblk;
    return sb;
}

// The L1 loss's plan: the cameras' table and pixel bases of a render plan; it touches
// only the head of the layout (status word, camera table, loss shares), at the same
// offsets as every render plan, so a render workspace can be passed to it between the
// forward and the backward pass.
constexpr oit_tuning kL1Tuning{16, 64, 1, OIT_BWD_PER_SPLAT, 0};

oit_status l1_plan(const oit_camera *cams, int32_t n_views, Plan &p)
{
    const oit_capacity cap{1, 1, 0};
    return make_plan(&cap, cams, n_views, &kL1Tuning, p);
}

}  // namespace

namespace {
constexpr size_t align256c(size_t x) { return (x + 255) & ~(size_t)255; }

// bytes of the selection workspace for n splats (the layout of select_buffers)
constexpr size_t select_bytes(int64_t n)
{
    return align256c(align256c(align256c(align256c(align256c(4) + 4 * 8) + 4 * 2048) +
                               4 * 3 * (size_t)((n + 1023) / 1024 + 1)) +
                     (size_t)n);
}

// The no-allocation selection's scratch: one file-scope array per device, held until
// the process ends.  Host code never uses its name as an address: the device address
// of each GPU's copy comes from hipGetSymbolAddress, once per device.
constexpr int64_t kNoAllocMaxN = OIT_NOALLOC_SELECT_MAX_N;
constexpr size_t kNoAllocBytes = select_bytes(kNoAllocMaxN);
constexpr int kMaxDevices = 64;
__device__ __align__(256) uint8_t scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array (resolved on the first call)
oit_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(OIT_ERR_HIP, "no-allocation selection: current device %d unusable", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(OIT_ERR_HIP, "no-allocation selection: scratch address on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return OIT_OK;
}
}  // namespace

extern "C" {

size_t oit_l1_loss_workspace_bytes(void)
{
    // the head of every render layout: status word, camera table, the loss's block shares
    return align256(align256(align256(4) + sizeof(CamDev) * kMaxViews) + 8 * (size_t)kSigPixParts);
}

size_t oit_workspace_bytes(const oit_capacity *cap, const oit_camera *cams, int32_t n_views,
                           const oit_tuning *tuning)
{
    Plan p;
    if (make_plan(cap, cams, n_views, tuning, p) != OIT_OK) return 0;
    return p.total;
}

oit_status oit_render_fwd(const oit_splats *splats, const float *sigma, const float *bg, const oit_camera *cams,
                          int32_t n_views, const oit_capacity *cap, const int32_t *active_idx,
                          const int32_t *n_active, const int32_t *delta_idx, const int8_t *delta_sign,
                          const int32_t *n_delta, const oit_splats *delta_splats, float *pre, float *image,
                          float *pixstate, void *ws, size_t ws_bytes, const oit_tuning *tuning, oit_stream stream)
{
    Plan p;
    oit_status st;
    if ((st = make_plan(cap, cams, n_views, tuning, p)) != OIT_OK) return st;
    if ((st = check_splats(splats, cap)) != OIT_OK) return st;
    if (delta_splats && (st = check_splats(delta_splats, cap)) != OIT_OK) return st;
    if ((st = check_rows(cap, active_idx, n_active, delta_idx, delta_sign, n_delta, pre)) != OIT_OK) return st;
    if (!sigma || !bg || !image || !pixstate) return fail(OIT_ERR_INVALID, "sigma, bg, image and pixstate are required");
    if (!aligned(image, 4) || !aligned(pixstate, 4) || (pre && !aligned(pre, 4)))
        return fail(OIT_ERR_INVALID, "image buffers must be 4-byte aligned");
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < p.total)
        return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p.total);
    hipStream_t s = (hipStream_t)stream;
    if ((st = timing_guard(s, "oit_render_fwd")) != OIT_OK) return st;
    const Buffers b = buffers(p, ws, n_views, tuning);
    const RowList rl = rows(cap, active_idx, n_active, delta_idx, delta_sign, n_delta, p);
    upload_cams(p.cams_host, n_views, b.cams, s);
    fill_u32(b.counters + CNT_PAIRS, CNT_CAP + 1 - CNT_PAIRS, 0u, s);   // pair and cap counters
    auto mark = [&](int k) {
        if (g_timing_on) (void)hipEventRecord(g_ev[k], s);
    };
    mark(4);
    launch_preprocess_count(splat_ptrs(splats), splat_ptrs(delta_splats ? delta_splats : splats), sigma, rl, b, s);
    mark(5);
    launch_binning(rl, b, s);
    mark(6);
    const KTimer fwd_t{g_ev[0], g_ev[1]};
    if (!launch_raster_fwd(b, sigma, bg, pre, delta_idx != nullptr, image, pixstate, tuning->batch, s,
                           g_timing_on ? &fwd_t : nullptr))
        return fail(OIT_ERR_INVALID, "no forward kernel for tile %d batch %d", tuning->tile, tuning->batch);
    mark(7);
    return check_launch("oit_render_fwd");
}

oit_status oit_l1_loss(const float *image, const float *target, const oit_camera *cams, int32_t n_views,
                       float *grad_image, double *loss, void *ws, size_t ws_bytes, oit_stream stream)
{
    oit_status st;
    if ((st = check_cams(cams, n_views)) != OIT_OK) return st;
    if (!image || !target || !grad_image || !loss) return fail(OIT_ERR_INVALID, "oit_l1_loss: NULL buffer");
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    const size_t need = oit_l1_loss_workspace_bytes();
    if (ws_bytes < need) return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    Plan p;
    if ((st = l1_plan(cams, n_views, p)) != OIT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Buffers b = buffers(p, ws, n_views, &kL1Tuning);
    upload_cams(p.cams_host, n_views, b.cams, s);
    launch_l1_loss(b, image, target, grad_image, loss, s);
    return check_launch("oit_l1_loss");
}

namespace {
struct LossPlan {
    size_t cams, acc, parts, maps, total;
    int64_t total_px;
    int tiles16;
};

oit_status loss_plan(const oit_camera *cams, int32_t n_views, LossPlan &lp, Plan &p)
{
    oit_capacity cap{1, 1, 0};
    oit_tuning tu{16, 64, 1, OIT_BWD_PER_SPLAT, 0};
    oit_status st = make_plan(&cap, cams, n_views, &tu, p);
    if (st != OIT_OK) return st;
    lp.total_px = p.total_px;
    lp.tiles16 = p.T;
    size_t o = align256(4);
    lp.cams = o;
    o = align256(o + sizeof(CamDev) * kMaxViews);
    lp.acc = o;
    o = align256(o + 2 * sizeof(double));
    lp.parts = o;   // per-block shares of both sums, one block per 16 x 16 tile and channel
    o = align256(o + 2 * 3 * sizeof(double) * (size_t)p.T);
    lp.maps = o;
    o = align256(o + 9 * sizeof(float) * (size_t)p.total_px);
    lp.total = o;
    return OIT_OK;
}
}  // namespace

size_t oit_loss_workspace_bytes(const oit_camera *cams, int32_t n_views)
{
    LossPlan lp;
    Plan p;
    if (loss_plan(cams, n_views, lp, p) != OIT_OK) return 0;
    return lp.total;
}

oit_status oit_l1_dssim_loss(const float *image, const float *target, const oit_camera *cams, int32_t n_views,
                             float lambda, float *grad_image, double *loss, void *ws, size_t ws_bytes,
                             oit_stream stream)
{
    LossPlan lp;
    Plan p;
    oit_status st;
    if ((st = loss_plan(cams, n_views, lp, p)) != OIT_OK) return st;
    if (!image || !target || !grad_image || !loss) return fail(OIT_ERR_INVALID, "oit_l1_dssim_loss: NULL buffer");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(OIT_ERR_INVALID, "lambda must be in [0, 1]");
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < lp.total) return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lp.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    CamDev *dcams = (CamDev *)(w + lp.cams);
    upload_cams(p.cams_host, n_views, dcams, s);
    launch_l1_dssim(dcams, n_views, lp.total_px, lp.tiles16, image, target, lambda, grad_image, loss,
                    (float *)(w + lp.maps), (double *)(w + lp.acc), (double *)(w + lp.parts), s);
    return check_launch("oit_l1_dssim_loss");
}

oit_status oit_render_bwd(const oit_splats *splats, const float *sigma, const float *bg, const oit_camera *cams,
                          int32_t n_views, const oit_capacity *cap, const int32_t *active_idx,
                          const int32_t *n_active, const int32_t *delta_idx, const int8_t *delta_sign,
                          const int32_t *n_delta, const float *pre, const float *grad_image,
                          const float *pixstate, const oit_grads *grads, double *grad_sigma, float *score,
                          const float *eps, void *ws, size_t ws_bytes, const oit_tuning *tuning,
                          oit_stream stream)
{
    Plan p;
    oit_status st;
    if ((st = make_plan(cap, cams, n_views, tuning, p)) != OIT_OK) return st;
    if ((st = check_splats(splats, cap)) != OIT_OK) return st;
    if ((st = check_rows(cap, active_idx, n_active, delta_idx, delta_sign, n_delta, pre)) != OIT_OK) return st;
    if (!sigma || !bg || !grad_image || !pixstate || !grads || !grad_sigma)
        return fail(OIT_ERR_INVALID, "sigma, bg, grad_image, pixstate, grads and grad_sigma are required");
    const void *gp[6] = {grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->sh, grads->vsh};
    for (int k = 0; k < 6; ++k)
        if (!gp[k] || !aligned(gp[k], 4)) return fail(OIT_ERR_INVALID, "gradient buffer %d NULL or misaligned", k);
    if (grads->stride < cap->active_capacity)
        return fail(OIT_ERR_INVALID, "grads.stride = %lld < active_capacity", (long long)grads->stride);
    if (!aligned(grad_sigma, 8)) return fail(OIT_ERR_INVALID, "grad_sigma must be 8-byte aligned");
    float e6[6] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
    if (eps)
        for (int k = 0; k < 6; ++k) {
            if (!(eps[k] > 0.f)) return fail(OIT_ERR_INVALID, "eps[%d] must be > 0", k);
            e6[k] = eps[k];
        }
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < p.total)
        return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p.total);
    hipStream_t s = (hipStream_t)stream;
    if ((st = timing_guard(s, "oit_render_bwd")) != OIT_OK) return st;
    const Buffers b = buffers(p, ws, n_views, tuning);
    const RowList rl = rows(cap, active_idx, n_active, delta_idx, delta_sign, n_delta, p);
    const GradPtrs g{grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->sh, grads->vsh,
                     grads->stride};
    upload_cams(p.cams_host, n_views, b.cams, s);
    // the backward's queues and walk counters in one fill (the forward's ticket among them
    // is reset again by the next forward's ordering kernel)
    static_assert(CNT_XQUEUE + kXcds == CNT_BOX_ITEMS && CNT_WAVE_ITEMS > CNT_BOX_ITEMS, "counter slots");
    fill_u32(b.counters + CNT_XQUEUE, CNT_WAVE_ITEMS + 1 - CNT_XQUEUE, 0u, s);
    auto mark = [&](int k) {
        if (g_timing_on) (void)hipEventRecord(g_ev[k], s);
    };
    mark(8);
    launch_pixconst(b, sigma, bg, active_idx ? pre : nullptr, grad_image, pixstate, grad_sigma, s);
    mark(9);
    const KTimer bwd_t{g_ev[2], g_ev[3]};
    if (!launch_raster_bwd(b, rl, s, g_timing_on ? &bwd_t : nullptr))
        return fail(OIT_ERR_INVALID, "no backward kernel for tile %d", tuning->tile);
    mark(10);
    launch_preprocess_bwd(splat_ptrs(splats), sigma, rl, b, g, grad_sigma, score, e6, s);
    mark(11);
    return check_launch("oit_render_bwd");
}

size_t oit_select_workspace_bytes(int64_t n)
{
    if (n <= 0) return 0;
    return select_bytes(n);
}

oit_status oit_update_active_set(const float *score, int64_t n, int32_t mode, int64_t k, float thresh,
                                 uint8_t *label, int32_t *active_idx, int64_t active_capacity, int32_t *n_active,
                                 int32_t *delta_idx, int8_t *delta_sign, int64_t delta_capacity, int32_t *n_delta,
                                 void *ws, size_t ws_bytes, oit_stream stream)
{
    if (n <= 0 || n > 0x7fffffffLL) return fail(OIT_ERR_INVALID, "n = %lld outside [1, 2^31)", (long long)n);
    if (mode != OIT_SELECT_TOPK && mode != OIT_SELECT_THRESHOLD)
        return fail(OIT_ERR_INVALID, "mode = %d unknown", mode);
    if (!score || !label || !active_idx || !n_active || !delta_idx || !delta_sign || !n_delta)
        return fail(OIT_ERR_INVALID, "oit_update_active_set: NULL buffer");
    if (active_capacity <= 0 || delta_capacity <= 0)
        return fail(OIT_ERR_INVALID, "capacities must be positive");
    if (mode == OIT_SELECT_THRESHOLD && !std::isfinite(thresh))
        return fail(OIT_ERR_INVALID, "threshold must be finite");
    const size_t need = oit_select_workspace_bytes(n);
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < need) return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const SelectBuffers sb = select_buffers(ws, n);
    launch_select(score, n, mode, k, thresh, label, active_idx, active_capacity, n_active, delta_idx, delta_sign,
                  delta_capacity, n_delta, sb, (hipStream_t)stream);
    return check_launch("oit_update_active_set");
}


oit_status oit_update_active_set_noalloc(const float *score, int64_t n, int32_t mode, int64_t k, float thresh,
                                         uint8_t *label, int32_t *active_idx, int64_t active_capacity,
                                         int32_t *n_active, int32_t *delta_idx, int8_t *delta_sign,
                                         int64_t delta_capacity, int32_t *n_delta, int32_t *status,
                                         oit_stream stream)
{
    if (n <= 0 || n > kNoAllocMaxN)
        return fail(OIT_ERR_INVALID, "oit_update_active_set_noalloc: n = %lld outside [1, %lld] (its static scratch)",
                    (long long)n, (long long)kNoAllocMaxN);
    if (mode != OIT_SELECT_TOPK && mode != OIT_SELECT_THRESHOLD)
        return fail(OIT_ERR_INVALID, "mode = %d unknown", mode);
    if (!score || !label || !active_idx || !n_active || !delta_idx || !delta_sign || !n_delta || !status)
        return fail(OIT_ERR_INVALID, "oit_update_active_set_noalloc: NULL buffer");
    if (active_capacity <= 0 || delta_capacity <= 0)
        return fail(OIT_ERR_INVALID, "capacities must be positive");
    if (mode == OIT_SELECT_THRESHOLD && !std::isfinite(thresh))
        return fail(OIT_ERR_INVALID, "threshold must be finite");
    void *base = nullptr;
    const oit_status st = scratch_address(&base);
    if (st != OIT_OK) return st;
    // the scratch keeps the last call's contents: the selection kernels clear or fully
    // write everything they read, and the status word is the caller's, cleared here
    SelectBuffers sb = select_buffers(base, n);
    sb.status = status;
    const hipStream_t s = (hipStream_t)stream;
    fill_u32((uint32_t *)status, 1, 0u, s);
    launch_select(score, n, mode, k, thresh, label, active_idx, active_capacity, n_active, delta_idx, delta_sign,
                  delta_capacity, n_delta, sb, s);
    return check_launch("oit_update_active_set_noalloc");
}

oit_status oit_label_delta(const uint8_t *old_label, const uint8_t *new_label, int64_t n, int32_t *active_idx,
                           int64_t active_capacity, int32_t *n_active, int32_t *delta_idx, int8_t *delta_sign,
                           int64_t delta_capacity, int32_t *n_delta, void *ws, size_t ws_bytes, oit_stream stream)
{
    if (n <= 0 || n > 0x7fffffffLL) return fail(OIT_ERR_INVALID, "n = %lld outside [1, 2^31)", (long long)n);
    if (!old_label || !new_label || !delta_idx || !delta_sign || !n_delta)
        return fail(OIT_ERR_INVALID, "oit_label_delta: NULL buffer");
    if ((active_idx == nullptr) != (n_active == nullptr))
        return fail(OIT_ERR_INVALID, "active_idx and n_active go together");
    if (delta_capacity <= 0 || (active_idx && active_capacity <= 0))
        return fail(OIT_ERR_INVALID, "capacities must be positive");
    const size_t need = oit_select_workspace_bytes(n);
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < need) return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    launch_label_delta(old_label, new_label, n, active_idx, active_capacity, n_active, delta_idx, delta_sign,
                       delta_capacity, n_delta, select_buffers(ws, n), (hipStream_t)stream);
    return check_launch("oit_label_delta");
}

oit_status oit_fps_views(const float *centres, int32_t n, int32_t s, int32_t start, int32_t *out)
{
    if (!centres || !out) return fail(OIT_ERR_INVALID, "oit_fps_views: NULL argument");
    if (n <= 0 || s <= 0 || s > n) return fail(OIT_ERR_INVALID, "oit_fps_views: need 0 < s <= n");
    if (start < 0 || start >= n) return fail(OIT_ERR_INVALID, "oit_fps_views: start outside [0, n)");
    std::vector<double> d(n);
    auto dist2 = [&](int i, int j) {
        const double dx = (double)centres[3 * i] - (double)centres[3 * j];
        const double dy = (double)centres[3 * i + 1] - (double)centres[3 * j + 1];
        const double dz = (double)centres[3 * i + 2] - (double)centres[3 * j + 2];
        return dx * dx + dy * dy + dz * dz;
    };
    out[0] = start;
    for (int i = 0; i < n; ++i) d[i] = dist2(i, start);
    for (int k = 1; k < s; ++k) {
        int best = 0;
        for (int i = 1; i < n; ++i)
            if (d[i] > d[best]) best = i;
        out[k] = best;
        for (int i = 0; i < n; ++i) {
            const double e = dist2(i, best);
            if (e < d[i]) d[i] = e;
        }
    }
    return ok();
}

oit_status oit_sparse_adam_step(float *const *params, const oit_grads *grads, float *const *m, float *const *v,
                                const int32_t *active_idx, const int32_t *n_active, int64_t n, const float *lr,
                                float beta1, float beta2, float eps, int32_t *step, oit_stream stream)
{
    if (!params || !grads || !m || !v || !lr || !step) return fail(OIT_ERR_INVALID, "oit_sparse_adam_step: NULL argument");
    if (n <= 0 || n > 0x7fffffffLL) return fail(OIT_ERR_INVALID, "n = %lld outside [1, 2^31)", (long long)n);
    if (!active_idx && n_active) return fail(OIT_ERR_INVALID, "n_active without active_idx");
    if (active_idx && !n_active) return fail(OIT_ERR_INVALID, "active_idx without n_active");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return fail(OIT_ERR_INVALID, "bad Adam hyper-parameters");
    AdamPtrs a;
    const float *gg[6] = {grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->sh, grads->vsh};
    for (int k = 0; k < 6; ++k) {
        if (!params[k] || !m[k] || !v[k] || !gg[k]) return fail(OIT_ERR_INVALID, "group %d: NULL pointer", k);
        a.p[k] = params[k];
        a.g[k] = gg[k];
        a.m[k] = m[k];
        a.v[k] = v[k];
        a.lr[k] = lr[k];
    }
    const int64_t rows_cap = active_idx ? grads->stride : n;
    if (grads->stride <= 0 || (!active_idx && grads->stride < n))
        return fail(OIT_ERR_INVALID, "grads.stride = %lld too small", (long long)grads->stride);
    launch_sparse_adam(a, grads->stride, active_idx, n_active, n, rows_cap, beta1, beta2, eps, step,
                       (hipStream_t)stream);
    return check_launch("oit_sparse_adam_step");
}

oit_status oit_sigma_adam_step(float *sigma, const double *grad_sigma, float *m, float *v, float lr, float beta1,
                               float beta2, float eps, int32_t *step, oit_stream stream)
{
    if (!sigma || !grad_sigma || !m || !v || !step) return fail(OIT_ERR_INVALID, "oit_sigma_adam_step: NULL argument");
    launch_sigma_adam(sigma, grad_sigma, m, v, lr, beta1, beta2, eps, step, (hipStream_t)stream);
    return check_launch("oit_sigma_adam_step");
}

// ---------------------------------------------------------------------------------
// densification of the first training phase (k_density.hip)
// ---------------------------------------------------------------------------------
oit_status oit_densify_stats(const oit_camera *cams, int32_t n_views, const oit_capacity *cap,
                             const int32_t *active_idx, const int32_t *n_active, const int32_t *n_delta,
                             float *grad_accum, float *denom, float *max_radius, const void *ws, size_t ws_bytes,
                             const oit_tuning *tuning, oit_stream stream)
{
    Plan p;
    oit_status st;
    if ((st = make_plan(cap, cams, n_views, tuning, p)) != OIT_OK) return st;
    if (!grad_accum || !denom || !max_radius) return fail(OIT_ERR_INVALID, "grad_accum, denom and max_radius are required");
    if (!active_idx && (n_active || n_delta || cap->active_capacity != cap->n))
        return fail(OIT_ERR_INVALID, "dense mode takes no n_active or n_delta and needs active_capacity == n");
    if (active_idx && !n_active) return fail(OIT_ERR_INVALID, "active_idx given without n_active");
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < p.total) return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p.total);
    const Buffers b = buffers(p, const_cast<void *>(ws), n_views, tuning);
    const RowList rl = rows(cap, active_idx, n_active, nullptr, nullptr, n_delta, p);
    launch_densify_stats(b, rl, grad_accum, denom, max_radius, (hipStream_t)stream);
    return check_launch("oit_densify_stats");
}

size_t oit_densify_workspace_bytes(int64_t n)
{
    return n > 0 ? density_workspace_bytes(n) : 0;
}

namespace {
oit_status check_density_splats(const oit_splats *s)
{
    if (!s) return fail(OIT_ERR_INVALID, "splats is NULL");
    if (s->n <= 0 || s->n > 0x7fffffffLL) return fail(OIT_ERR_INVALID, "splats.n = %lld outside [1, 2^31)", (long long)s->n);
    const void *ptrs[6] = {s->mean, s->log_scale, s->quat, s->opacity_logit, s->sh, s->vsh};
    for (int k = 0; k < 6; ++k)
        if (!ptrs[k] || !aligned(ptrs[k], 4)) return fail(OIT_ERR_INVALID, "splat group %d NULL or misaligned", k);
    return OIT_OK;
}

oit_status check_density_ws(const void *ws, size_t ws_bytes, int64_t n)
{
    if (!ws || !aligned(ws, 256)) return fail(OIT_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    const size_t need = density_workspace_bytes(n);
    if (ws_bytes < need) return fail(OIT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return OIT_OK;
}
}  // namespace

oit_status oit_densify_plan(const oit_splats *splats, const float *grad_accum, const float *denom,
                            const float *max_radius, const float *uniform, const oit_density_rules *rules,
                            int64_t *n_new, void *ws, size_t ws_bytes, oit_stream stream)
{
    oit_status st;
    if ((st = check_density_splats(splats)) != OIT_OK) return st;
    if (!grad_accum || !denom || !max_radius || !uniform || !rules || !n_new)
        return fail(OIT_ERR_INVALID, "oit_densify_plan: NULL argument");
    if (!aligned(n_new, 8)) return fail(OIT_ERR_INVALID, "n_new must be 8-byte aligned");
    if (!(rules->scene_extent > 0.f) || !(rules->keep_probability >= 0.f && rules->keep_probability <= 1.f) ||
        !(rules->percent_dense >= 0.f) || rules->reserved != 0)
        return fail(OIT_ERR_INVALID, "bad density rules (scene_extent > 0, keep_probability in [0, 1], reserved 0)");
    if ((st = check_density_ws(ws, ws_bytes, splats->n)) != OIT_OK) return st;
    launch_densify_plan(splat_ptrs(splats), grad_accum, denom, max_radius, uniform, *rules, n_new,
                        density_buffers(ws, splats->n), (hipStream_t)stream);
    return check_launch("oit_densify_plan");
}

oit_status oit_densify_apply(const oit_splats *splats, const float *const *m, const float *const *v,
                             const float *normals, float *const *params_new, float *const *m_new,
                             float *const *v_new, int64_t cap_new, const void *ws, size_t ws_bytes,
                             oit_stream stream)
{
    oit_status st;
    if ((st = check_density_splats(splats)) != OIT_OK) return st;
    if (!m || !v || !normals || !params_new || !m_new || !v_new) return fail(OIT_ERR_INVALID, "oit_densify_apply: NULL argument");
    for (int k = 0; k < 6; ++k)
        if (!m[k] || !v[k] || !params_new[k] || !m_new[k] || !v_new[k])
            return fail(OIT_ERR_INVALID, "group %d: NULL pointer", k);
    if (cap_new < 0) return fail(OIT_ERR_INVALID, "cap_new < 0");
    if ((st = check_density_ws(ws, ws_bytes, splats->n)) != OIT_OK) return st;
    launch_densify_apply(splat_ptrs(splats), m, v, normals, params_new, m_new, v_new, cap_new,
                         density_buffers(const_cast<void *>(ws), splats->n), (hipStream_t)stream);
    return check_launch("oit_densify_apply");
}

oit_status oit_reset_opacity(float *opacity_logit, float *m_opacity, float *v_opacity, int64_t n, float max_opacity,
                             oit_stream stream)
{
    if (!opacity_logit || !m_opacity || !v_opacity) return fail(OIT_ERR_INVALID, "oit_reset_opacity: NULL argument");
    if (n <= 0) return fail(OIT_ERR_INVALID, "n = %lld must be > 0", (long long)n);
    if (!(max_opacity > 0.f && max_opacity < 1.f)) return fail(OIT_ERR_INVALID, "max_opacity must be in (0, 1)");
    const float max_logit = (float)std::log((double)max_opacity / (1.0 - (double)max_opacity));
    launch_reset_opacity(opacity_logit, m_opacity, v_opacity, n, max_logit, (hipStream_t)stream);
    return check_launch("oit_reset_opacity");
}

oit_status oit_read_status(const void *ws, size_t ws_bytes, int32_t *out, oit_stream stream)
{
    if (!ws || !out || ws_bytes < 4) return fail(OIT_ERR_INVALID, "oit_read_status: bad arguments");
    hipError_t e = hipMemcpyAsync(out, ws, 4, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(OIT_ERR_HIP, "oit_read_status: %s", hipGetErrorString(e));
    return ok();
}

oit_status oit_read_counters(const void *ws, size_t ws_bytes, const oit_capacity *cap, const oit_camera *cams,
                             int32_t n_views, const oit_tuning *tuning, int64_t *out, oit_stream stream)
{
    Plan p;
    oit_status st;
    if ((st = make_plan(cap, cams, n_views, tuning, p)) != OIT_OK) return st;
    if (!ws || !out || ws_bytes < p.total) return fail(OIT_ERR_INVALID, "oit_read_counters: bad arguments");
    uint32_t v[CNT_SLOTS];
    hipError_t e = hipMemcpyAsync(v, (const char *)ws + p.counters, sizeof(v), hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(OIT_ERR_HIP, "oit_read_counters: %s", hipGetErrorString(e));
    out[0] = (int64_t)v[CNT_TOTAL_ENTRIES];
    out[1] = (int64_t)((uint64_t)v[CNT_PAIRS] | ((uint64_t)v[CNT_PAIRS + 1] << 32));
    out[2] = (int64_t)((uint64_t)v[CNT_EVAL] | ((uint64_t)v[CNT_EVAL + 1] << 32));
    out[3] = (int64_t)v[CNT_TOTAL_CHUNKS];
    out[4] = (int64_t)v[CNT_BOX_ITEMS];
    out[5] = (int64_t)v[CNT_WAVE_ITEMS];
    return ok();
}

oit_status oit_read_tile_entries(const void *ws, size_t ws_bytes, const oit_capacity *cap, const oit_camera *cams,
                                 int32_t n_views, const oit_tuning *tuning, uint32_t *out, int64_t out_len,
                                 oit_stream stream)
{
    Plan p;
    oit_status st;
    if ((st = make_plan(cap, cams, n_views, tuning, p)) != OIT_OK) return st;
    if (!ws || !out || ws_bytes < p.total || out_len < 2 * (int64_t)p.T)
        return fail(OIT_ERR_INVALID, "oit_read_tile_entries: bad arguments");
    // active counts then label-change counts, contiguous in the workspace
    hipError_t e = hipMemcpyAsync(out, (const char *)ws + p.tiles, 4 * 2 * (size_t)p.T, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(OIT_ERR_HIP, "oit_read_tile_entries: %s", hipGetErrorString(e));
    return ok();
}

oit_status oit_timing_enable(int32_t on)
{
    if (on && !g_timing_ready) {
        for (int k = 0; k < kTimingEvents; ++k) {
            const hipError_t e = hipEventCreate(&g_ev[k]);
            if (e != hipSuccess) return fail(OIT_ERR_HIP, "oit_timing_enable: %s", hipGetErrorString(e));
        }
        g_timing_ready = true;
    }
    g_timing_on = on != 0;
    return ok();
}

oit_status oit_timing_read(float *out)
{
    if (!out) return fail(OIT_ERR_INVALID, "oit_timing_read: NULL output");
    if (!g_timing_ready) return fail(OIT_ERR_INVALID, "oit_timing_read: timing was never enabled");
    for (int k = 0; k < 2; ++k) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(g_ev[2 * k + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_ev[2 * k], g_ev[2 * k + 1]);
        out[k] = e == hipSuccess ? ms : -1.f;
    }
    return ok();
}

oit_status oit_timing_read_stages(float *out)
{
    if (!out) return fail(OIT_ERR_INVALID, "oit_timing_read_stages: NULL output");
    if (!g_timing_ready) return fail(OIT_ERR_INVALID, "oit_timing_read_stages: timing was never enabled");
    // consecutive boundary events of the forward (4-7) and of the backward (8-11)
    const int pairs[6][2] = {{4, 5}, {5, 6}, {6, 7}, {8, 9}, {9, 10}, {10, 11}};
    for (int k = 0; k < 6; ++k) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(g_ev[pairs[k][1]]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_ev[pairs[k][0]], g_ev[pairs[k][1]]);
        out[k] = e == hipSuccess ? ms : -1.f;
    }
    return ok();
}

oit_status oit_clear_status(void *ws, size_t ws_bytes, oit_stream stream)
{
    if (!ws || ws_bytes < 4) return fail(OIT_ERR_INVALID, "oit_clear_status: bad arguments");
    fill_u32((uint32_t *)ws, 1, 0u, (hipStream_t)stream);
    return check_launch("oit_clear_status");
}

const char *oit_last_error(void) { return g_err; }

}  // extern "C"
