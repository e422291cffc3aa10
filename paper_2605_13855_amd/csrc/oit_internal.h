// Internal interface between the C ABI (oit_api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oit.h"
#include "oit_device.h"

namespace oit {

constexpr int kMaxViews = 64;
constexpr int kBwdLanes = 64;   // splats per backward work item (one wave)
constexpr int kScanThreads = 1024;
constexpr int kEpStride = 12;                  // floats per entry partial (11 used, 16-byte rows)
constexpr int kEpUsed = 11;                    // screen-space partials per entry row
constexpr int kPixStatePlanes = OIT_PIXSTATE_PLANES;   // T, Q, F (rgb), dQ/dsigma per pixel
constexpr int kScanBlockItems = 256 * 16;      // values per block of the device-wide scan
constexpr int kSortGrid = 1024;                // blocks of a radix-sort pass (each a contiguous range)
constexpr int kRadixBits = 5;                  // digit width of a radix-sort pass
constexpr int kRadixBuckets = 1 << kRadixBits;
constexpr int kSizeBits = 5;                   // footprint-size class below (tile, class) in the sort key
constexpr int kSigPixParts = 2048;             // blocks of the per-pixel backward kernels (at most)
constexpr int kSigPreParts = 4096;             // blocks of the preprocess backward (at most)

// counters[] slots in the workspace
// (CNT_PAIRS and CNT_EVAL are 64-bit counters occupying two slots each)
// CNT_NPAIRS: (listed record, view) pairs of the call; CNT_SORT_N: tile entries that fit
// the pair capacity (the sorted list's length)
// CNT_CAP: nonzero if a record listed by the forward call may reach the opacity cap
// CNT_XQUEUE .. CNT_XQUEUE + 7: the backward's per-XCD work-queue tickets
// CNT_BOX_ITEMS: backward work items that took the footprint-box walk
// CNT_FQUEUE: the forward's work-queue ticket (positions in the heavy-first tile order)
// CNT_WAVE_ITEMS: backward work items walked group by group by the whole wave
enum { CNT_NPAIRS = 0, CNT_TOTAL_CHUNKS = 1, CNT_TOTAL_ENTRIES = 2, CNT_SORT_N = 3, CNT_PAIRS = 4, CNT_EVAL = 6, CNT_CAP = 8,
       CNT_XQUEUE = 9, CNT_BOX_ITEMS = 17, CNT_FQUEUE = 18, CNT_WAVE_ITEMS = 19, CNT_SLOTS = 32 };
constexpr int kXcds = 8;        // XCDs of the device; workgroup b runs on XCD b mod 8

struct SplatPtrs {
    const float *mean, *log_scale, *quat, *logit, *sh, *vsh;
    int64_t n;
};

struct GradPtrs {
    float *mean, *log_scale, *quat, *logit, *sh, *vsh;
    int64_t stride;
};

// Which rows a call renders: records [0, n_active) are active rows, records
// [Acap, Acap + n_delta) are label changes.
struct RowList {
    const int32_t *active_idx;   // NULL: row r is splat r
    const int32_t *n_active;     // NULL: n_active_host
    int64_t n_active_host;
    const int32_t *delta_idx;
    const int8_t *delta_sign;
    const int32_t *n_delta;      // NULL: no label changes
    int64_t Acap, Rcap;          // Rcap = Acap + Dcap: record stride of one view
};

struct Buffers {
    int32_t *status;
    CamDev *cams;
    uint32_t *counters;
    uint32_t *cnt_a, *cnt_d;                    // [T] active / label-change entries per tile
    uint32_t *tile_off, *chunk_off;             // [T + 1]
    uint32_t *chunk_tile;                       // [max_chunks] tile of each backward work item
    uint32_t *tile_order;                       // [T] the forward's launch order: heaviest tiles first
    // Tile entries.  Every (listed record, view) pair -- index view * nrec + k for the
    // k-th listed record, nrec = listed records of the call -- owns the slots
    // [hoff, hoff + nhits) of the unsorted list, one per tile it reaches; the list is
    // sorted by (tile, class, size class) into `entries` (record index) and `orig` (the entry's
    // unsorted slot).
    uint32_t *entries;                          // [pair_cap]
    uint32_t *orig;                             // [pair_cap]
    uint32_t *keys[2], *vals[2], *recs[2];      // [pair_cap] radix-sort buffers
    uint32_t *hist, *hist_off;                  // [kRadixBuckets][kSortGrid] digit counts and their scan
    Rec *rec;                                   // [V][Rcap]
    short4 *rect;                               // [V][Rcap] tile rectangle [x0, x1) x [y0, y1)
    uint32_t *nhits;                            // [pairs] tiles the (listed record, view) pair reaches
    uint32_t *hoff;                             // [pairs] exclusive scan of nhits
    uint32_t *scan_tmp;                         // block sums of the device-wide scans
    float *ep;                                  // [pair_cap][kEpStride] screen-space partials, by unsorted slot
    float4 *pixconst;                           // [total_px] (A_r, A_g, A_b, -s1)
    float2 *pixB;                               // [total_px] (B, lambda = (dQ/dsigma) / Q)
    double *sig_part;                           // [kSigPixParts + kSigPreParts] per-block shares of dL/dsigma
    double *loss_part;                          // [kSigPixParts] per-block shares of the L1 loss
    unsigned long long *tile_cnt;               // [T][2] contributing / evaluated active pairs per tile
    uint32_t max_chunks;
    int n_views, T, tile, bwd_mode;
    int64_t total_px, pair_cap;
    int64_t Acap, Rcap;                         // record stride: Rcap per view
};

// View of a batch tile (views are packed in order; at most kMaxViews of them).
__device__ __forceinline__ int view_of_tile(const CamDev *cams, int n_views, int tile)
{
    int v = 0;
    for (int k = 1; k < n_views; ++k)
        if (tile >= cams[k].tile_base) v = k;
    return v;
}

void upload_cams(const CamDev *host, int n_views, CamDev *dst, hipStream_t s);
void fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
void fill_f32(float *p, size_t n, float v, hipStream_t s);
void fill_f64(double *p, size_t n, double v, hipStream_t s);

void launch_preprocess_count(const SplatPtrs &sp, const SplatPtrs &dsp, const float *sigma, const RowList &rl,
                             const Buffers &b, hipStream_t s);
void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
// count scan, entry list, sort by (tile, class, size class), per-tile ranges (after preprocess)
void launch_binning(const RowList &rl, const Buffers &b, hipStream_t s);
// Optional kernel timing: a launch given a KTimer records `start` when the kernel
// begins and `stop` when it ends (hipExtLaunchKernelGGL; not for graph capture).
struct KTimer {
    hipEvent_t start, stop;
};

// deltas: the call lists label changes (their entries are blended into pre first)
bool launch_raster_fwd(const Buffers &b, const float *sigma, const float bg[3], float *pre, bool deltas,
                       float *image, float *pixstate, int batch, hipStream_t s, const KTimer *fwd_t = nullptr);

void launch_l1_loss(const Buffers &b, const float *image, const float *target, float *grad, double *loss,
                    hipStream_t s);
// *dst = sum of parts[0 .. n), added in a fixed order by one block
void launch_sum_shares(const double *parts, int n, double *dst, hipStream_t s);
void launch_pixconst(const Buffers &b, const float *sigma, const float bg[3], const float *pre,
                     const float *grad_image, const float *pixstate, double *grad_sigma, hipStream_t s);
bool launch_raster_bwd(const Buffers &b, const RowList &rl, hipStream_t s, const KTimer *t = nullptr);
void launch_preprocess_bwd(const SplatPtrs &sp, const float *sigma, const RowList &rl, const Buffers &b,
                           const GradPtrs &g, double *grad_sigma, float *score, const float eps[6],
                           hipStream_t s);

// acc: the two sums (L1, SSIM); parts: 2 x 3 x tiles16 per-block shares of them
void launch_l1_dssim(const CamDev *cams, int n_views, int64_t total_px, int tiles16, const float *image,
                     const float *target, float lambda, float *grad, double *loss, float *maps, double *acc,
                     double *parts, hipStream_t s);

struct SelectBuffers {
    int32_t *status;
    uint32_t *state;      // [8]: prefix, k_remaining, digit results
    uint32_t *hist;       // [2048]
    uint32_t *blk_a, *blk_b, *blk_c;  // per-block counts / offsets [nblk + 1]
    uint8_t *flags;       // [n]
    int64_t nblk;
};
void launch_select(const float *score, int64_t n, int mode, int64_t k, float thresh, uint8_t *label,
                   int32_t *active_idx, int64_t acap, int32_t *n_active, int32_t *delta_idx,
                   int8_t *delta_sign, int64_t dcap, int32_t *n_delta, const SelectBuffers &sb,
                   hipStream_t s);

void launch_label_delta(const uint8_t *old_label, const uint8_t *new_label, int64_t n, int32_t *active_idx,
                        int64_t acap, int32_t *n_active, int32_t *delta_idx, int8_t *delta_sign, int64_t dcap,
                        int32_t *n_delta, const SelectBuffers &sb, hipStream_t s);

struct AdamPtrs {
    float *p[6];
    const float *g[6];
    float *m[6];
    float *v[6];
    float lr[6];
};
void launch_sparse_adam(const AdamPtrs &a, int64_t gstride, const int32_t *active_idx, const int32_t *n_active,
                        int64_t n, int64_t rows_cap, float b1, float b2, float eps, int32_t *step,
                        hipStream_t s);
void launch_sigma_adam(float *sigma, const double *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int32_t *step, hipStream_t s);

}  // namespace oit
