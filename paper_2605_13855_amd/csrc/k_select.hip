// Active-set update (Sec. 4.1): pick the active splats from their scores and emit
// the label changes.  Top-k uses a three-pass radix select on order-preserving keys
// of the float scores (11 + 11 + 10 bits), then a stable compaction that gives the
// tied scores at the k-th value to the lowest splat ids.
#include <cstring>

#include "oit_internal.h"

namespace oit {

constexpr int kSelThreads = 256;
constexpr int kSelPerThread = 4;
constexpr int kSelBlock = kSelThreads * kSelPerThread;   // elements per block
constexpr int kBins = 2048;

enum { ST_PREFIX = 0, ST_KREM = 1, ST_MASK = 2, ST_SLOTS = 8 };

__device__ __forceinline__ uint32_t order_key(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// exclusive scan of one uint32 per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t s_w[kSelThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) {
        if (w < wave) wbase += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

struct SelArgs {
    const float *score;
    int64_t n;
    uint8_t *label;
    int32_t *active_idx;
    int64_t acap;
    int32_t *n_active;
    int32_t *delta_idx;
    int8_t *delta_sign;
    int64_t dcap;
    int32_t *n_delta;
    SelectBuffers sb;
    const uint8_t *new_label;   // label-diff mode: the target labels
    bool write_label;           // store the new labels into `label`
};

__global__ void k_sel_init(SelArgs a, uint32_t prefix, uint32_t krem, uint32_t mask)
{
    const int i = threadIdx.x;
    if (i == 0) {
        a.sb.state[ST_PREFIX] = prefix;
        a.sb.state[ST_KREM] = krem;
        a.sb.state[ST_MASK] = mask;
    }
    for (int b = i; b < kBins; b += blockDim.x) a.sb.hist[b] = 0;
}

__global__ __launch_bounds__(kSelThreads) void k_sel_hist(SelArgs a, int shift, int width)
{
    __shared__ uint32_t s_h[kBins];
    for (int b = threadIdx.x; b < kBins; b += kSelThreads) s_h[b] = 0;
    __syncthreads();
    const uint32_t prefix = a.sb.state[ST_PREFIX], mask = a.sb.state[ST_MASK];
    const uint32_t dmask = (1u << width) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kSelBlock;
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + (int64_t)k * kSelThreads + threadIdx.x;
        if (i < a.n) {
            const uint32_t key = order_key(a.score[i]);
            if ((key & mask) == prefix) atomicAdd(&s_h[(key >> shift) & dmask], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kSelThreads)
        if (s_h[b]) atomicAdd(&a.sb.hist[b], s_h[b]);
}

// one block of 1024 threads: find the digit holding the k_rem-th largest key
__global__ __launch_bounds__(1024) void k_sel_find(SelArgs a, int shift, int width)
{
    __shared__ uint32_t s_suf[kBins + 1];
    const int nb = 1 << width;
    for (int b = threadIdx.x; b < kBins; b += 1024) s_suf[b] = b < nb ? a.sb.hist[b] : 0;
    if (threadIdx.x == 0) s_suf[kBins] = 0;
    __syncthreads();
    // suffix sums: s_suf[b] = sum_{b' >= b} hist[b']  (simple in-place doubling scan)
    for (int o = 1; o < kBins; o <<= 1) {
        uint32_t v0 = 0, v1 = 0;
        const int b0 = threadIdx.x, b1 = threadIdx.x + 1024;
        if (b0 + o < kBins) v0 = s_suf[b0 + o];
        if (b1 + o < kBins) v1 = s_suf[b1 + o];
        __syncthreads();
        s_suf[b0] += v0;
        s_suf[b1] += v1;
        __syncthreads();
    }
    const uint32_t krem = a.sb.state[ST_KREM];
    for (int b = threadIdx.x; b < nb; b += 1024) {
        const uint32_t above = s_suf[b + 1], atb = s_suf[b];
        if (above < krem && atb >= krem) {
            a.sb.state[ST_PREFIX] |= (uint32_t)b << shift;
            a.sb.state[ST_MASK] |= ((1u << width) - 1u) << shift;
            a.sb.state[ST_KREM] = krem - above;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += 1024) a.sb.hist[b] = 0;
}

// per block: count keys equal to the threshold key
__global__ __launch_bounds__(kSelThreads) void k_sel_count_eq(SelArgs a)
{
    const uint32_t K = a.sb.state[ST_PREFIX];
    const int64_t base = (int64_t)blockIdx.x * kSelBlock + (int64_t)threadIdx.x * kSelPerThread;
    uint32_t c = 0;
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + k;
        if (i < a.n && order_key(a.score[i]) == K) ++c;
    }
    uint32_t tot;
    block_excl_scan(c, &tot);
    if (threadIdx.x == 0) a.sb.blk_a[blockIdx.x] = tot;
}

// single block: exclusive scans of up to two per-block count arrays (in place; entry
// nblk receives the total)
__global__ __launch_bounds__(1024) void k_sel_scan(uint32_t *x, uint32_t *y, int64_t nblk)
{
    __shared__ uint32_t s_x[1024], s_y[1024];
    const int tid = threadIdx.x;
    const int64_t seg = (nblk + 1023) / 1024;
    const int64_t t0 = tid * seg < nblk ? tid * seg : nblk;
    const int64_t t1 = t0 + seg < nblk ? t0 + seg : nblk;
    uint32_t sx = 0, sy = 0;
    for (int64_t t = t0; t < t1; ++t) {
        sx += x[t];
        if (y) sy += y[t];
    }
    s_x[tid] = sx;
    s_y[tid] = sy;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t vx = tid >= o ? s_x[tid - o] : 0, vy = tid >= o ? s_y[tid - o] : 0;
        __syncthreads();
        s_x[tid] += vx;
        s_y[tid] += vy;
        __syncthreads();
    }
    uint32_t px = s_x[tid] - sx, py = s_y[tid] - sy;
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t cx = x[t];
        x[t] = px;
        px += cx;
        if (y) {
            const uint32_t cy = y[t];
            y[t] = py;
            py += cy;
        }
    }
    if (tid == 1023) {
        x[nblk] = s_x[1023];
        if (y) y[nblk] = s_y[1023];
    }
}

// per block: selection flags (bit0 selected, bit1 label changed) and counts
__global__ __launch_bounds__(kSelThreads) void k_sel_flags(SelArgs a)
{
    const uint32_t K = a.sb.state[ST_PREFIX], krem = a.sb.state[ST_KREM];
    const int64_t base = (int64_t)blockIdx.x * kSelBlock + (int64_t)threadIdx.x * kSelPerThread;
    uint32_t keys[kSelPerThread];
    uint32_t ceq = 0;
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + k;
        keys[k] = i < a.n ? order_key(a.score[i]) : 0u;
        if (i < a.n && keys[k] == K) ++ceq;
    }
    uint32_t tot;
    uint32_t eq_rank = a.sb.blk_a[blockIdx.x] + block_excl_scan(ceq, &tot);
    uint32_t csel = 0, cdel = 0;
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + k;
        if (i >= a.n) break;
        bool sel = keys[k] > K;
        if (keys[k] == K) {
            sel = eq_rank < krem;
            ++eq_rank;
        }
        const bool chg = (a.label[i] != 0) != sel;
        a.sb.flags[i] = (uint8_t)((sel ? 1 : 0) | (chg ? 2 : 0));
        csel += sel;
        cdel += chg;
    }
    uint32_t ts, td;
    block_excl_scan(csel, &ts);
    block_excl_scan(cdel, &td);
    if (threadIdx.x == 0) {
        a.sb.blk_b[blockIdx.x] = ts;
        a.sb.blk_c[blockIdx.x] = td;
    }
}

__global__ __launch_bounds__(kSelThreads) void k_sel_write(SelArgs a)
{
    const int64_t base = (int64_t)blockIdx.x * kSelBlock + (int64_t)threadIdx.x * kSelPerThread;
    uint8_t f[kSelPerThread];
    uint32_t csel = 0, cdel = 0;
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + k;
        f[k] = i < a.n ? a.sb.flags[i] : 0;
        csel += f[k] & 1;
        cdel += (f[k] >> 1) & 1;
    }
    uint32_t ts, td;
    uint32_t ps = a.sb.blk_b[blockIdx.x] + block_excl_scan(csel, &ts);
    uint32_t pd = a.sb.blk_c[blockIdx.x] + block_excl_scan(cdel, &td);
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + k;
        if (i >= a.n) break;
        const bool sel = f[k] & 1, chg = (f[k] >> 1) & 1;
        if (sel) {
            if (a.active_idx && (int64_t)ps < a.acap) a.active_idx[ps] = (int32_t)i;
            ++ps;
        }
        if (chg) {
            if ((int64_t)pd < a.dcap) {
                a.delta_idx[pd] = (int32_t)i;
                a.delta_sign[pd] = sel ? (int8_t)-1 : (int8_t)1;
            }
            ++pd;
        }
        if (a.write_label) a.label[i] = sel ? 1 : 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t tsel = a.sb.blk_b[a.sb.nblk], tdel = a.sb.blk_c[a.sb.nblk];
        if (a.n_active) *a.n_active = (int32_t)((int64_t)tsel < a.acap ? tsel : a.acap);
        *a.n_delta = (int32_t)((int64_t)tdel < a.dcap ? tdel : a.dcap);
        if (a.active_idx && (int64_t)tsel > a.acap) atomicOr(a.sb.status, OIT_STATUS_ACTIVE_OVERFLOW);
        if ((int64_t)tdel > a.dcap) atomicOr(a.sb.status, OIT_STATUS_DELTA_OVERFLOW);
    }
}

// label-diff mode: flags and per-block counts from two label arrays
__global__ __launch_bounds__(kSelThreads) void k_lab_flags(SelArgs a)
{
    const int64_t base = (int64_t)blockIdx.x * kSelBlock + (int64_t)threadIdx.x * kSelPerThread;
    uint32_t csel = 0, cdel = 0;
    for (int k = 0; k < kSelPerThread; ++k) {
        const int64_t i = base + k;
        if (i >= a.n) break;
        const bool sel = a.new_label[i] != 0;
        const bool chg = (a.label[i] != 0) != sel;
        a.sb.flags[i] = (uint8_t)((sel ? 1 : 0) | (chg ? 2 : 0));
        csel += sel;
        cdel += chg;
    }
    uint32_t ts, td;
    block_excl_scan(csel, &ts);
    block_excl_scan(cdel, &td);
    if (threadIdx.x == 0) {
        a.sb.blk_b[blockIdx.x] = ts;
        a.sb.blk_c[blockIdx.x] = td;
    }
}

void launch_label_delta(const uint8_t *old_label, const uint8_t *new_label, int64_t n, int32_t *active_idx,
                        int64_t acap, int32_t *n_active, int32_t *delta_idx, int8_t *delta_sign, int64_t dcap,
                        int32_t *n_delta, const SelectBuffers &sb, hipStream_t s)
{
    SelArgs a{nullptr, n, const_cast<uint8_t *>(old_label), active_idx, acap, n_active, delta_idx, delta_sign,
              dcap, n_delta, sb, new_label, false};
    const unsigned nblk = (unsigned)sb.nblk;
    hipLaunchKernelGGL(k_lab_flags, dim3(nblk), dim3(kSelThreads), 0, s, a);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, s, sb.blk_b, sb.blk_c, sb.nblk);
    hipLaunchKernelGGL(k_sel_write, dim3(nblk), dim3(kSelThreads), 0, s, a);
}

static uint32_t host_order_key(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

void launch_select(const float *score, int64_t n, int mode, int64_t k, float thresh, uint8_t *label,
                   int32_t *active_idx, int64_t acap, int32_t *n_active, int32_t *delta_idx,
                   int8_t *delta_sign, int64_t dcap, int32_t *n_delta, const SelectBuffers &sb,
                   hipStream_t s)
{
    SelArgs a{score, n, label, active_idx, acap, n_active, delta_idx, delta_sign, dcap, n_delta, sb, nullptr, true};
    const unsigned nblk = (unsigned)sb.nblk;
    bool radix = false;
    if (mode == OIT_SELECT_THRESHOLD) {
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, a, host_order_key(thresh), 0u, 0xffffffffu);
    } else if (k <= 0) {
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, a, 0xffffffffu, 0u, 0xffffffffu);
    } else if (k >= n) {
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, a, 0u, (uint32_t)n, 0xffffffffu);
    } else {
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, a, 0u, (uint32_t)k, 0u);
        radix = true;
    }
    if (radix) {
        const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
        for (int p = 0; p < 3; ++p) {
            hipLaunchKernelGGL(k_sel_hist, dim3(nblk), dim3(kSelThreads), 0, s, a, shifts[p], widths[p]);
            hipLaunchKernelGGL(k_sel_find, dim3(1), dim3(1024), 0, s, a, shifts[p], widths[p]);
        }
    }
    hipLaunchKernelGGL(k_sel_count_eq, dim3(nblk), dim3(kSelThreads), 0, s, a);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, s, sb.blk_a, (uint32_t *)nullptr, sb.nblk);
    hipLaunchKernelGGL(k_sel_flags, dim3(nblk), dim3(kSelThreads), 0, s, a);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, s, sb.blk_b, sb.blk_c, sb.nblk);
    hipLaunchKernelGGL(k_sel_write, dim3(nblk), dim3(kSelThreads), 0, s, a);
}

}  // namespace oit
