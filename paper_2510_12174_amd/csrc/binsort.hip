// Stages S2-S4: tile binning, (tile, depth) key sort and per-tile ranges.
//
// The pair count P stays on the device: every kernel after the scan reads it
// from the counters block and uses a fixed grid, so the whole sequence can be
// captured in a HIP graph.  The sort is a stable least-significant-digit radix
// sort (8-bit digits) over only the key bits in use (32 depth bits plus the
// bits of the largest global tile id).  Because pairs are emitted in increasing
// Gaussian index within a view and every pass is stable, equal (tile, depth)
// keys stay in index order: the result is the unique (tile, depth, index) order.
#include "ugs_internal.h"

namespace ugs {
namespace {

constexpr int kScanThreads = 256;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of 256 threads' values within a block (4 waves).
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t *lds4, uint32_t &total)
{
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(x);
    if (lane == 63) lds4[wave] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += lds4[w];
    total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    __syncthreads();
    return pre + inc - x;
}

__global__ void __launch_bounds__(kScanThreads) scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                          uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds4[4];
    int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k)
        if (base + k < n) s += in[base + k];
    uint32_t tot;
    block_excl_scan256(s, lds4, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block partials; stores P and the overflow flag.
__global__ void __launch_bounds__(1024) scan_top(uint32_t *__restrict__ part, int nb, int64_t cap,
                                                 DevCounters *__restrict__ cnt)
{
    __shared__ unsigned long long lds[16];
    const int t = threadIdx.x, lane = __lane_id(), wave = t >> 6;
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per;
    unsigned long long s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) s += part[b0 + k];
    unsigned long long inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    unsigned long long pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) pre += lds[w];
        tot += lds[w];
    }
    unsigned long long run = pre + inc - s;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) {
            uint32_t v = part[b0 + k];
            part[b0 + k] = (uint32_t)(run < 0xffffffffull ? run : 0xffffffffull);
            run += v;
        }
    if (t == 0) {
        bool over = tot > (unsigned long long)cap;
        cnt->P = (uint32_t)(tot < 0xffffffffull ? tot : 0xffffffffull);
        cnt->overflow = over ? 1u : 0u;
        cnt->n_eval = 0;
        cnt->n_contrib = 0;
    }
}

__global__ void __launch_bounds__(kScanThreads) scan_down(const uint32_t *__restrict__ in, int64_t n,
                                                        const uint32_t *__restrict__ part,
                                                        uint32_t *__restrict__ out)
{
    __shared__ uint32_t lds4[4];
    int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan256(s, lds4, tot) + part[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

// One thread per (view, Gaussian): writes its pairs at its scanned offset.
__global__ void __launch_bounds__(256) emit_pairs(const DevCam *__restrict__ cams, int64_t N, int64_t VN,
                                                  const uint32_t *__restrict__ touched,
                                                  const uint32_t *__restrict__ offs, const uint2 *__restrict__ rect,
                                                  const float4 *__restrict__ rec, int64_t cap,
                                                  const DevCounters *__restrict__ cnt,
                                                  unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= VN) return;
    const uint32_t nt = touched[idx];
    if (nt == 0 || cnt->overflow) return;
    const uint64_t off = offs[idx];
    if (off + nt > (uint64_t)cap) return;
    const int v = (int)(idx / N);
    const uint32_t gid = (uint32_t)(idx - (int64_t)v * N);
    const DevCam &cam = cams[v];
    const uint2 rc = rect[idx];
    const int tx0 = rc.x & 0xffff, ty0 = rc.x >> 16, tx1 = rc.y & 0xffff, ty1 = rc.y >> 16;
    const uint32_t dbits = __float_as_uint(rec[idx * 4 + 1].w);
    uint64_t o = off;
    for (int ty = ty0; ty < ty1; ++ty)
        for (int tx = tx0; tx < tx1; ++tx) {
            uint64_t tile = cam.tile_base + (uint32_t)(ty * cam.tiles_x + tx);
            keys[o] = (tile << 32) | dbits;
            vals[o] = gid;
            ++o;
        }
}

__device__ __forceinline__ uint32_t pair_count(const DevCounters *cnt) { return cnt->overflow ? 0u : cnt->P; }

// Per-block digit histogram of the block's contiguous chunk.
__global__ void __launch_bounds__(kSortThreads) radix_hist(const unsigned long long *__restrict__ keys,
                                                           const DevCounters *__restrict__ cnt, int shift,
                                                           uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t P = pair_count(cnt);
    const uint32_t per = ((P + kSortBlocks - 1) / kSortBlocks + 255) & ~255u;
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = min((uint64_t)P, b0 + per);
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += kSortThreads) {
        uint32_t d = (uint32_t)(keys[i] >> shift) & 255u;
        atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * kSortBlocks + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's per-block counts.
__global__ void __launch_bounds__(kSortThreads) radix_scan_digit(uint32_t *__restrict__ hist,
                                                                 uint32_t *__restrict__ digit_tot)
{
    __shared__ uint32_t lds4[4];
    uint32_t *row = hist + (size_t)blockIdx.x * kSortBlocks;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = row[threadIdx.x * 4 + k];
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan256(s, lds4, tot);
    for (int k = 0; k < 4; ++k) {
        row[threadIdx.x * 4 + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = tot;
}

// Stable scatter: each block walks its chunk in order, 256 keys at a time; ranks
// within a wave come from eight ballots (lanes sharing the digit), ranks across
// waves and tiles from per-digit running counters in LDS.
__global__ void __launch_bounds__(kSortThreads) radix_scatter(
    const unsigned long long *__restrict__ kin, const uint32_t *__restrict__ vin, unsigned long long *__restrict__ kout,
    uint32_t *__restrict__ vout, const DevCounters *__restrict__ cnt, int shift, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ digit_tot)
{
    __shared__ uint32_t base[256], run[256], lds4[4];
    __shared__ uint32_t wcnt[4][256], wpre[4][256];
    const int t = threadIdx.x, lane = __lane_id(), wave = t >> 6;
    uint32_t dt = digit_tot[t], tot;
    uint32_t dex = block_excl_scan256(dt, lds4, tot);
    base[t] = dex + hist[t * kSortBlocks + blockIdx.x];
    run[t] = 0;
    for (int w = 0; w < 4; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint32_t P = pair_count(cnt);
    const uint32_t per = ((P + kSortBlocks - 1) / kSortBlocks + 255) & ~255u;
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = min((uint64_t)P, b0 + per);
    const uint64_t lt = __lanemask_lt();
    for (uint64_t tb = b0; tb < b1; tb += kSortThreads) {
        const uint64_t i = tb + t;
        const bool valid = i < b1;
        unsigned long long key = valid ? kin[i] : 0ull;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        {
            uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
            uint32_t r = run[t];
            wpre[0][t] = r;
            wpre[1][t] = r + c0;
            wpre[2][t] = r + c0 + c1;
            wpre[3][t] = r + c0 + c1 + c2;
            run[t] = r + c0 + c1 + c2 + c3;
            wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + wpre[wave][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
    }
}

__global__ void __launch_bounds__(256) tile_ranges(const unsigned long long *__restrict__ keys,
                                                   const DevCounters *__restrict__ cnt, uint2 *__restrict__ ranges)
{
    const uint32_t P = pair_count(cnt);
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < P; i += (uint64_t)gridDim.x * 256) {
        uint32_t tile = (uint32_t)(keys[i] >> 32);
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[tile].x = (uint32_t)i;
        if (i + 1 == P || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[tile].y = (uint32_t)(i + 1);
    }
}

__global__ void __launch_bounds__(256) fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_binsort(const Problem &pb, const WsLayout &L, char *ws, hipStream_t s, int *final_buf)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto touched = (uint32_t *)(ws + L.touched);
    auto offs = (uint32_t *)(ws + L.offs);
    auto part = (uint32_t *)(ws + L.scan_part);
    auto cnt = (DevCounters *)(ws + L.counters);
    auto rect = (const uint2 *)(ws + L.rect);
    auto rec = (const float4 *)(ws + L.rec);
    unsigned long long *keys[2] = {(unsigned long long *)(ws + L.keys0), (unsigned long long *)(ws + L.keys1)};
    uint32_t *vals[2] = {(uint32_t *)(ws + L.vals0), (uint32_t *)(ws + L.vals1)};
    auto hist = (uint32_t *)(ws + L.hist);
    auto dtot = (uint32_t *)(ws + L.digit_tot);
    auto ranges = (uint2 *)(ws + L.ranges);
    const int64_t VN = L.VN;
    hipError_t e;
    hipLaunchKernelGGL(scan_reduce, dim3(L.nb_scan), dim3(kScanThreads), 0, s, touched, VN, part);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, part, L.nb_scan, L.pair_cap, cnt);
    if (VN > 0) {
        hipLaunchKernelGGL(scan_down, dim3(L.nb_scan), dim3(kScanThreads), 0, s, touched, VN, part, offs);
        hipLaunchKernelGGL(emit_pairs, dim3((unsigned)((VN + 255) / 256)), dim3(256), 0, s, cams, L.N, VN, touched,
                           offs, rect, rec, L.pair_cap, cnt, keys[0], vals[0]);
    }
    int cur = 0;
    for (int pass = 0; pass < L.sort_passes; ++pass) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(radix_hist, dim3(kSortBlocks), dim3(kSortThreads), 0, s, keys[cur], cnt, shift, hist);
        hipLaunchKernelGGL(radix_scan_digit, dim3(256), dim3(kSortThreads), 0, s, hist, dtot);
        hipLaunchKernelGGL(radix_scatter, dim3(kSortBlocks), dim3(kSortThreads), 0, s, keys[cur], vals[cur],
                           keys[cur ^ 1], vals[cur ^ 1], cnt, shift, hist, dtot);
        cur ^= 1;
    }
    if ((e = launch_fill_u32((uint32_t *)ranges, 0u, 2 * L.total_tiles, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(tile_ranges, dim3(4096), dim3(256), 0, s, keys[cur], cnt, ranges);
    *final_buf = cur;
    return hipGetLastError();
}

}  // namespace ugs
