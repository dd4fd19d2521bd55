// Stages S2-S4: tile binning, (tile, depth) ordering and per-tile ranges.
//
// Order of work:
//   1. compact the visible (view, Gaussian) records (rectangle not empty);
//   2. sort them by camera depth -- a stable LSD radix sort of the 32 depth
//      bits, on ~R records only (views need no key bits: tile ids keep them
//      apart and every later pass is stable);
//   3. count, in that order, the rectangle tiles that each record's alpha
//      ellipse reaches, scan the counts and emit one (tile, index) pair per
//      kept tile: pairs come out in (depth, index) order;
//   4. stable LSD radix sort of the pairs by global tile id (32-bit keys, only
//      the bits in use, in passes of at most 9 bits: two passes up to 262,144
//      tiles);
//   5. per-tile [start, end) ranges.
// Because every sort pass is stable and the compaction keeps index order, each
// tile's list ends up in the unique (depth bits, index) order.  The pair count
// stays on the device: every kernel after the scans reads it from the counters
// block and uses a fixed grid, so the whole sequence can be captured in a graph.
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

// Scan input: element i of `in` (0 beyond the device count), or its flag (> 0).
struct ScanIn {
    const uint32_t *in;
    int64_t n;                // host bound (grid size)
    const uint32_t *n_dev;    // optional device bound
    int flag;                 // 1: scan (in[i] > 0), 0: scan in[i]
    __device__ __forceinline__ uint32_t at(int64_t i) const
    {
        if (i >= n || (n_dev && i >= (int64_t)*n_dev)) return 0u;
        uint32_t v = in[i];
        return flag ? (v > 0u ? 1u : 0u) : v;
    }
};

__global__ void __launch_bounds__(kScanThreads) scan_reduce(ScanIn si, uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds4[4];
    int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) s += si.at(base + k);
    uint32_t tot;
    block_excl_scan256(s, lds4, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block partials.  Stores the total in
// *total; with cap >= 0 also the overflow flag and the usable count.
__global__ void __launch_bounds__(1024) scan_top(uint32_t *__restrict__ part, int nb, int64_t cap,
                                                 uint32_t *__restrict__ total, uint32_t *__restrict__ overflow,
                                                 uint32_t *__restrict__ usable, DevCounters *__restrict__ cnt_reset)
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
        *total = (uint32_t)(tot < 0xffffffffull ? tot : 0xffffffffull);
        if (overflow) {
            bool over = tot > (unsigned long long)cap;
            *overflow = over ? 1u : 0u;
            *usable = over ? 0u : (uint32_t)tot;
        }
        if (cnt_reset) {
            cnt_reset->n_eval = 0;
            cnt_reset->n_contrib = 0;
        }
    }
}

__global__ void __launch_bounds__(kScanThreads) scan_down(ScanIn si, const uint32_t *__restrict__ part,
                                                        uint32_t *__restrict__ out)
{
    __shared__ uint32_t lds4[4];
    int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = si.at(base + k);
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan256(s, lds4, tot) + part[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        if (base + k < si.n) out[base + k] = ex;
        ex += v[k];
    }
}

// Visible records -> (depth bits, record index), in index order.  zbits holds
// the record's depth bits, written densely by the projection.
__global__ void __launch_bounds__(256) compact_visible(int64_t N, int64_t VN, const uint32_t *__restrict__ touched,
                                                       const uint32_t *__restrict__ voff,
                                                       const uint32_t *__restrict__ zbits,
                                                       uint32_t *__restrict__ dkey, uint32_t *__restrict__ didx)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= VN || touched[idx] == 0) return;
    const uint32_t r = voff[idx];
    // the camera depth is > z_near > 0, so its float bits order as integers;
    // the view needs no key bits (tile ids keep views apart and the tile sort
    // is stable)
    dkey[r] = zbits[idx];
    didx[r] = (uint32_t)idx;
}

// Visible views of each Gaussian (reads of neighbouring threads coalesce per
// view), and their records in (Gaussian, view) order at the scanned offsets.
__global__ void __launch_bounds__(256) gauss_views(int64_t N, int V, const uint32_t *__restrict__ touched,
                                                   uint32_t *__restrict__ count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    uint32_t c = 0;
    for (int v = 0; v < V; ++v) c += touched[(int64_t)v * N + i] > 0u ? 1u : 0u;
    count[i] = c;
}

__global__ void __launch_bounds__(256) gauss_emit(int64_t N, int V, const uint32_t *__restrict__ touched,
                                                  const uint32_t *__restrict__ off, uint32_t *__restrict__ list)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    uint32_t o = off[i];
    for (int v = 0; v < V; ++v) {
        const int64_t idx = (int64_t)v * N + i;
        if (touched[idx] > 0u) list[o++] = (uint32_t)idx;
    }
}

// One depth-sorted record as the binning walk sees it: rectangle, view
// geometry and the culling data of its FP32 projection record (96 B, so that
// a wavefront can stage its 64 records in LDS).
struct __align__(16) WalkRec {
    uint32_t idx, gid, rx, ry, w, area, tb, tw;
    int W, H;
    float rw;        // 1 / w
    uint32_t start;  // first position of the record in the wavefront's tile run
    CullGeom c;
    uint32_t nt, off, pad0, pad1;  // emission: counted slots and first pair
};

__device__ __forceinline__ void walk_load(WalkRec &k, const DevCam *cams, int64_t N, uint32_t idx,
                                          const uint2 *rect, const float4 *rec)
{
    k.idx = idx;
    const int v = (int)(idx / (uint64_t)N);
    k.gid = (uint32_t)(idx - (uint64_t)v * N);
    const DevCam &cam = cams[v];
    const uint2 rc = rect[idx];
    k.rx = rc.x & 0xffff;
    k.ry = rc.x >> 16;
    k.w = (rc.y & 0xffff) - k.rx;
    k.area = k.w * ((rc.y >> 16) - k.ry);
    k.rw = __frcp_rn((float)max(k.w, 1u));
    k.tb = cam.tile_base;
    k.tw = (uint32_t)cam.tiles_x;
    k.W = cam.W;
    k.H = cam.H;
    k.c = cull_geom(rec[(int64_t)idx * 4], rec[(int64_t)idx * 4 + 1]);
}

// Tile q (row-major in the rectangle) of record k, and whether its alpha
// ellipse reaches it.
__device__ __forceinline__ bool walk_hit(const WalkRec &k, uint32_t q, int tile_w, int tile_h, uint32_t &tile)
{
    if (k.area > (uint32_t)kCullMaxTiles) {
        const uint32_t ty = q / k.w, tx = q - ty * k.w;
        tile = k.tb + (k.ry + ty) * k.tw + k.rx + tx;
        return true;
    }
    // q < 1024: (q + 1/2) / w lies at least 1/(2w) from an integer, far more
    // than the rounding of the product with the rounded reciprocal
    const uint32_t ty = (uint32_t)__fmul_rn((float)q + 0.5f, k.rw), tx = q - ty * k.w;
    tile = k.tb + (k.ry + ty) * k.tw + k.rx + tx;
    int bx0, bx1, by0, by1;
    tile_box((int)(k.rx + tx), (int)(k.ry + ty), tile_w, tile_h, k.W, k.H, bx0, bx1, by0, by1);
    return cull_hits(k.c, bx0, bx1, by0, by1);
}

// The binning walk over the depth-sorted records, one wavefront per run of 64:
// the records' rectangles are laid end to end (an inclusive scan of their
// areas), and the wavefront walks that run 64 tiles at a time with every lane
// busy -- each lane finds its record in the scan (stepping through the few
// records a chunk overlaps, else by binary search), reads it from LDS and
// tests its tile against the alpha ellipse.  Per-record counts of
// kept tiles live in LDS.  COUNT: writes the counts (in depth order and back to
// the records).  EMIT: writes each kept tile's (tile, index) pair at the
// record's offset plus the number of kept tiles before it, never past the
// counted slots.  Both modes take bit-identical decisions (same routine, same
// FP32 record).
template <bool EMIT>
__global__ void __launch_bounds__(256) walk_pairs(const DevCam *__restrict__ cams, int64_t N,
                                                  const uint32_t *__restrict__ didx, const uint2 *__restrict__ rect,
                                                  const float4 *__restrict__ rec, int tile_w, int tile_h,
                                                  const DevCounters *__restrict__ cnt, uint32_t *__restrict__ tsorted,
                                                  uint32_t *__restrict__ touched, const uint32_t *__restrict__ poff,
                                                  int64_t cap, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    __shared__ WalkRec srec[4][64];
    __shared__ uint32_t scnt[4][64];
    if (EMIT && cnt->overflow) return;
    const uint32_t R = cnt->R;
    const int lane = __lane_id(), wave = (int)(threadIdx.x >> 6);
    const uint64_t lt = __lanemask_lt();
    const uint64_t wave0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * 256) >> 6;
    WalkRec *wr = srec[wave];
    uint32_t *wc = scnt[wave];
    for (uint64_t base = wave0 * 64; base < R; base += nwaves * 64) {
        const uint64_t r = base + lane;
        WalkRec mine;
        mine.area = 0;
        mine.nt = 0;
        mine.off = 0;
        if (r < R) {
            walk_load(mine, cams, N, didx[r], rect, rec);
            if (EMIT) {
                mine.nt = tsorted[r];
                mine.off = poff[r];
                if ((uint64_t)mine.off + mine.nt > (uint64_t)cap) mine.nt = 0;
                if (mine.nt == 0) mine.area = 0;
            }
        }
        const uint32_t incl = wave_incl_scan(mine.area);
        mine.start = incl - mine.area;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        __builtin_amdgcn_wave_barrier();
        wr[lane] = mine;
        wc[lane] = 0;
        __builtin_amdgcn_wave_barrier();
        int kc = 0;  // first record that ends after t0 (wavefront-uniform)
        for (uint32_t t0 = 0; t0 < total; t0 += 64) {
            const uint32_t t = t0 + (uint32_t)lane;
            const bool valid = t < total;
            // record of position t: the first k with incl[k] > t.  A chunk of
            // 64 positions usually overlaps a few records: step through them
            // with uniform lane reads (no LDS round trip); a chunk that
            // overlaps more than eight takes a binary search instead.
            while (kc < 63 && (uint32_t)__builtin_amdgcn_readlane((int)incl, kc) <= t0) ++kc;
            int kf = kc, kk = kc;
            uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)incl, kc);
            for (int it = 0; it < 8 && e < t0 + 64u && kk < 63; ++it) {
                ++kk;
                kf = t >= e ? kk : kf;
                e = (uint32_t)__builtin_amdgcn_readlane((int)incl, kk);
            }
            if (e < t0 + 64u && kk < 63) {
                int lo = 0, hi = 63;
#pragma unroll
                for (int it = 0; it < 6; ++it) {
                    const int mid = (lo + hi) >> 1;
                    const uint32_t v = (uint32_t)__shfl((int)incl, mid, 64);
                    if (v > t) hi = mid;
                    else lo = mid + 1;
                }
                kf = lo;
            }
            const int k = valid ? kf : 63;
            const WalkRec kr = wr[k];
            uint32_t tile = 0;
            const bool hit = valid && walk_hit(kr, t - kr.start, tile_w, tile_h, tile);
            const uint64_t hm = __ballot(hit);
            // lanes [a, b) of this chunk belong to record k
            const int a = (int)max((int64_t)kr.start - (int64_t)t0, (int64_t)0);
            const int64_t bend = (int64_t)kr.start + kr.area - (int64_t)t0;
            const uint64_t from_a = ~((1ull << a) - 1ull);
            const uint64_t upto_b = bend >= 64 ? ~0ull : ((1ull << bend) - 1ull);
            const uint32_t before = wc[k];
            if (EMIT && hit) {
                const uint32_t slot = before + (uint32_t)__popcll(hm & lt & from_a);
                if (slot < kr.nt) {
                    keys[kr.off + slot] = tile;
                    vals[kr.off + slot] = kr.gid;
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (valid && lane == a) wc[k] = before + (uint32_t)__popcll(hm & from_a & upto_b);
            __builtin_amdgcn_wave_barrier();
        }
        if (!EMIT && r < R) {
            const uint32_t c = wc[lane];
            tsorted[r] = c;
            touched[mine.idx] = c;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Digits of a sort pass: at most kRadixBits bits, kRadix values.
constexpr int kRadixBits = 9, kRadix = 1 << kRadixBits;

// Digit of `width` (<= kRadixBits) bits at `shift`.
template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, int width)
{
    return (uint32_t)(key >> shift) & ((1u << width) - 1u);
}

// Lanes of the wavefront whose digit equals this lane's (`valid` lanes only):
// one ballot per digit bit.  `width` is uniform across the wavefront.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, int width)
{
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < width; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return peers;
}

// The sort runs with one wavefront per block (kSortThreads = 64) and a fixed
// grid of kSortBlocks blocks, each owning a contiguous chunk of the input.  A
// single wavefront per block keeps too few loads in flight to cover HBM latency
// if it walks its chunk 64 keys at a time, so both kernels below load
// kSortUnroll groups of 64 keys before using any of them.
constexpr int kSortUnroll = 8;

// Per-block digit histogram of the block's chunk: one LDS atomic per key, into
// one of kHistCopies copies of the histogram by lane, summed at the end.  The
// digits of a group of 64 keys are often few (the top digit of tile ids that
// are already ordered by their low bits), and lanes adding to one LDS word
// serialise.
constexpr int kHistCopies = 4;

template <typename K>
__global__ void __launch_bounds__(kSortThreads) radix_hist(const K *__restrict__ keys, const uint32_t *__restrict__ n_dev,
                                                           int shift, int width, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[kHistCopies][kRadix];
    for (int d = threadIdx.x; d < kHistCopies * kRadix; d += kSortThreads) (&h[0][0])[d] = 0;
    __syncthreads();
    uint32_t *hc = h[threadIdx.x % kHistCopies];
    const uint32_t P = *n_dev;
    const uint32_t per = ((P + kSortBlocks - 1) / kSortBlocks + 63) & ~63u;
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = min((uint64_t)P, b0 + per);
    for (uint64_t tb = b0; tb < b1; tb += kSortThreads * kSortUnroll) {
        K key[kSortUnroll];
#pragma unroll
        for (int u = 0; u < kSortUnroll; ++u) {
            const uint64_t i = tb + u * kSortThreads + threadIdx.x;
            key[u] = i < b1 ? keys[i] : K(0);
        }
#pragma unroll
        for (int u = 0; u < kSortUnroll; ++u)
            if (tb + u * kSortThreads + threadIdx.x < b1) atomicAdd(&hc[digit_of(key[u], shift, width)], 1u);
    }
    __syncthreads();
    // all kRadix rows (zero past 2^width), so that no row keeps a count of an
    // earlier, wider pass
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kHistCopies; ++k) c += h[k][d];
        hist[(size_t)d * kSortBlocks + blockIdx.x] = c;
    }
}

// One block per digit: exclusive scan of that digit's per-block counts.
__global__ void __launch_bounds__(256) radix_scan_digit(uint32_t *__restrict__ hist, uint32_t *__restrict__ digit_tot)
{
    __shared__ uint32_t lds4[4];
    constexpr int PER = kSortBlocks / 256;
    uint32_t *row = hist + (size_t)blockIdx.x * kSortBlocks;
    uint32_t v[PER], s = 0;
    for (int k = 0; k < PER; ++k) {
        v[k] = row[threadIdx.x * PER + k];
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan256(s, lds4, tot);
    for (int k = 0; k < PER; ++k) {
        row[threadIdx.x * PER + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = tot;
}

// Stable scatter of one block's chunk, in tiles of 256 ROUNDS keys.  Each of
// the four wavefronts ranks its quarter of the tile 64 keys at a time (a key's
// rank among equal digits below it in the wavefront comes from one ballot per
// digit bit, plus the wavefront's running per-digit count in LDS); the
// per-digit counts of the four wavefronts and of the tile are then scanned
// (thread t owns digits 2t and 2t + 1), every key is placed at its
// digit-sorted position in an LDS copy of the tile, and the tile is written out
// in that order, so each digit's run of keys leaves as consecutive addresses
// instead of as scattered single words.
constexpr int kScatThreads = 256;
static_assert(kRadix == 2 * kScatThreads, "two digits per scatter thread");

// ROUNDS: 64-key rounds per wavefront and tile (tile = 256 ROUNDS keys).  16
// (4096 keys, four blocks per CU) in general; 32 (8192 keys, two blocks per
// CU) for the first pass of the tile sort, whose digits arrive in random
// order: twice the keys per tile double each digit's output run (2.8 against
// 3.1 ms over 409M pairs; the second pass, whose input is ordered by the low
// digit, is faster with the smaller tile: 2.4 against 2.8 ms).
template <typename K, int ROUNDS>
__global__ void __launch_bounds__(kScatThreads) __attribute__((amdgpu_waves_per_eu(ROUNDS > 16 ? 2 : 4)))
radix_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
              uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev, int shift, int width,
              const uint32_t *__restrict__ hist, const uint32_t *__restrict__ digit_tot)
{
    constexpr int kScatRounds = ROUNDS;
    constexpr int kScatTile = kScatThreads * kScatRounds;  // keys per tile
    constexpr int kScatQuarter = kScatTile / 4;            // keys per wavefront and tile
    // (counts and offsets within a tile fit 16 bits; a digit's tile total is
    // the difference of neighbouring offsets: 39,952 bytes in all at 16
    // rounds, four blocks per CU)
    __shared__ uint32_t gbase[kRadix], lds4[4];
    __shared__ uint16_t loff[kRadix], wcnt[4][kRadix];
    __shared__ K skey[kScatTile];
    __shared__ uint32_t sval[kScatTile];
    const int t = threadIdx.x, lane = __lane_id(), wave = t >> 6;
    const int d0 = 2 * t, d1 = 2 * t + 1;
    {
        // global start of each digit's run for this block
        uint32_t total;
        const uint32_t a0 = digit_tot[d0], a1 = digit_tot[d1];
        const uint32_t ex = block_excl_scan256(a0 + a1, lds4, total);
        gbase[d0] = ex + hist[(size_t)d0 * kSortBlocks + blockIdx.x];
        gbase[d1] = ex + a0 + hist[(size_t)d1 * kSortBlocks + blockIdx.x];
    }
    const uint32_t P = *n_dev;
    const uint32_t per = ((P + kSortBlocks - 1) / kSortBlocks + 63) & ~63u;
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = min((uint64_t)P, b0 + per);
    const uint64_t lt = __lanemask_lt();
    for (uint64_t ts = b0; ts < b1; ts += kScatTile) {
        const uint32_t nt = (uint32_t)min((uint64_t)kScatTile, b1 - ts);
        for (int d = lane; d < kRadix; d += 64) wcnt[wave][d] = 0;
        K key[kScatRounds];
        uint32_t val[kScatRounds], pw[kScatRounds];
#pragma unroll
        for (int i = 0; i < kScatRounds; ++i) {
            const uint32_t li = (uint32_t)(wave * kScatQuarter + i * 64 + lane);
            key[i] = li < nt ? kin[ts + li] : K(0);
            val[i] = li < nt ? vin[ts + li] : 0u;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kScatRounds; ++i) {
            const uint32_t li = (uint32_t)(wave * kScatQuarter + i * 64 + lane);
            const bool valid = li < nt;
            const uint32_t d = digit_of(key[i], shift, width);
            const uint64_t peers = digit_peers(d, valid, width);
            const uint32_t rank = __popcll(peers & lt);
            pw[i] = valid ? (uint32_t)wcnt[wave][d] + rank : 0u;
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) wcnt[wave][d] = (uint16_t)(wcnt[wave][d] + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        {
            // per digit: offsets of the four wavefronts' keys, tile total, local start
            uint32_t td[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int d = d0 + k;
                const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
                wcnt[0][d] = 0;
                wcnt[1][d] = (uint16_t)c0;
                wcnt[2][d] = (uint16_t)(c0 + c1);
                wcnt[3][d] = (uint16_t)(c0 + c1 + c2);
                td[k] = c0 + c1 + c2 + c3;
            }
            uint32_t total;
            const uint32_t ex = block_excl_scan256(td[0] + td[1], lds4, total);
            loff[d0] = (uint16_t)ex;
            loff[d1] = (uint16_t)(ex + td[0]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScatRounds; ++i) {
            const uint32_t li = (uint32_t)(wave * kScatQuarter + i * 64 + lane);
            if (li < nt) {
                const uint32_t d = digit_of(key[i], shift, width);
                const uint32_t lp = (uint32_t)loff[d] + wcnt[wave][d] + pw[i];
                skey[lp] = key[i];
                sval[lp] = val[i];
            }
        }
        __syncthreads();
        for (uint32_t i = (uint32_t)t; i < nt; i += kScatThreads) {
            const K k = skey[i];
            const uint32_t d = digit_of(k, shift, width);
            const uint32_t g = gbase[d] + (i - (uint32_t)loff[d]);
            kout[g] = k;
            vout[g] = sval[i];
        }
        __syncthreads();
        const uint32_t o0 = loff[d0], o1 = loff[d1], o2 = d1 + 1 < kRadix ? (uint32_t)loff[d1 + 1] : nt;
        gbase[d0] += o1 - o0;
        gbase[d1] += o2 - o1;
        __syncthreads();
    }
}

// Four sorted keys per thread (one 16-byte load; the neighbours across the
// group boundary come from the same cache lines as the adjacent threads' loads).
__global__ void __launch_bounds__(256) tile_ranges(const uint32_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ n_dev, uint2 *__restrict__ ranges)
{
    const uint64_t P = *n_dev;
    for (uint64_t b = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 4; b < P; b += (uint64_t)gridDim.x * 256 * 4) {
        uint32_t k[6];  // keys b-1 .. b+4 (sentinels beyond the ends)
        if (b + 4 <= P) {
            const uint4 q = *reinterpret_cast<const uint4 *>(keys + b);
            k[1] = q.x, k[2] = q.y, k[3] = q.z, k[4] = q.w;
        } else {
            for (int j = 0; j < 4; ++j) k[1 + j] = b + j < P ? keys[b + j] : 0xffffffffu;
        }
        k[0] = b > 0 ? keys[b - 1] : 0xffffffffu;
        k[5] = b + 4 < P ? keys[b + 4] : 0xffffffffu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t i = b + j;
            if (i >= P) break;
            const uint32_t tile = k[1 + j];
            if (i == 0 || k[j] != tile) ranges[tile].x = (uint32_t)i;
            if (i + 1 == P || k[2 + j] != tile) ranges[tile].y = (uint32_t)(i + 1);
        }
    }
}

__global__ void __launch_bounds__(256) fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

void scan(const ScanIn &si, int nb, uint32_t *part, uint32_t *out, int64_t cap, uint32_t *total, uint32_t *overflow,
          uint32_t *usable, DevCounters *reset, hipStream_t s)
{
    hipLaunchKernelGGL(scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, si, part);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, part, nb, cap, total, overflow, usable, reset);
    hipLaunchKernelGGL(scan_down, dim3(nb), dim3(kScanThreads), 0, s, si, (const uint32_t *)part, out);
}

// Sorts (keys, vals) in place over bits [0, bits); returns the buffer index
// (0: k0/v0, 1: k1/v1) holding the result.  Passes of at most 9 bits, split
// evenly (17 bits: 8 + 9, not 9 + 8): a scatter pass writes one run per digit
// and LDS tile, so the first pass, whose digits come in random order, gets the
// narrower digit and (with wide_first) the larger tile.
template <typename K>
int radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const uint32_t *n_dev, int bits, uint32_t *hist,
               uint32_t *dtot, bool wide_first, hipStream_t s)
{
    K *k[2] = {k0, k1};
    uint32_t *v[2] = {v0, v1};
    int cur = 0;
    const int passes = radix_passes(bits);
    for (int p = 0, shift = 0; p < passes; ++p) {
        // even split, the wider digits last: the first pass sees digits in
        // random order (its output runs are shortest), the last only the few
        // top-digit values that the key range reaches
        const int width = (bits - shift) / (passes - p);
        hipLaunchKernelGGL(radix_hist<K>, dim3(kSortBlocks), dim3(kSortThreads), 0, s, (const K *)k[cur], n_dev, shift,
                           width, hist);
        hipLaunchKernelGGL(radix_scan_digit, dim3(kRadix), dim3(256), 0, s, hist, dtot);
        auto scat = wide_first && p == 0 ? radix_scatter<K, 32> : radix_scatter<K, 16>;
        hipLaunchKernelGGL(scat, dim3(kSortBlocks), dim3(kScatThreads), 0, s, (const K *)k[cur],
                           (const uint32_t *)v[cur], k[cur ^ 1], v[cur ^ 1], n_dev, shift, width,
                           (const uint32_t *)hist, (const uint32_t *)dtot);
        shift += width;
        cur ^= 1;
    }
    return cur;
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

hipError_t launch_scan_flags(const uint32_t *flags, int64_t n, uint32_t *part, uint32_t *out, uint32_t *total,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int nb = (int)((n + kScanBlock - 1) / kScanBlock);
    scan(ScanIn{flags, n, nullptr, 1}, nb, part, out, -1, total, nullptr, nullptr, nullptr, s);
    return hipGetLastError();
}

hipError_t launch_binsort(const Problem &pb, const WsLayout &L, char *ws, hipStream_t s, int *final_buf)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto touched = (uint32_t *)(ws + L.touched);
    auto voff = (uint32_t *)(ws + L.voff);
    auto poff = (uint32_t *)(ws + L.poff);
    auto tsorted = (uint32_t *)(ws + L.tsorted);
    auto part = (uint32_t *)(ws + L.scan_part);
    auto cnt = (DevCounters *)(ws + L.counters);
    auto rect = (const uint2 *)(ws + L.rect);
    auto rec = (const float4 *)(ws + L.rec);
    auto dk0 = (uint32_t *)(ws + L.dkey0), dk1 = (uint32_t *)(ws + L.dkey1);
    auto di0 = (uint32_t *)(ws + L.didx0), di1 = (uint32_t *)(ws + L.didx1);
    auto k0 = (uint32_t *)(ws + L.keys0), k1 = (uint32_t *)(ws + L.keys1);
    auto v0 = (uint32_t *)(ws + L.vals0), v1 = (uint32_t *)(ws + L.vals1);
    auto hist = (uint32_t *)(ws + L.hist);
    auto dtot = (uint32_t *)(ws + L.digit_tot);
    auto ranges = (uint2 *)(ws + L.ranges);
    const int64_t VN = L.VN;
    const unsigned vn_blocks = (unsigned)((VN + 255) / 256 > 0 ? (VN + 255) / 256 : 1);
    const unsigned gs_blocks = vn_blocks < 8192 ? vn_blocks : 8192;
    hipError_t e;

    // 1. compact visible records
    scan(ScanIn{touched, VN, nullptr, 1}, L.nb_scan, part, voff, -1, &cnt->R, nullptr, nullptr, cnt, s);
    if (VN > 0)
        hipLaunchKernelGGL(compact_visible, dim3(vn_blocks), dim3(256), 0, s, L.N, VN, (const uint32_t *)touched,
                           (const uint32_t *)voff, (const uint32_t *)dk1, dk0, di0);
    // 2. sort by depth
    const int dcur = radix_sort<uint32_t>(dk0, di0, dk1, di1, &cnt->R, L.depth_bits, hist, dtot, false, s);
    uint32_t *didx = dcur ? di1 : di0;
    // 3. tile counts in depth order, pair offsets, emission
    hipLaunchKernelGGL(walk_pairs<false>, dim3(gs_blocks), dim3(256), 0, s, cams, L.N, (const uint32_t *)didx, rect,
                       rec, pb.tile_w, pb.tile_h, (const DevCounters *)cnt, tsorted, touched, (const uint32_t *)poff,
                       (int64_t)0, k0, v0);
    scan(ScanIn{tsorted, VN, &cnt->R, 0}, L.nb_scan, part, poff, L.pair_cap, &cnt->P, &cnt->overflow, &cnt->P_eff,
         nullptr, s);
    hipLaunchKernelGGL(walk_pairs<true>, dim3(gs_blocks), dim3(256), 0, s, cams, L.N, (const uint32_t *)didx, rect,
                       rec, pb.tile_w, pb.tile_h, (const DevCounters *)cnt, tsorted, touched, (const uint32_t *)poff,
                       L.pair_cap, k0, v0);
    // 4. stable sort of the pairs by tile
    const int cur = radix_sort<uint32_t>(k0, v0, k1, v1, &cnt->P_eff, L.tile_bits, hist, dtot, true, s);
    // 5. ranges
    if ((e = launch_fill_u32((uint32_t *)ranges, 0u, 2 * L.total_tiles, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(tile_ranges, dim3(4096), dim3(256), 0, s, (const uint32_t *)(cur ? k1 : k0),
                       (const uint32_t *)&cnt->P_eff, ranges);
    *final_buf = cur;
    return hipGetLastError();
}

hipError_t launch_gauss_major_list(const WsLayout &L, char *ws, int V, hipStream_t s)
{
    const int64_t N = L.N;
    if (N <= 0) return hipSuccess;
    auto touched = (const uint32_t *)(ws + L.touched);
    auto count = (uint32_t *)(ws + L.tsorted);
    auto off = (uint32_t *)(ws + L.poff);
    auto part = (uint32_t *)(ws + L.scan_part);
    auto cnt = (DevCounters *)(ws + L.counters);
    const unsigned blocks = (unsigned)((N + 255) / 256);
    const int nb = (int)((N + kScanBlock - 1) / kScanBlock);  // <= L.nb_scan (N <= V N)
    hipLaunchKernelGGL(gauss_views, dim3(blocks), dim3(256), 0, s, N, V, touched, count);
    scan(ScanIn{count, N, nullptr, 0}, nb, part, off, -1, &cnt->R_gauss, nullptr, nullptr, nullptr, s);
    hipLaunchKernelGGL(gauss_emit, dim3(blocks), dim3(256), 0, s, N, V, touched, (const uint32_t *)off,
                       (uint32_t *)(ws + L.vlist));
    return hipGetLastError();
}

}  // namespace ugs
