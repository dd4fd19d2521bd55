// Stages S5 and S8 for 9..256 semantic channels, with the two contractions of
// Eq. semantic_render (O~[p][c] = sum_f w_f[p] o_f[c]) and of Eq. gradiento
// (dO[f][c] = sum_p w_f[p] G_p[c]), plus the semantic part of the alpha
// gradient of Alg. backward_render (S[f][p] = sum_c o_f[c] G_p[c]), on the FP32
// matrix cores (v_mfma_f32_16x16x4_f32: FP32 products, FP32 accumulation).
//
// The compositing walk is the per-pixel walk of the plain kernels (one
// workgroup per (view, tile), one lane per pixel, the tile's sorted list staged
// in LDS batch by batch, T and the depth accumulated in FP64).  What changes is
// how the channel work is done:
//
//  * Active entries only.  A list entry is "active" for a wavefront when at
//    least one of its 64 pixels takes it (alpha >= 1/255 before termination).
//    Only active entries enter the matrix products.  The forward appends each
//    active entry's weights to a per-wavefront LDS buffer and multiplies every
//    4 of them (the MFMA's K) into the accumulators; it also records, per
//    wavefront, one bit per list entry (the activity mask in the workspace).
//    The backward reads that mask and walks only the marked entries, in groups
//    of 16 (the MFMA's M): S for the group, the reverse walk, dO.  On gfx950
//    the FP32 matrix instructions share the FP32 datapath with the vector ALU
//    (they do not co-issue, unlike the bf16 ones), so every matrix product
//    spent on an idle entry would cost vector time.
//  * Channel chunks.  A pass covers CCH channels (forward: up to 64, held as
//    CCH accumulators per lane; backward: 32 or 64, whose upstream gradients
//    live in registers in the two operand layouts the products need).  Wider C_o runs
//    further passes over the same lists with a channel offset: a forward pass
//    recovers the weights and adds only its channels (in a training forward it
//    visits only the entries of the first pass's activity mask, each pixel up
//    to its contributor count; otherwise it repeats the walk); a backward
//    chunk pass adds the chunk's dO and its share of the alpha
//    gradient (the alpha gradient is linear in the semantic upstream, so the
//    chunks' shares add up to the full one: dL/dalpha_i = T_i s_i -
//    A_i / (1 - alpha_i) with s_i and A_i sums over channels).
#include <algorithm>

#include "render_common.h"



namespace ugs {
namespace {

typedef float mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mma(float a, float b, mf4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Float add to an LDS word (no return value needed).
__device__ __forceinline__ void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}


constexpr int kFRows = 4;   // active entries per forward product (the MFMA's K)
constexpr int kFwdMaxBatch = 128;  // forward batch bound (ids held in two lane registers)
constexpr int kFwdFmax = 4;        // forward staging: feature loads per lane in flight
constexpr int kBGrp = 16;   // active entries per backward group (the MFMA's M)
constexpr int kSW = 68;     // floats per row of the per-wavefront S / w buffer

__host__ __device__ constexpr int feat_stride(int CCH) { return CCH + 4; }

// LDS bytes of the forward kernel for `batch` entries, CCH channels per pass,
// NW wavefronts.
__host__ __device__ constexpr size_t fwd_mm_lds(int batch, int CCH, int NW, bool hit)
{
    return (size_t)batch * (64 + 4 * feat_stride(CCH) + (hit ? 4 : 0)) + (size_t)NW * kFRows * 64 * 4;
}

// LDS bytes of the backward kernel (channel passes after the first hold a
// second per-wavefront row buffer, for dpow and the moments).
__host__ __device__ constexpr size_t bwd_mm_lds(int batch, int CCH, int NW, bool hit, bool main)
{
    return (size_t)batch * (64 + 4 * feat_stride(CCH) + 8 + (hit ? 4 : 0) + 64) +
           (size_t)(main ? 1 : 2) * NW * kBGrp * kSW * 4;
}

// Loads n floats from LDS (n = 1, 2, 4 or 8; 4-float aligned when n >= 4).
template <int NF>
__device__ __forceinline__ void lds_row(const float *p, float (&x)[NF])
{
    if constexpr (NF >= 4) {
#pragma unroll
        for (int k = 0; k < NF / 4; ++k) {
            const float4 t = reinterpret_cast<const float4 *>(p)[k];
            x[4 * k] = t.x;
            x[4 * k + 1] = t.y;
            x[4 * k + 2] = t.z;
            x[4 * k + 3] = t.w;
        }
    } else if constexpr (NF == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        x[0] = t.x;
        x[1] = t.y;
    } else {
        x[0] = p[0];
    }
}

// The semantic share of one reverse step (backward channel passes after the
// first): the same T restoration and weight as frag_adjoint, s_i = s_sem (this
// pass's part of the dot product of the upstream gradients with the
// fragment's values) and A this pass's running sum.  Returns the weight w and
// sets dpow = dL/d(o G) of this share (zero through the 0.99 clamp): every
// record slot it reaches (mean2d, Cholesky conic, opacity) is dpow times a
// polynomial of degree <= 2 in the pixel offset.
__device__ __forceinline__ float frag_weight_sem(bool contrib, float alpha, float oG, float s_sem, double &T,
                                                 float &A, float &dpow)
{
    const float rom = rcp_nr(1.f - alpha);
    const double Tn = contrib ? T * rcp64(1.0 - (double)alpha) : T;
    const float w = contrib ? (float)((double)alpha * Tn) : 0.f;
    const float dalpha = contrib ? (float)Tn * s_sem - A * rom : 0.f;
    A += w * s_sem;
    T = Tn;
    dpow = oG < kAlphaMax ? dalpha * oG : 0.f;
    return w;
}

// Ids of a batch's entries, held in lane registers (lane l: entries l, 64 + l,
// ...), so that a batch's staging loads need no id load of their own and can
// all be in flight at once.
template <int MAXB>
struct BatchIds {
    static constexpr int R = (MAXB + 63) / 64;
    uint32_t v[R];
    __device__ __forceinline__ void load(const uint32_t *vals, uint32_t s0, int nn, int lane)
    {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = 64 * r + lane < nn ? vals[s0 + 64 * r + lane] : 0u;
    }
    // id of entry e (< MAXB); every lane of the wavefront must take part
    __device__ __forceinline__ uint32_t at(int e) const
    {
        uint32_t x = (uint32_t)__shfl((int)v[0], e & 63, 64);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const uint32_t y = (uint32_t)__shfl((int)v[r], e & 63, 64);
            x = (e >> 6) == r ? y : x;
        }
        return x;
    }
};

// Stages the n (<= MAXB) entries of a batch whose ids are in `ids`: the first
// NR float4 of their 64 B records (4: all; 2: mean2d, conic factor, opacity, k
// and z0, all that the alpha test needs) at a stride of 4 float4, the CCH
// feature channels [c0, c0 + CCH) (zero beyond C_o) in rows of
// feat_stride(CCH) floats, and with HIT the hit constants.  The loads go out
// in groups of up to FMAX per lane (registers) before their LDS writes.
template <int NT, int CCH, int NR, int FMAX, int MAXB, bool HIT>
__device__ __forceinline__ void stage_ids(float4 *srec, float *sfeat, float *shh, const BatchIds<MAXB> &ids, int n,
                                          const float4 *rec, int64_t recbase, const float *sem, int C_o, int c0,
                                          const float *hrec)
{
    // Items past the batch (or past a lane's share) load and store the last
    // entry's item again (same value to the same slot): no branches around the
    // loads or stores, which the compiler would otherwise sink into per-item
    // conditional blocks, one round trip each.
    constexpr int FS = feat_stride(CCH);
    constexpr int RPT = (MAXB * NR + NT - 1) / NT, FPT = (MAXB * CCH + NT - 1) / NT;
    constexpr int RCH = RPT < 4 ? RPT : 4, FCH = FPT < FMAX ? FPT : FMAX;
    const int t = (int)threadIdx.x;
#pragma unroll 1
    for (int i0 = 0; i0 < RPT && NT * i0 < n * NR; i0 += RCH) {
        float4 rr[RCH];
#pragma unroll
        for (int u = 0; u < RCH; ++u) {
            const int q = t + NT * (i0 + u), e = min(q / NR, n - 1), k = q % NR;
            rr[u] = rec[(recbase + ids.at(e)) * 4 + k];
        }
#pragma unroll
        for (int u = 0; u < RCH; ++u) {
            const int q = t + NT * (i0 + u), e = min(q / NR, n - 1), k = q % NR;
            srec[4 * e + k] = rr[u];
        }
    }
#pragma unroll 1
    for (int i0 = 0; i0 < FPT && NT * i0 < n * CCH; i0 += FCH) {
        float ff[FCH];
#pragma unroll
        for (int u = 0; u < FCH; ++u) {
            const int q = t + NT * (i0 + u), e = min(q / CCH, n - 1), c = q % CCH;
            const float x = sem[(int64_t)ids.at(e) * C_o + min(c0 + c, C_o - 1)];
            ff[u] = c0 + c < C_o ? x : 0.f;
        }
#pragma unroll
        for (int u = 0; u < FCH; ++u) {
            const int q = t + NT * (i0 + u), e = min(q / CCH, n - 1), c = q % CCH;
            sfeat[e * FS + c] = ff[u];
        }
    }
    if constexpr (HIT) {
#pragma unroll 1
        for (int e0 = 0; e0 < n; e0 += NT) {
            const int e = min(e0 + t, n - 1);
            shh[e] = hrec[recbase + ids.at(e)];
        }
    }
}

// ------------------------------------------------------------------ forward
// Per wavefront, the accumulators hold O~ transposed in the MFMA output layout:
// acc[q][pb][r] is channel c0 + CPL (4 (lane / 16) + r) + q of pixel
// 16 pb + lane % 16 (pixels numbered row-major in the wavefront's 8 x 8
// block), CPL = CCH / 16.  Product: A[m][k] = o_{row k}[c0 + CPL m + q] (each
// lane reads CPL consecutive floats of one staged feature row), B[k][n] =
// w_{row k}[pixel 16 pb + n] (one 16-byte LDS read gives the four pixel
// blocks), K = the 4 buffered active entries.  MAIN passes also composite
// colour, depth and the gradient factor, write T_final / n_contrib and the
// counters; other passes (C_o > CCH) only add their channels.
template <int TW, int TH, int CCH, int DM, bool MAIN>
__global__ void __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(4))) render_fwd_mm_kernel(
    const DevCam *__restrict__ cams, int V, int64_t N, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const float4 *__restrict__ rec, const float *__restrict__ sem, int C_o, int c0,
    ugs_outputs out, int batch, DevCounters *__restrict__ cnt, int count, uint32_t ntiles,
    const float *__restrict__ hrec, int half_out, uint32_t *__restrict__ amask, int64_t mwords,
    unsigned long long *__restrict__ tclk)
{
    static_assert(CCH == 16 || CCH == 32 || CCH == 64, "forward pass: 16, 32 or 64 channels");
    constexpr int NT = TW * TH, NW = NT / 64, FS = feat_stride(CCH), CPL = CCH / 16;
    constexpr bool HIT = DM == 2;
    constexpr float kd = DM == 1 ? 0.f : 1.f;  // depth form fixed per instantiation
    extern __shared__ float4 smem[];
    float4 *srec = smem;
    float *sfeat = (float *)(smem + 4 * batch);
    float *shh = sfeat + (size_t)batch * FS;
    float *wb = shh + (HIT ? batch : 0) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * (kFRows * 64);  // [row][lane % 16][pixel block]
    (void)NW;
    const uint32_t slot = xcd_tile(blockIdx.x, ntiles);
    if (slot >= ntiles) return;
    const TileInfo ti = tile_info<TW, TH>(cams, V, slot);
    const uint32_t tile = ti.tile;
    if (tclk && threadIdx.x == 0) tclk[2 * tile] = __builtin_amdgcn_s_memrealtime();
    const uint2 range = ranges[tile];
    const float fx = (float)ti.px, fy = (float)ti.py;
    const int64_t recbase = (int64_t)ti.v * N;
    const int lane = __lane_id(), l16 = lane & 15, h16 = lane >> 4;
    const int wslot = l16 * 4 + h16;  // this lane's pixel (16 h16 + l16) in a row of wb

    double T = 1.0, D = 0.0;
    float cr = 0.f, cg = 0.f, cb = 0.f, K = 0.f;
    mf4 acc[CPL][4];
#pragma unroll
    for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) acc[q][pb] = mf4{0.f, 0.f, 0.f, 0.f};
    uint32_t last = 0, n_eval = 0, n_con = 0;
    bool done = !ti.inside;
    // activity mask of this wavefront (MAIN passes of training steps): bits of
    // the current 32-entry word, flushed with one atomic OR per word
    uint32_t *mplane = amask ? amask + (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * mwords : nullptr;
    uint32_t mbits = 0;
    int64_t mword = -1;
    auto mflush = [&]() {
        if (mbits && lane == 0) atomicOr(&mplane[mword], mbits);
        mbits = 0;
    };

    // the weights' matrix product for the nrow buffered rows (rows past nrow
    // zeroed first)
    auto flush_rows = [&](int nrow, int rid) {
        for (int r = nrow; r < kFRows; ++r) wb[r * 64 + wslot] = 0.f;
        __builtin_amdgcn_wave_barrier();
        const float4 bw = *reinterpret_cast<const float4 *>(wb + h16 * 64 + l16 * 4);
        float a[CPL];
        lds_row<CPL>(sfeat + rid * FS + CPL * l16, a);
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            acc[q][0] = mma(a[q], bw.x, acc[q][0]);
            acc[q][1] = mma(a[q], bw.y, acc[q][1]);
            acc[q][2] = mma(a[q], bw.z, acc[q][2]);
            acc[q][3] = mma(a[q], bw.w, acc[q][3]);
        }
        __builtin_amdgcn_wave_barrier();
    };

    if (!MAIN && amask) {
        // A further channel pass of a forward that keeps the backward's state:
        // the first pass has left this wavefront's activity mask and every
        // pixel's contributor count, so the walk visits only the marked
        // entries and stops each pixel at its count.  The weights are the
        // first pass's (same alpha, same FP64 transmittance updates in the
        // same order); entries no lane takes change no weight.
        uint32_t lastp = 0;
        if (ti.inside) {
            const uint32_t rel = out.n_contrib[ti.off + ti.pix];
            lastp = rel ? range.x + rel : 0u;
        }
        __shared__ uint32_t s_end;
        if (threadIdx.x == 0) s_end = 0;
        __syncthreads();
        if (lastp) atomicMax(&s_end, lastp);
        __syncthreads();
        const uint32_t end_all = s_end;
        // ids and mask words (lanes 0..4) of the batch at s0, one batch ahead
        BatchIds<kFwdMaxBatch> nid;
        uint32_t nmk = 0;
        auto prefetch = [&](uint32_t s0) {
            const int nn = (int)min((uint32_t)batch, end_all - s0);
            nid.load(vals, s0, nn, lane);
            nmk = lane < (nn > 64 ? 5 : 3) ? mplane[(s0 >> 5) + lane] : 0u;
        };
        if (range.x < end_all) prefetch(range.x);
        for (uint32_t start = range.x; start < end_all; start += (uint32_t)batch) {
            const int n = (int)min((uint32_t)batch, end_all - start);
            const BatchIds<kFwdMaxBatch> cid = nid;
            const uint32_t cmk = nmk;
            __syncthreads();
            stage_ids<NT, CCH, 2, kFwdFmax, kFwdMaxBatch, false>(srec, sfeat, nullptr, cid, n, rec, recbase, sem, C_o,
                                                                 c0, hrec);
            __syncthreads();
            if (start + (uint32_t)batch < end_all) prefetch(start + (uint32_t)batch);
            int nrow = 0, rid = 0;
            for (int w0 = 0; w0 < n; w0 += 64) {
                // mask bits of entries start + w0 .. start + w0 + 63
                const uint32_t e0 = start + (uint32_t)w0;
                const int wi = (int)((e0 >> 5) - (start >> 5));
                const uint32_t m0 = __builtin_amdgcn_readlane(cmk, wi), m1 = __builtin_amdgcn_readlane(cmk, wi + 1),
                               m2 = __builtin_amdgcn_readlane(cmk, wi + 2);
                const int sh = (int)(e0 & 31);
                const uint64_t lo = ((uint64_t)m1 << 32) | m0;
                uint64_t m = sh ? (lo >> sh) | ((uint64_t)m2 << (64 - sh)) : lo;
                if (n - w0 < 64) m &= (1ull << (n - w0)) - 1ull;
                // (readfirstlane returns int: widen through uint32_t, or bit 31
                // would be sign-extended into phantom entries 32..63)
                m = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32) |
                    (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)m);
                // the next marked entry's record is read while this one is
                // used (an empty mask names the batch's last entry instead)
                auto next_of = [&](uint64_t mm) { return min(w0 + (int)__builtin_ctzll(mm | (1ull << 63)), n - 1); };
                int jn = next_of(m);
                float4 n0 = srec[4 * jn], n1 = srec[4 * jn + 1];
                while (m) {
                    const int j = jn;
                    const float4 r0 = n0, r1 = n1;
                    m &= m - 1ull;
                    jn = next_of(m);
                    n0 = srec[4 * jn];
                    n1 = srec[4 * jn + 1];
                    const float dx = fx - r0.x, dy = fy - r0.y;
                    const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                    const float alpha = fminf(kAlphaMax, r1.y * gauss_of(t1, t2));
                    float wf = 0.f;
                    if (start + (uint32_t)j < lastp && alpha >= kAlphaMin) {
                        wf = (float)((double)alpha * T);
                        T = T * (1.0 - (double)alpha);
                    }
                    wb[nrow * 64 + wslot] = wf;
                    rid = h16 == nrow ? j : rid;
                    if (++nrow == kFRows) {
                        flush_rows(nrow, rid);
                        nrow = 0;
                    }
                }
            }
            if (nrow) flush_rows(nrow, rid);
        }
    }

    const bool walk_all = MAIN || !amask;
    BatchIds<kFwdMaxBatch> nid;  // ids of the next batch, loaded one batch ahead
    if (walk_all && range.x < range.y) nid.load(vals, range.x, (int)min((uint32_t)batch, range.y - range.x), lane);
    for (uint32_t start = range.x; start < range.y && walk_all; start += (uint32_t)batch) {
        if (__syncthreads_count(done) == NT) break;
        const int n = (int)min((uint32_t)batch, range.y - start);
        const BatchIds<kFwdMaxBatch> cid = nid;
        stage_ids<NT, CCH, MAIN ? 4 : 2, kFwdFmax, kFwdMaxBatch, HIT && MAIN>(srec, sfeat, shh, cid, n, rec, recbase,
                                                                            sem, C_o, c0, hrec);
        __syncthreads();
        if (start + (uint32_t)batch < range.y)
            nid.load(vals, start + (uint32_t)batch, (int)min((uint32_t)batch, range.y - start - (uint32_t)batch), lane);
        if (__all(done)) continue;  // the other wavefronts may still walk this batch
        int nrow = 0;
        int rid = 0;  // lane l: batch index of buffered row l / 16
        for (int j = 0; j < n; ++j) {
            float wf = 0.f;
            if (!done) {
                const float4 r0 = srec[4 * j], r1 = srec[4 * j + 1];
                const float dx = fx - r0.x, dy = fy - r0.y;
                const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                const float alpha = fminf(kAlphaMax, r1.y * gauss_of(t1, t2));
                ++n_eval;
                if (alpha >= kAlphaMin) {
                    const double tT = T * (1.0 - (double)alpha);
                    if (tT < kTStop) {
                        done = true;
                    } else {
                        const double w = (double)alpha * T;
                        wf = (float)w;
                        if constexpr (MAIN) {
                            const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
                            const float kdj = frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy);
                            const float B = kdj * (r2.x * dx + r2.y * dy);
                            const float Cq = kdj * (r2.z * dx * dx + 2.f * r2.w * dx * dy + r3.x * dy * dy);
                            const float d = r1.w * (1.f + B) * rcp_nr(1.f + 2.f * B + Cq);
                            cr += wf * r3.y;
                            cg += wf * r3.z;
                            cb += wf * r3.w;
                            K += wf * r1.z;
                            D += w * (double)d;
                        }
                        T = tT;
                        last = start + (uint32_t)j + 1;
                        ++n_con;
                    }
                }
            }
            if (__any(wf != 0.f)) {  // an active entry: buffer its weights
                if constexpr (MAIN) {
                    if (mplane) {
                        const uint32_t e = start + (uint32_t)j;
                        if ((int64_t)(e >> 5) != mword) {
                            mflush();
                            mword = e >> 5;
                        }
                        mbits |= 1u << (e & 31);
                    }
                }
                wb[nrow * 64 + wslot] = wf;
                rid = h16 == nrow ? j : rid;
                if (++nrow == kFRows) {
                    flush_rows(nrow, rid);
                    nrow = 0;
                }
            }
            if (__all(done)) break;
        }
        if (nrow) flush_rows(nrow, rid);  // the batch's remaining rows, padded with zero weights
    }
    if constexpr (MAIN) {
        if (mplane) mflush();
        if (ti.inside) {
            const int64_t p = ti.pix, HW = ti.HW, off = ti.off;
            put_out(out.rgb, 3 * off + p, cr, half_out);
            put_out(out.rgb, 3 * off + HW + p, cg, half_out);
            put_out(out.rgb, 3 * off + 2 * HW + p, cb, half_out);
            out.depth[off + p] = (float)D;
            put_out(out.kmap, off + p, K, half_out);
            if (out.T_final) out.T_final[off + p] = (float)T;  // optional in forward-only use
            if (out.n_contrib) out.n_contrib[off + p] = last ? last - range.x : 0u;
        }
    }
    {
        // value (q, r) of a lane is channel cl + CPL r + q: one base address
        // per pixel block advanced by the (wavefront-uniform) plane size per
        // channel, and the output type chosen once for all the stores
        const int W = cams[ti.v].W, H = cams[ti.v].H;
        const int qx0 = ti.px - (lane & 7), qy0 = ti.py - (lane >> 3);
        const int cl = c0 + CPL * 4 * h16, nc = C_o - cl;
        const int64_t HW = ti.HW;
        auto store_all = [&](auto *dst) {
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                const int pp = 16 * pb + l16;
                const int x = qx0 + (pp & 7), y = qy0 + (pp >> 3);
                if (x < W && y < H) {
                    auto *b = dst + ((int64_t)C_o * ti.off + (int64_t)cl * HW + (int64_t)y * W + x);
#pragma unroll
                    for (int k = 0; k < 4 * CPL; ++k, b += HW)  // channel cl + k
                        if (k < nc) *b = acc[k % CPL][pb][k / CPL];
                }
            }
        };
        if (half_out)
            store_all(reinterpret_cast<_Float16 *>(out.sem));
        else
            store_all(out.sem);
    }
    if (tclk) {
        __syncthreads();
        if (threadIdx.x == 0) tclk[2 * tile + 1] = __builtin_amdgcn_s_memrealtime();
    }
    if constexpr (MAIN) {
        if (count) {
            unsigned long long e = n_eval, c = n_con;
            for (int o = 32; o > 0; o >>= 1) {
                e += __shfl_xor(e, o, 64);
                c += __shfl_xor(c, o, 64);
            }
            if (lane == 0) {
                atomicAdd(&cnt->n_eval, e);
                atomicAdd(&cnt->n_contrib, c);
            }
        }
    }
}

// ------------------------------------------------------------------ backward
// One pass over CCH = 32 or 64 channels [c0, c0 + CCH).  The wavefront walks only its
// active entries (the forward's activity mask), last first, in groups of 16.
// The upstream semantic gradients G of its 64 pixels for these channels stay
// in registers in the two B-operand layouts:
//   GS[ks][pb] = G[pixel 16 pb + lane % 16][channel KS (lane / 16) + ks]  (S)
//   GD[ks][cb] = G[pixel 16 (lane / 16) + ks][channel 16 cb + lane % 16] (dO)
// S[f][p] = sum_c o_f[c] G_p[c]: A[m = f][k] = o_{act f}[KS (lane / 16) + ks]
// (KS = CCH / 4 consecutive floats of the staged feature row), output rows f = entries,
// columns p = pixels, stored in the wavefront's S / w buffer.  The reverse walk
// reads its S there and overwrites it with w.  dO[f][c] = sum_p w_f[p] G_p[c]:
// A[m = f][k] = w_f[16 (lane / 16) + ks], output D[f][c], added to the
// semantic gradient of entry f.  MAIN passes (c0 = 0) carry every term of the
// fragment adjoint and the 16 record slots (reduced over the wavefront's
// lanes); 64-channel passes after the first (c0 > 0) only the semantic share
// of the alpha gradient, i.e. record slots 0..5 (mean2d, conic, opacity), which
// they take from six pixel moments of dpow = dL/d(o G) with one more product,
// M[f][n] = sum_p dpow_f[p] phi_n(p).  The record-slot sums of the tile's
// wavefronts meet in LDS (one row of 16 per batch entry) and go to the
// gradient records with one atomic per entry and slot when the next batch is
// staged; the dO rows (CCH floats per entry) go straight from the matrix
// layout to the semantic gradients.
template <int TW, int TH, int CCH, int DM, bool MAIN>
__global__ void __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(CCH > 32 ? 2 : 4))) render_bwd_mm_kernel(
    const DevCam *__restrict__ cams, int V, int64_t N, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const float4 *__restrict__ rec, const float *__restrict__ sem, int C_o, int c0,
    const float *__restrict__ T_final, const uint32_t *__restrict__ n_contrib, const float *__restrict__ up_rgb,
    const float *__restrict__ gD_img, const float *__restrict__ up_kmap, const float *__restrict__ up_sem,
    float *__restrict__ grec, float *__restrict__ dsem, int batch, uint32_t ntiles, const float *__restrict__ hrec,
    SemSeed seed, const uint32_t *__restrict__ amask, int64_t mwords, unsigned long long *__restrict__ tclk)
{
    static_assert(CCH == 32 || CCH == 64, "backward pass: 32 or 64 channels");
    constexpr int NT = TW * TH, FS = feat_stride(CCH);
    constexpr int KS = CCH / 4, NCB = CCH / 16;
    constexpr bool HIT = DM == 2;
    constexpr float kd = DM == 1 ? 0.f : 1.f;
    extern __shared__ float4 smem[];
    __shared__ uint32_t s_max;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    float4 *srec = smem;
    float *sfeat = (float *)(smem + 4 * batch);
    uint32_t *sid = (uint32_t *)(sfeat + (size_t)batch * FS);  // two buffers of `batch` ids
    float *shh = (float *)(sid + 2 * batch);
    float *sgr = shh + (HIT ? batch : 0);  // [batch][16] record-slot sums of the tile's wavefronts
    float *swb = sgr + (size_t)batch * 16 + wave * (kBGrp * kSW);
    float *sdp = sgr + (size_t)batch * 16 + (NT / 64 + wave) * (kBGrp * kSW);  // channel passes: dpow, then moments
    for (int q = threadIdx.x; q < batch * 16; q += NT) sgr[q] = 0.f;
    const uint32_t slot = xcd_tile(blockIdx.x, ntiles);
    if (slot >= ntiles) return;
    const TileInfo ti = tile_info<TW, TH>(cams, V, slot);
    const uint32_t tile = ti.tile;
    if (tclk && threadIdx.x == 0) tclk[2 * tile] = __builtin_amdgcn_s_memrealtime();
    const uint2 range = ranges[tile];
    const float fx = (float)ti.px, fy = (float)ti.py;
    const int64_t recbase = (int64_t)ti.v * N;
    const int lane = __lane_id(), l16 = lane & 15, h16 = lane >> 4;
    const uint32_t *mplane = amask + (int64_t)wave * mwords;

    // upstream semantic gradients (or the fused cross-entropy seed) of the
    // wavefront's pixels for this pass's channels
    const int W = cams[ti.v].W, H = cams[ti.v].H;
    const int qx0 = ti.px - (lane & 7), qy0 = ti.py - (lane >> 3);
    const bool fused = !up_sem && seed.label;
    float my_lse = 0.f, my_sc = 0.f;
    int my_lab = -1;
    if (fused && ti.inside) seed_pixel(seed, C_o, ti.off, ti.HW, ti.pix, my_lse, my_lab, my_sc);
    // Addresses are clamped into the view and the channel range and the value
    // selected afterwards: no branch around a load, so that all of them are in
    // flight together instead of one round trip each.
    auto up_idx = [&](int p, int c, bool &ok) -> int64_t {
        const int x = qx0 + (p & 7), y = qy0 + (p >> 3);
        ok = c < C_o && x < W && y < H;
        return (int64_t)C_o * ti.off + (int64_t)min(c, C_o - 1) * ti.HW + (int64_t)min(y, H - 1) * W + min(x, W - 1);
    };
    float GSr[KS][4], GDr[16][NCB];
    auto fill = [&](auto up_at) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) GSr[ks][pb] = up_at(16 * pb + l16, c0 + KS * h16 + ks);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) GDr[ks][cb] = up_at(16 * h16 + ks, c0 + 16 * cb + l16);
    };
    if (fused) {
        fill([&](int p, int c) {
            bool ok;
            const float o = seed.logits[up_idx(p, c, ok)];
            const float l = __shfl(my_lse, p, 64), sc = __shfl(my_sc, p, 64);
            const int lb = __shfl(my_lab, p, 64);
            return ok ? sc * (__expf(o - l) - (c == lb ? 1.f : 0.f)) : 0.f;
        });
    } else if (up_sem) {
        fill([&](int p, int c) {
            bool ok;
            const float v = up_sem[up_idx(p, c, ok)];
            return ok ? v : 0.f;
        });
    } else {
        fill([&](int, int) { return 0.f; });
    }

    // Channel passes: the B operand of the dpow moments, column n = lane % 16
    // of phi = (1, x, y, x^2, x y, y^2) (zero past 5) at pixel 16 (lane / 16) + ks
    // of the wavefront's 8 x 8 block, where x = ks % 8 and y = 2 (lane / 16) +
    // ks / 8.  As a polynomial in x: phi = pa[ks / 8] + pb[ks / 8] x + pc x^2.
    const float bx0 = (float)qx0, by0 = (float)qy0;  // the block's origin pixel
    float pa[2], pb[2], pc;
    {
        const float y0 = (float)(2 * h16), y1 = y0 + 1.f;
        pa[0] = l16 == 0 ? 1.f : l16 == 2 ? y0 : l16 == 5 ? y0 * y0 : 0.f;
        pa[1] = l16 == 0 ? 1.f : l16 == 2 ? y1 : l16 == 5 ? y1 * y1 : 0.f;
        pb[0] = l16 == 1 ? 1.f : l16 == 4 ? y0 : 0.f;
        pb[1] = l16 == 1 ? 1.f : l16 == 4 ? y1 : 0.f;
        pc = l16 == 3 ? 1.f : 0.f;
    }
    auto phi = [&](int ks) -> float {
        const float x = (float)(ks & 7);
        return pa[ks >> 3] + (pb[ks >> 3] + pc * x) * x;
    };
    double T = 1.0;
    float gR = 0.f, gG = 0.f, gB = 0.f, gDp = 0.f, gK = 0.f;
    uint32_t last = 0;
    if (ti.inside) {
        const int64_t p = ti.pix, HW = ti.HW, off = ti.off;
        T = T_final[off + p];
        const uint32_t rel = n_contrib[off + p];
        last = rel ? range.x + rel : 0u;
        if constexpr (MAIN) {
            if (up_rgb) {
                gR = up_rgb[3 * off + p];
                gG = up_rgb[3 * off + HW + p];
                gB = up_rgb[3 * off + 2 * HW + p];
            }
            gDp = gD_img[off + p];
            if (up_kmap) gK = up_kmap[off + p];
        }
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (last) atomicMax(&s_max, last);
    __syncthreads();
    const uint32_t end_all = s_max;
    float A = 0.f;

    // Staging.  The ids of a batch's entries and this wavefront's mask words
    // for it are loaded one batch ahead (while the batch before is walked), so
    // that staging a batch costs one round trip to memory (records, feature
    // rows and hit constants at known ids, all in flight together) instead of
    // three (ids, then those loads, then the mask).
    const int t = (int)threadIdx.x;
    auto batch_start = [&](uint32_t e) -> uint32_t {
        return e - range.x > (uint32_t)batch ? e - (uint32_t)batch : range.x;
    };
    // mask words (lanes 0..2) of the batch at s0
    auto mask_of = [&](uint32_t s0) -> uint32_t { return lane < 3 ? mplane[(s0 >> 5) + lane] : 0u; };
    BatchIds<64> nid;
    uint32_t nmask = 0;
    nid.v[0] = 0;
    if (end_all > range.x) {
        const uint32_t s0 = batch_start(end_all);
        nid.load(vals, s0, (int)(end_all - s0), lane);
        nmask = mask_of(s0);
    }

    // the record-slot sums of the previous batch (ids in sidp) to the
    // gradient records: one atomic per entry and slot for the whole tile
    auto flush = [&](int nn, const uint32_t *sidp) {
        for (int q = t; q < nn * 16; q += NT) {
            const float x = sgr[q];
            if (x != 0.f) {
                unsafeAtomicAdd(&grec[(recbase + sidp[q >> 4]) * kRecFloats + (q & 15)], x);
                sgr[q] = 0.f;
            }
        }
    };
    int kb = 0, n_prev = 0;
    for (uint32_t end = end_all; end > range.x; ++kb) {
        const uint32_t start = batch_start(end);
        const int n = (int)(end - start);
        const BatchIds<64> cid = nid;
        const uint32_t cm = nmask;
        uint32_t *sidc = sid + (kb & 1) * batch;
        __syncthreads();
        stage_ids<NT, CCH, MAIN ? 4 : 2, (CCH > 32 ? 16 : 4), 64, HIT>(srec, sfeat, shh, cid, n, rec, recbase, sem,
                                                                    C_o, c0, hrec);
        if (t < n) sidc[t] = cid.v[0];
        if (kb) flush(n_prev, sid + ((kb - 1) & 1) * batch);

        __syncthreads();
        if (start > range.x) {
            const uint32_t s1 = batch_start(start);
            nid.load(vals, s1, (int)(start - s1), lane);
            nmask = mask_of(s1);
        }
        // the batch's active entries for this wavefront, last first, from the
        // forward's activity mask (bits of entries start .. start + n - 1)
        int nact = 0, myact = 0;
        {
            const uint32_t m0 = __builtin_amdgcn_readlane(cm, 0), m1 = __builtin_amdgcn_readlane(cm, 1),
                           m2 = __builtin_amdgcn_readlane(cm, 2);
            const uint64_t lo = ((uint64_t)m1 << 32) | m0;
            const int sh = (int)(start & 31);
            uint64_t m = sh ? (lo >> sh) | ((uint64_t)m2 << (64 - sh)) : lo;
            if (n < 64) m &= (1ull << n) - 1ull;
            while (m) {
                const int j = 63 - __builtin_clzll(m);
                m &= ~(1ull << j);
                myact = lane == nact ? j : myact;
                ++nact;
            }
        }
        for (int g0 = 0; g0 < nact; g0 += kBGrp) {
            // 64 channels: the Gaussian id of group row lane % 16, read now
            // (beside the S products) so that the dO atomics below need one
            // shuffle per row instead of a shuffle and a dependent LDS read
            // (the 32-channel form has no register to hold it)
            uint32_t gid_row = 0;
            // S for the group's 16 entries (rows past nact repeat an active entry; their w is 0)
            {
                const int fa = __shfl(myact, min(g0 + l16, nact - 1), 64);
                if constexpr (CCH > 32) gid_row = sidc[fa];
                const float *arow = sfeat + fa * FS + KS * h16;
                // 64 channels: four independent accumulators (one per 16-pixel
                // block), so that each feature value is read from LDS once and
                // the products issue back to back instead of as four dependent
                // chains
                // (the 32-channel form keeps one chain at a time: its 128
                // registers have no room for the other three accumulators)
                constexpr int PBI = CCH > 32 ? 4 : 1;
                mf4 s4[4];
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) s4[pb] = mf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int pb0 = 0; pb0 < 4; pb0 += PBI) {
#pragma unroll
                    for (int k4 = 0; k4 < KS / 4; ++k4) {
                        const float4 a = reinterpret_cast<const float4 *>(arow)[k4];
#pragma unroll
                        for (int pb = pb0; pb < pb0 + PBI; ++pb) {
                            s4[pb] = mma(a.x, GSr[4 * k4][pb], s4[pb]);
                            s4[pb] = mma(a.y, GSr[4 * k4 + 1][pb], s4[pb]);
                            s4[pb] = mma(a.z, GSr[4 * k4 + 2][pb], s4[pb]);
                            s4[pb] = mma(a.w, GSr[4 * k4 + 3][pb], s4[pb]);
                        }
                    }
#pragma unroll
                    for (int pb = pb0; pb < pb0 + PBI; ++pb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) swb[(4 * h16 + r) * kSW + 16 * pb + l16] = s4[pb][r];
                }
            }
            __builtin_amdgcn_wave_barrier();
            // reverse walk over the group
            const int ng = min(kBGrp, nact - g0);
            if constexpr (!MAIN) {
                // Channel passes after the first: per entry only w (for the dO
                // product below) and dpow, both to LDS rows; the record slots
                // follow from moments of dpow after the walk.  Entries go in
                // pairs (two independent alpha evaluations), and an entry's LDS
                // operands (its S value and the alpha-test half of its record)
                // are read one pair ahead, so that a pair's arithmetic does not
                // start with a wait for them.
                struct EntIn {
                    int j;
                    float s;
                    float4 r0, r1;
                };
                auto entry_load = [&](int f) -> EntIn {
                    EntIn e;
                    e.j = __builtin_amdgcn_readlane(myact, g0 + f);
                    e.s = swb[f * kSW + lane];
                    e.r0 = srec[4 * e.j];
                    e.r1 = srec[4 * e.j + 1];
                    return e;
                };
                auto entry_w = [&](const EntIn &e, bool valid, float &dp) -> float {
                    const uint32_t entry = start + (uint32_t)e.j;
                    const float4 r0 = e.r0, r1 = e.r1;
                    const float dx = fx - r0.x, dy = fy - r0.y;
                    const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                    const float oG = r1.y * gauss_of(t1, t2);
                    const float alpha = fminf(kAlphaMax, oG);
                    const bool contrib = valid && entry < last && alpha >= kAlphaMin;
                    return frag_weight_sem(contrib, alpha, oG, e.s, T, A, dp);
                };
                EntIn ea = entry_load(0), eb = entry_load(min(1, ng - 1));
                for (int f = 0; f < ng; f += 2) {
                    const bool has1 = f + 1 < ng;
                    float d0, d1;
                    const float w0 = entry_w(ea, true, d0);
                    const float w1 = entry_w(eb, has1, d1);
                    // (rows past ng reload the last entry; the loop ends before using them)
                    ea = entry_load(min(f + 2, ng - 1));
                    eb = entry_load(min(f + 3, ng - 1));
                    swb[f * kSW + lane] = w0;
                    sdp[f * kSW + lane] = d0;
                    if (has1) {
                        swb[(f + 1) * kSW + lane] = w1;
                        sdp[(f + 1) * kSW + lane] = d1;
                    }
                }
                // (dpow rows past ng are left as they are: a product row
                // depends only on its own A row, and those rows are not used)
                for (int f = ng; f < kBGrp; ++f) swb[f * kSW + lane] = 0.f;
            }
            constexpr bool PAIR_MAIN = MAIN && CCH > 32;  // (the 32-channel form has no registers to spare)
            if constexpr (PAIR_MAIN) {
                // a 64-channel first pass pairs its entries the same way (16
                // slots each, one 32-value reduction)
                auto entry_all = [&](int f, bool valid, float (&v)[16], int &jo) -> float {
                    const int j = __builtin_amdgcn_readlane(myact, g0 + f);
                    const uint32_t entry = start + (uint32_t)j;
                    const float s_sem = swb[f * kSW + lane];
                    const float4 r0 = srec[4 * j], r1 = srec[4 * j + 1];
                    const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
                    const float dx = fx - r0.x, dy = fy - r0.y;
                    const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                    const float G = gauss_of(t1, t2);
                    const float oG = r1.y * G;
                    const float alpha = fminf(kAlphaMax, oG);
                    const bool contrib = valid && entry < last && alpha >= kAlphaMin;
                    jo = j;
                    return frag_adjoint(contrib, r0, r1, r2, r3, dx, dy, t1, t2, G, oG, alpha, s_sem, gR, gG, gB, gDp,
                                        gK, frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy), T, A, v);
                };
                for (int f = 0; f < ng; f += 2) {
                    const bool has1 = f + 1 < ng;
                    float v0[16], v1[16], v[32];
                    int id0, id1;
                    const float w0 = entry_all(f, true, v0, id0);
                    const float w1 = entry_all(has1 ? f + 1 : f, has1, v1, id1);
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        v[k] = v0[k];
                        v[16 + k] = v1[k];
                    }
                    const float tot = reduce_scatter<32>(v);
                    const int slot = lane >> 1, e1 = slot >> 4, k = slot & 15;
                    if ((lane & 1) == 0 && (e1 == 0 || has1)) lds_add(&sgr[(e1 ? id1 : id0) * 16 + k], tot);
                    swb[f * kSW + lane] = w0;
                    if (has1) swb[(f + 1) * kSW + lane] = w1;
                }
                for (int f = ng; f < kBGrp; ++f) swb[f * kSW + lane] = 0.f;
            }
            for (int f = 0; f < kBGrp && MAIN && !PAIR_MAIN; ++f) {
                float w = 0.f;
                if (f < ng) {
                    const int j = __builtin_amdgcn_readlane(myact, g0 + f);
                    const uint32_t entry = start + (uint32_t)j;
                    const float s_sem = swb[f * kSW + lane];
                    const float4 r0 = srec[4 * j], r1 = srec[4 * j + 1];
                    const float dx = fx - r0.x, dy = fy - r0.y;
                    const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                    const float G = gauss_of(t1, t2);
                    const float oG = r1.y * G;
                    const float alpha = fminf(kAlphaMax, oG);
                    const bool contrib = entry < last && alpha >= kAlphaMin;
                    float *gr = sgr + j * 16;
                    if constexpr (MAIN) {
                        float v[16];
                        const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
                        w = frag_adjoint(contrib, r0, r1, r2, r3, dx, dy, t1, t2, G, oG, alpha, s_sem, gR, gG, gB,
                                         gDp, gK, frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy), T, A, v);
                        const float tot = reduce_scatter<16>(v);
                        if ((lane & 3) == 0) lds_add(&gr[lane >> 2], tot);
                    }
                }
                swb[f * kSW + lane] = w;
            }
            __builtin_amdgcn_wave_barrier();
            // dO[f][c] = sum_p w_f[p] G_p[c] over the wavefront's pixels
            {
                mf4 d4[NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) d4[cb] = mf4{0.f, 0.f, 0.f, 0.f};
                const float *wrow = swb + l16 * kSW + 16 * h16;
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const float4 a = reinterpret_cast<const float4 *>(wrow)[k4];
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        d4[cb] = mma(a.x, GDr[4 * k4][cb], d4[cb]);
                        d4[cb] = mma(a.y, GDr[4 * k4 + 1][cb], d4[cb]);
                        d4[cb] = mma(a.z, GDr[4 * k4 + 2][cb], d4[cb]);
                        d4[cb] = mma(a.w, GDr[4 * k4 + 3][cb], d4[cb]);
                    }
                }
                if constexpr (CCH <= 32) {
                    // 32 channels: D to LDS rows (the wavefront's w buffer,
                    // free after the products), then one atomic instruction per
                    // two entries, each a whole 128-byte row (12.85 -> 12.34 ms
                    // on the 1M-Gaussian 16-view step; slower at 64 channels)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) swb[(4 * h16 + r) * kSW + 16 * cb + l16] = d4[cb][r];
                    __builtin_amdgcn_wave_barrier();
                    const int fl = lane >> 5, cl = lane & 31;
                    for (int f0 = 0; f0 < ng; f0 += 2) {
                        const int f = f0 + fl;
                        const int jf = __shfl(myact, min(g0 + f, nact - 1), 64);
                        const float x = swb[f * kSW + cl];
                        if (f < ng && x != 0.f && c0 + cl < C_o)
                            unsafeAtomicAdd(&dsem[(int64_t)sidc[jf] * C_o + c0 + cl], x);
                    }
                } else {
                    uint32_t idr[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) idr[r] = (uint32_t)__shfl((int)gid_row, 4 * h16 + r, 64);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int f = 4 * h16 + r;
                        if (f < ng) {
                            const int64_t row = (int64_t)idr[r] * C_o + c0;
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb) {
                                const float x = d4[cb][r];
                                if (x != 0.f && c0 + 16 * cb + l16 < C_o)
                                    unsafeAtomicAdd(&dsem[row + 16 * cb + l16], x);
                            }
                        }
                    }
                }
            }
            if constexpr (!MAIN) {
                // M[f][n] = sum_p dpow_f[p] phi_n(p): B[k][n] = phi_n(pixel
                // 16 (lane / 16) + ks) for step ks, output M[4 (lane / 16) + r][lane % 16]
                mf4 m4 = mf4{0.f, 0.f, 0.f, 0.f};
                const float *drow = sdp + l16 * kSW + 16 * h16;
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const float4 a = reinterpret_cast<const float4 *>(drow)[k4];
                    m4 = mma(a.x, phi(4 * k4), m4);
                    m4 = mma(a.y, phi(4 * k4 + 1), m4);
                    m4 = mma(a.z, phi(4 * k4 + 2), m4);
                    m4 = mma(a.w, phi(4 * k4 + 3), m4);
                }
                const int jrow = __shfl(myact, min(g0 + lane, nact - 1), 64);  // entry of row `lane` (< 16)
                if (l16 < 6) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sdp[(4 * h16 + r) * kSW + l16] = m4[r];
                }
                __builtin_amdgcn_wave_barrier();
                if (lane < ng) {
                    // the six record slots of entry row `lane` from its moments
                    // about the block origin, re-centred on the entry's mean
                    const float4 mq = *reinterpret_cast<const float4 *>(sdp + lane * kSW);
                    const float2 mr = *reinterpret_cast<const float2 *>(sdp + lane * kSW + 4);
                    const float M0 = mq.x, Mx = mq.y, My = mq.z, Mxx = mq.w, Mxy = mr.x, Myy = mr.y;
                    const float4 r0 = srec[4 * jrow], r1 = srec[4 * jrow + 1];
                    const float mx = r0.x - bx0, my = r0.y - by0;
                    const float l11 = r0.z, l21 = r0.w, l22 = r1.x;
                    // centred moments: sums of dpow (dx, dy, dx^2, dx dy, dy^2), d = pixel - mean
                    const float Sx = Mx - mx * M0, Sy = My - my * M0;
                    const float Sxx = (Mxx - mx * Mx) - mx * Sx;
                    const float Sxy = (Mxy - my * Mx) - mx * Sy;
                    const float Syy = (Myy - my * My) - my * Sy;
                    const float St1 = l11 * Sx + l21 * Sy;  // sum of dpow t1
                    float *gr = sgr + jrow * 16;
                    lds_add(&gr[0], l11 * St1);
                    lds_add(&gr[1], l21 * St1 + l22 * l22 * Sy);
                    lds_add(&gr[2], -(l11 * Sxx + l21 * Sxy));
                    lds_add(&gr[3], -(l11 * Sxy + l21 * Syy));
                    lds_add(&gr[4], -l22 * Syy);
                    lds_add(&gr[5], r1.y > 0.f ? M0 / r1.y : 0.f);  // sum of dalpha G = sum of dpow / o
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        n_prev = n;
        end = start;
    }
    if (kb) {
        __syncthreads();
        flush(n_prev, sid + ((kb - 1) & 1) * batch);
    }
    if (tclk) {
        __syncthreads();
        if (threadIdx.x == 0) tclk[2 * tile + 1] = __builtin_amdgcn_s_memrealtime();
    }
}

// Largest batch (a multiple of 16, at most `want`) whose LDS fits `cap` bytes.
template <typename F>
int fit_batch(int want, size_t cap, F lds)
{
    int b = (want + 15) / 16 * 16;
    if (b < 16) b = 16;
    while (b > 16 && lds(b) > cap) b -= 16;
    return b;
}

template <int TW, int TH, int CCH>
hipError_t fwd_mm_launch(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                         const ugs_outputs &out, int batch, bool counters, int final_buf, int c0, hipStream_t s)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto ranges = (const uint2 *)(ws + L.ranges);
    auto vals = (const uint32_t *)(ws + (final_buf ? L.vals1 : L.vals0));
    auto rec = (const float4 *)(ws + L.rec);
    auto cnt = (DevCounters *)(ws + L.counters);
    auto hrec = (const float *)(ws + L.hrec);
    constexpr int NW = TW * TH / 64;
    const bool hit = pb.depth_mode == 2;
    const int b = std::min(kFwdMaxBatch, fit_batch(batch, 64 * 1024, [&](int x) { return fwd_mm_lds(x, CCH, NW, hit); }));
    const size_t lds = fwd_mm_lds(b, CCH, NW, hit);
    const bool main_pass = c0 == 0;
    auto tclk = (counters && main_pass) ? (unsigned long long *)(ws + L.tclk) : nullptr;
    // the activity mask: written by the first pass of a forward that keeps the
    // backward's state (T_final, n_contrib), read by its further channel passes
    // and by the backward
    uint32_t *amask = nullptr;
    if (out.T_final && out.n_contrib) {
        amask = (uint32_t *)(ws + L.amask);
        if (main_pass) {
            hipError_t e = launch_fill_u32(amask, 0u, (int64_t)kMaskPlanes * L.amask_words, s);
            if (e != hipSuccess) return e;
        }
    }
#define UGS_FWD_MM(DMV, MAINV)                                                                                  \
    hipLaunchKernelGGL((render_fwd_mm_kernel<TW, TH, CCH, DMV, MAINV>), dim3(xcd_grid(pb.total_tiles)),        \
                       dim3(TW * TH), lds, s, cams, pb.V, pb.N, ranges, vals, rec, g.sem, pb.C_o, c0, out, b, cnt, \
                       (int)counters, (uint32_t)pb.total_tiles, hrec, pb.half_out, amask, L.amask_words, tclk)
    if (main_pass) {
        if (pb.depth_mode == 2) UGS_FWD_MM(2, true);
        else if (pb.depth_mode == 1) UGS_FWD_MM(1, true);
        else UGS_FWD_MM(0, true);
    } else {
        if (pb.depth_mode == 2) UGS_FWD_MM(2, false);
        else UGS_FWD_MM(0, false);  // no depth in chunk passes: modes 0 and 1 walk alike
    }
#undef UGS_FWD_MM
    return hipGetLastError();
}

template <int TW, int TH, int CCH>
hipError_t bwd_mm_launch(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                         const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg, int batch,
                         int final_buf, int c0, bool counters, hipStream_t s)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto ranges = (const uint2 *)(ws + L.ranges);
    auto vals = (const uint32_t *)(ws + (final_buf ? L.vals1 : L.vals0));
    auto rec = (const float4 *)(ws + L.rec);
    auto grec = (float *)(ws + L.grec);
    auto gd = (const float *)(ws + L.gd);
    auto hrec = (const float *)(ws + L.hrec);
    const SemSeed seed{out.sem, up.sem ? nullptr : up.sem_label, up.sem_scale};
    constexpr int NW = TW * TH / 64;
    const bool hit = pb.depth_mode == 2, main_pass = c0 == 0;
    auto tclk = (counters && main_pass) ? (unsigned long long *)(ws + L.tclk + (size_t)pb.total_tiles * 16) : nullptr;
    const int b =
        std::min(64, fit_batch(batch, 64 * 1024, [&](int x) { return bwd_mm_lds(x, CCH, NW, hit, main_pass); }));
    const size_t lds = bwd_mm_lds(b, CCH, NW, hit, main_pass);
#define UGS_BWD_MM(DMV, MAINV)                                                                                    \
    hipLaunchKernelGGL((render_bwd_mm_kernel<TW, TH, CCH, DMV, MAINV>), dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), \
                       lds, s, cams, pb.V, pb.N, ranges, vals, rec, g.sem, pb.C_o, c0, out.T_final, out.n_contrib,   \
                       up.rgb, gd, up.kmap, up.sem, grec, dg.sem, b, (uint32_t)pb.total_tiles, hrec, seed,     \
                       (const uint32_t *)(ws + L.amask), L.amask_words, tclk)
    if (main_pass) {
        if (pb.depth_mode == 2) UGS_BWD_MM(2, true);
        else if (pb.depth_mode == 1) UGS_BWD_MM(1, true);
        else UGS_BWD_MM(0, true);
    } else if constexpr (CCH > 32) {
        if (pb.depth_mode == 2) UGS_BWD_MM(2, false);
        else UGS_BWD_MM(0, false);
    } else {
        return hipErrorInvalidValue;  // channel passes after the first are 64 wide
    }
#undef UGS_BWD_MM
    return hipGetLastError();
}

// Channels per forward pass for C_o channels (9..256): at most 64, so that the
// accumulators (one register per channel) leave room for four wavefronts per
// SIMD; 128 channels in one pass (two wavefronts per SIMD) measured 38.4 ms
// against 32.0 ms for two 64-channel passes on the 3M-Gaussian 16-view step.
int fwd_pass_channels(int C_o) { return C_o <= 16 ? 16 : C_o <= 32 ? 32 : 64; }

template <int TW, int TH>
hipError_t fwd_mm_tile(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out,
                       int batch, bool counters, int final_buf, hipStream_t s)
{
    const int cch = fwd_pass_channels(pb.C_o);
    for (int c0 = 0; c0 < pb.C_o; c0 += cch) {
        hipError_t e;
        switch (cch) {
        case 16: e = fwd_mm_launch<TW, TH, 16>(g, pb, L, ws, out, batch, counters, final_buf, c0, s); break;
        case 32: e = fwd_mm_launch<TW, TH, 32>(g, pb, L, ws, out, batch, counters, final_buf, c0, s); break;
        default: e = fwd_mm_launch<TW, TH, 64>(g, pb, L, ws, out, batch, counters, final_buf, c0, s); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Channels per backward pass: 32 up to 32 channels (upstream in 64 registers,
// four wavefronts per SIMD), else 64 (128 registers, two wavefronts per SIMD):
// on the 3M-Gaussian 128-channel step two 64-channel passes take 85.8 ms
// against 87.8 ms for four 32-channel ones.
int bwd_pass_channels(int C_o) { return C_o <= 32 ? 32 : 64; }

template <int TW, int TH>
hipError_t bwd_mm_tile(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out,
                       const ugs_upstream &up, const ugs_gaussian_grads &dg, int batch, int final_buf, bool counters,
                       hipStream_t s)
{
    const int cch = bwd_pass_channels(pb.C_o);
    for (int c0 = 0; c0 < pb.C_o; c0 += cch) {
        hipError_t e = cch == 32 ? bwd_mm_launch<TW, TH, 32>(g, pb, L, ws, out, up, dg, batch, final_buf, c0, counters, s)
                                 : bwd_mm_launch<TW, TH, 64>(g, pb, L, ws, out, up, dg, batch, final_buf, c0, counters, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_render_fwd_mm(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                                const ugs_outputs &out, int batch, bool counters, int final_buf, hipStream_t s)
{
    if (pb.total_tiles == 0) return hipSuccess;
    if (pb.tile_w == 8 && pb.tile_h == 8) return fwd_mm_tile<8, 8>(g, pb, L, ws, out, batch, counters, final_buf, s);
    if (pb.tile_w == 32 && pb.tile_h == 8) return fwd_mm_tile<32, 8>(g, pb, L, ws, out, batch, counters, final_buf, s);
    return fwd_mm_tile<16, 16>(g, pb, L, ws, out, batch, counters, final_buf, s);
}

hipError_t launch_render_bwd_mm(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                                const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg,
                                int batch, int final_buf, bool counters, hipStream_t s)
{
    if (pb.total_tiles == 0) return hipSuccess;
    if (pb.tile_w == 8 && pb.tile_h == 8)
        return bwd_mm_tile<8, 8>(g, pb, L, ws, out, up, dg, batch, final_buf, counters, s);
    if (pb.tile_w == 32 && pb.tile_h == 8)
        return bwd_mm_tile<32, 8>(g, pb, L, ws, out, up, dg, batch, final_buf, counters, s);
    return bwd_mm_tile<16, 16>(g, pb, L, ws, out, up, dg, batch, final_buf, counters, s);
}

}  // namespace ugs
