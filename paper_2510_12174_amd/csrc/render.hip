// Stages S5 and S8: the per-pixel compositing loop of Alg. forward_render and
// its reverse of Alg. backward_render, for gfx950.
//
// One workgroup per (view, tile), one lane per pixel.  The tile's sorted list is
// walked in batches that the workgroup stages in LDS (64 B record + the C_o
// semantic logits per Gaussian); every lane then reads the batch with broadcast
// LDS loads.  The forward keeps transmittance and depth in FP64 (the depth
// feeds a finite-difference normal, which amplifies its error), everything else
// in FP32.  The backward recovers T from T_final by division, keeps the pixel's
// adjoint state O(1) (a running sum A of w_j s_j over later fragments, with s_j
// the dot product of the upstream gradients with fragment j's values), reduces
// each fragment's gradient over the 64 lanes of a wavefront with DPP, and
// issues one coalesced atomic per wavefront and fragment.
#include "render_common.h"

namespace ugs {
namespace {

template <int TW, int TH, int CO, int DM>
__global__ void __launch_bounds__(TW *TH) render_fwd_kernel(
    const DevCam *__restrict__ cams, int V, int64_t N, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const float4 *__restrict__ rec, const float *__restrict__ sem, int C_o,
    ugs_outputs out, int batch, DevCounters *__restrict__ cnt, int count, uint32_t ntiles, int depth_mode, const float *__restrict__ hrec,
    int half_out)
{
    constexpr int NT = TW * TH;
    extern __shared__ float4 smem[];
    float4 *srec = smem;
    float *ssem = (float *)(smem + 4 * batch);
    float *shh = DM == 2 ? ssem + (size_t)batch * CO : nullptr;
    const uint32_t slot = xcd_tile(blockIdx.x, ntiles);
    if (slot >= ntiles) return;
    const TileInfo ti = tile_info<TW, TH>(cams, V, slot);
    const uint32_t tile = ti.tile;
    const uint2 range = ranges[tile];
    const float fx = (float)ti.px, fy = (float)ti.py;
    const int64_t recbase = (int64_t)ti.v * N;

    double T = 1.0, D = 0.0;
    float cr = 0.f, cg = 0.f, cb = 0.f, K = 0.f;
    float acc[CO > 0 ? CO : 1];
#pragma unroll
    for (int c = 0; c < (CO > 0 ? CO : 1); ++c) acc[c] = 0.f;
    uint32_t last = 0, n_eval = 0, n_con = 0;
    bool done = !ti.inside;
    constexpr bool HIT = DM == 2;
    constexpr float kd = DM == 1 ? 0.f : 1.f;  // depth form fixed per instantiation

    for (uint32_t start = range.x; start < range.y; start += (uint32_t)batch) {
        if (__syncthreads_count(done) == NT) break;
        const int n = (int)min((uint32_t)batch, range.y - start);
        stage_batch<NT, CO>(srec, ssem, vals, start, n, rec, recbase, sem, C_o);
        stage_hits<NT, HIT>(shh, vals, start, n, hrec, recbase);
        __syncthreads();
        if (!done) {
            for (int j = 0; j < n; ++j) {
                const float4 r0 = srec[4 * j], r1 = srec[4 * j + 1];
                const float dx = fx - r0.x, dy = fy - r0.y;
                const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                const float alpha = fminf(kAlphaMax, r1.y * gauss_of(t1, t2));
                ++n_eval;
                if (alpha < kAlphaMin) continue;
                const double tT = T * (1.0 - (double)alpha);
                if (tT < kTStop) {
                    done = true;
                    break;
                }
                const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
                const float kdj = frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy);
                const float B = kdj * (r2.x * dx + r2.y * dy);
                const float Cq = kdj * (r2.z * dx * dx + 2.f * r2.w * dx * dy + r3.x * dy * dy);
                const float d = r1.w * (1.f + B) * rcp_nr(1.f + 2.f * B + Cq);
                const double w = (double)alpha * T;
                const float wf = (float)w;
                cr += wf * r3.y;
                cg += wf * r3.z;
                cb += wf * r3.w;
                K += wf * r1.z;
                D += w * (double)d;
                if constexpr (CO > 0) {
                    const float4 *s4 = (const float4 *)(ssem + j * CO);
#pragma unroll
                    for (int c = 0; c < CO / 4; ++c) {
                        float4 o = s4[c];
                        acc[4 * c] += wf * o.x;
                        acc[4 * c + 1] += wf * o.y;
                        acc[4 * c + 2] += wf * o.z;
                        acc[4 * c + 3] += wf * o.w;
                    }
                }
                T = tT;
                last = start + (uint32_t)j + 1;
                ++n_con;
            }
        }
    }
    if (ti.inside) {
        const int64_t p = ti.pix, HW = ti.HW, off = ti.off;
        put_out(out.rgb, 3 * off + p, cr, half_out);
        put_out(out.rgb, 3 * off + HW + p, cg, half_out);
        put_out(out.rgb, 3 * off + 2 * HW + p, cb, half_out);
        out.depth[off + p] = (float)D;
        put_out(out.kmap, off + p, K, half_out);
        if (out.T_final) out.T_final[off + p] = (float)T;  // optional in forward-only use
        if (out.n_contrib) out.n_contrib[off + p] = last ? last - range.x : 0u;
        if constexpr (CO > 0) {
#pragma unroll
            for (int c = 0; c < CO; ++c)
                if (c < C_o) put_out(out.sem, (int64_t)C_o * off + c * HW + p, acc[c], half_out);
        }
    }
    if (count) {
        unsigned long long e = n_eval, c = n_con;
        for (int o = 32; o > 0; o >>= 1) {
            e += __shfl_xor(e, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if (__lane_id() == 0) {
            atomicAdd(&cnt->n_eval, e);
            atomicAdd(&cnt->n_contrib, c);
        }
    }
}

// Reduces and adds one fragment's 16 + C_o gradient values (slots 0..15 the
// gradient record, slots 16.. the semantic logits, zero beyond C_o) in groups of
// 64, 32, 16 or 8 slots, largest first, so that no reduction work is spent on
// padding beyond the next multiple of 8.  One lane per slot issues the atomic.
template <int OFF, int REM, int CO, int CA>
__device__ __forceinline__ void emit_groups(const float (&v)[16], float w, const float (&gO)[CA], int lane,
                                            float *__restrict__ grec_i, float *__restrict__ dsem_i, int C_o)
{
    constexpr int G = REM >= 64 ? 64 : REM >= 32 ? 32 : REM >= 16 ? 16 : 8;
    constexpr int SH = G == 64 ? 0 : G == 32 ? 1 : G == 16 ? 2 : 3;  // log2(64 / G)
    float x[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int slot = OFF + q;
        if (slot < 16) x[q] = v[slot];
        else if (slot - 16 < CO) x[q] = w * gO[slot - 16];
        else x[q] = 0.f;
    }
    const float tot = reduce_scatter<G>(x);
    if ((lane & ((1 << SH) - 1)) == 0) {
        const int slot = OFF + (lane >> SH);
        if (slot < 16) unsafeAtomicAdd(&grec_i[slot], tot);
        else if (slot - 16 < C_o) unsafeAtomicAdd(&dsem_i[slot - 16], tot);
    }
    if constexpr (REM > G) emit_groups<OFF + G, REM - G, CO, CA>(v, w, gO, lane, grec_i, dsem_i, C_o);
}

template <int TW, int TH, int CO, int DM>
__global__ void __launch_bounds__(TW *TH) render_bwd_kernel(
    const DevCam *__restrict__ cams, int V, int64_t N, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const float4 *__restrict__ rec, const float *__restrict__ sem, int C_o,
    const float *__restrict__ T_final, const uint32_t *__restrict__ n_contrib, const float *__restrict__ up_rgb,
    const float *__restrict__ gD_img, const float *__restrict__ up_kmap, const float *__restrict__ up_sem,
    float *__restrict__ grec, float *__restrict__ dsem, int batch, uint32_t ntiles, int depth_mode, const float *__restrict__ hrec,
    SemSeed seed)
{
    constexpr int NT = TW * TH;
    constexpr int CA = CO > 0 ? CO : 1;
    extern __shared__ float4 smem[];
    __shared__ uint32_t s_max;
    float4 *srec = smem;
    float *ssem = (float *)(smem + 4 * batch);
    float *shh = DM == 2 ? ssem + (size_t)batch * CO : nullptr;
    const uint32_t slot = xcd_tile(blockIdx.x, ntiles);
    if (slot >= ntiles) return;
    const TileInfo ti = tile_info<TW, TH>(cams, V, slot);
    const uint32_t tile = ti.tile;
    const uint2 range = ranges[tile];
    const float fx = (float)ti.px, fy = (float)ti.py;
    const int64_t recbase = (int64_t)ti.v * N;
    const int lane = __lane_id();

    double T = 1.0;
    float gR = 0.f, gG = 0.f, gB = 0.f, gDp = 0.f, gK = 0.f;
    uint32_t last = 0;
    float gO[CA];
#pragma unroll
    for (int c = 0; c < CA; ++c) gO[c] = 0.f;
    if (ti.inside) {
        const int64_t p = ti.pix, HW = ti.HW, off = ti.off;
        T = T_final[off + p];
        const uint32_t rel = n_contrib[off + p];
        last = rel ? range.x + rel : 0u;
        if (up_rgb) {
            gR = up_rgb[3 * off + p];
            gG = up_rgb[3 * off + HW + p];
            gB = up_rgb[3 * off + 2 * HW + p];
        }
        gDp = gD_img[off + p];
        if (up_kmap) gK = up_kmap[off + p];
        if constexpr (CO > 0) {
            if (up_sem) {
#pragma unroll
                for (int c = 0; c < CO; ++c)
                    if (c < C_o) gO[c] = up_sem[(int64_t)C_o * off + c * HW + p];
            } else if (seed.label) {
                float lse, sc;
                int lab;
                seed_pixel(seed, C_o, off, HW, p, lse, lab, sc);
#pragma unroll
                for (int c = 0; c < CO; ++c)
                    if (c < C_o)
                        gO[c] = sc * (__expf(seed.logits[(int64_t)C_o * off + c * HW + p] - lse) - (c == lab ? 1.f : 0.f));
            }
        }
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (last) atomicMax(&s_max, last);
    __syncthreads();
    const uint32_t end_all = s_max;
    uint32_t wave_last = last;
    for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, o, 64));
    wave_last = __builtin_amdgcn_readfirstlane(wave_last);
    float A = 0.f;
    constexpr bool HIT = DM == 2;
    constexpr float kd = DM == 1 ? 0.f : 1.f;  // depth form fixed per instantiation

    for (uint32_t end = end_all; end > range.x;) {
        const uint32_t start = end - range.x > (uint32_t)batch ? end - (uint32_t)batch : range.x;
        const int n = (int)(end - start);
        __syncthreads();
        stage_batch<NT, CO>(srec, ssem, vals, start, n, rec, recbase, sem, C_o);
        stage_hits<NT, HIT>(shh, vals, start, n, hrec, recbase);
        __syncthreads();
        for (int j = n - 1; j >= 0; --j) {
            const uint32_t entry = start + (uint32_t)j;
            if (entry >= wave_last) continue;  // beyond every pixel of this wavefront
            const float4 r0 = srec[4 * j], r1 = srec[4 * j + 1];
            const float dx = fx - r0.x, dy = fy - r0.y;
            const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
            const float G = gauss_of(t1, t2);
            const float oG = r1.y * G;
            const float alpha = fminf(kAlphaMax, oG);
            const bool contrib = entry < last && alpha >= kAlphaMin;
            if (!__any(contrib)) continue;
            float s_sem = 0.f;
            if constexpr (CO > 0) {
                const float4 *s4 = (const float4 *)(ssem + j * CO);
#pragma unroll
                for (int c = 0; c < CO / 4; ++c) {
                    float4 o = s4[c];
                    s_sem += gO[4 * c] * o.x + gO[4 * c + 1] * o.y + gO[4 * c + 2] * o.z + gO[4 * c + 3] * o.w;
                }
            }
            float v[16];
            const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
            const float w = frag_adjoint(contrib, r0, r1, r2, r3, dx, dy, t1, t2, G, oG, alpha, s_sem, gR, gG, gB,
                                         gDp, gK, frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy), T, A, v);
            // per-fragment values: slots 0..15 are the gradient record (slot 6 the
            // gradient factor), slots 16..16+C_o the semantic logits
            const uint32_t id = vals[entry];
            const int64_t ridx = recbase + id;
            emit_groups<0, 16 + CO, CO>(v, w, gO, lane, grec + ridx * kRecFloats, dsem + (int64_t)id * C_o, C_o);
        }
        end = start;
    }
}

// ------------------------------------------------------------------------
// Backward with the semantic contractions on the matrix cores (C_o padded to
// 16 or 32).  Per wavefront (64 pixels, lane = pixel) and per group of 16
// list entries, two products replace the per-lane semantic work:
//   S[f][p]    = sum_c o_f[c] G_p[c]   (the semantic part of s_i, Alg.
//                backward_render), before the group's reverse walk;
//   dO[f][c]  += sum_p w_f[p] G_p[c]   (the semantic-logit gradient, the
//                transpose of the semantic rendering equation), after it.
// G_p is the upstream semantic gradient of pixel p.  Both products run on
// bf16 MFMAs with every FP32 operand split as x = hi + lo (hi = bf16(x),
// lo = bf16(x - hi)) and three products per tile (hi hi + hi lo + lo hi)
// accumulated in FP32: the dropped lo lo term and the residual of the split
// are below 2^-16 relative, far inside the FP32-level tolerance, at a sixth of
// the matrix-core time of FP32 MFMAs.  The G operands are split once per tile
// and stay in registers; the semantic features are split when staged.  The
// walk reads S from, and writes w back in place to, a per-wavefront 16 x 68
// FP32 LDS buffer.  The 16 record slots go through the wave reduce-scatter
// as in the plain kernel.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kGrp = 16;      // list entries per MFMA group
constexpr int kWbStride = 68;  // floats per row of the S / w buffer
constexpr int kSemRow = 72;    // bf16 per staged feature row: 32 hi, 32 lo, 8 pad

__host__ __device__ constexpr size_t bwd_mfma_lds(int batch, int NW)
{
    return (size_t)batch * (64 + 2 * kSemRow + 4 + 4) + (size_t)NW * kGrp * kWbStride * 4;
}

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ mf4 mfma3(const bf8 &ah, const bf8 &al, const bf8 &bh, const bf8 &bl, mf4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    return c;
}

template <int TW, int TH, int CO, int DM>
// Four wavefronts per SIMD (at most 128 registers per lane): the kernel is bound
// by VALU issue and dependency latency, and a fourth wavefront hides enough of
// the latter to pay for the tighter register budget (no spills).
__global__ void __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(4))) render_bwd_mfma_kernel(
    const DevCam *__restrict__ cams, int V, int64_t N, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const float4 *__restrict__ rec, const float *__restrict__ sem, int C_o,
    const float *__restrict__ T_final, const uint32_t *__restrict__ n_contrib, const float *__restrict__ up_rgb,
    const float *__restrict__ gD_img, const float *__restrict__ up_kmap, const float *__restrict__ up_sem,
    float *__restrict__ grec, float *__restrict__ dsem, int batch, uint32_t ntiles, int depth_mode, const float *__restrict__ hrec,
    SemSeed seed)
{
    static_assert(CO == 16 || CO == 32, "MFMA backward: C_o padded to 16 or 32");
    constexpr int NT = TW * TH;
    constexpr int NCB = CO / 16;  // 16-channel blocks of the dO product
    extern __shared__ float4 smem[];
    __shared__ uint32_t s_max;
    float4 *srec = smem;
    __bf16 *ssem = (__bf16 *)(smem + 4 * batch);  // [batch][kSemRow]: hi c0..31, lo c0..31
    uint32_t *sid = (uint32_t *)(ssem + (size_t)batch * kSemRow);
    const int wave = (int)(threadIdx.x >> 6);
    float *wb = (float *)(sid + batch) + wave * (kGrp * kWbStride);
    float *shh = DM == 2 ? (float *)(sid + batch) + (TW * TH / 64) * (kGrp * kWbStride) : nullptr;
    const uint32_t slot = xcd_tile(blockIdx.x, ntiles);
    if (slot >= ntiles) return;
    const TileInfo ti = tile_info<TW, TH>(cams, V, slot);
    const uint32_t tile = ti.tile;
    const uint2 range = ranges[tile];
    const float fx = (float)ti.px, fy = (float)ti.py;
    const int64_t recbase = (int64_t)ti.v * N;
    const int lane = __lane_id();
    const int l16 = lane & 15, h16 = lane >> 4;

    // upstream semantic gradients of the wavefront's 8 x 8 pixels, split, in the
    // two B-operand layouts: SB[pb] = G[16 pb + l16][8 h16 + e] (S product,
    // pixel = column, channel = reduction index) and DB[kk][cb] =
    // G[32 kk + 8 h16 + e][16 cb + l16] (dO product, pixel = reduction index)
    const int W = cams[ti.v].W, H = cams[ti.v].H;
    const int qx0 = ti.px - (lane & 7), qy0 = ti.py - (lane >> 3);
    // fused seed: each lane's own pixel's log-sum-exp, label and scale, read by
    // the lanes that stage that pixel's values
    const bool fused = !up_sem && seed.label;
    float my_lse = 0.f, my_sc = 0.f;
    int my_lab = -1;
    if (fused && ti.inside) seed_pixel(seed, C_o, ti.off, ti.HW, ti.pix, my_lse, my_lab, my_sc);
    auto up_at = [&](int p, int c) -> float {
        const int x = qx0 + (p & 7), y = qy0 + (p >> 3);
        if (fused) {
            const float l = __shfl(my_lse, p, 64), sc = __shfl(my_sc, p, 64);
            const int lb = __shfl(my_lab, p, 64);
            if (c >= C_o || x >= W || y >= H) return 0.f;
            const float o = seed.logits[(int64_t)C_o * ti.off + (int64_t)c * ti.HW + (int64_t)y * W + x];
            return sc * (__expf(o - l) - (c == lb ? 1.f : 0.f));
        }
        if (!up_sem || c >= C_o || x >= W || y >= H) return 0.f;
        return up_sem[(int64_t)C_o * ti.off + (int64_t)c * ti.HW + (int64_t)y * W + x];
    };
    bf8 SBh[4], SBl[4], DBh[2][NCB], DBl[2][NCB];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 h, l;
            split_bf16(up_at(16 * pb + l16, 8 * h16 + e), h, l);
            SBh[pb][e] = h;
            SBl[pb][e] = l;
        }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                __bf16 h, l;
                split_bf16(up_at(32 * kk + 8 * h16 + e, 16 * cb + l16), h, l);
                DBh[kk][cb][e] = h;
                DBl[kk][cb][e] = l;
            }

    double T = 1.0;
    float gR = 0.f, gG = 0.f, gB = 0.f, gDp = 0.f, gK = 0.f;
    uint32_t last = 0;
    if (ti.inside) {
        const int64_t p = ti.pix, HW = ti.HW, off = ti.off;
        T = T_final[off + p];
        const uint32_t rel = n_contrib[off + p];
        last = rel ? range.x + rel : 0u;
        if (up_rgb) {
            gR = up_rgb[3 * off + p];
            gG = up_rgb[3 * off + HW + p];
            gB = up_rgb[3 * off + 2 * HW + p];
        }
        gDp = gD_img[off + p];
        if (up_kmap) gK = up_kmap[off + p];
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (last) atomicMax(&s_max, last);
    __syncthreads();
    const uint32_t end_all = s_max;
    uint32_t wave_last = last;
    for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, o, 64));
    wave_last = __builtin_amdgcn_readfirstlane(wave_last);
    float A = 0.f;
    constexpr bool HIT = DM == 2;
    constexpr float kd = DM == 1 ? 0.f : 1.f;  // depth form fixed per instantiation

    for (uint32_t end = end_all; end > range.x;) {
        const uint32_t start = end - range.x > (uint32_t)batch ? end - (uint32_t)batch : range.x;
        const int n = (int)(end - start);
        __syncthreads();
        stage_records<NT>(srec, vals, start, n, rec, recbase);
        // features, split: 32 channels per row (zero beyond C_o)
        staged_copy<NT, 4, float>(
            n * 32, [&](int q) { return vals[start + (q >> 5)]; },
            [&](int q, uint32_t id) {
                const int c = q & 31;
                return c < C_o ? sem[(int64_t)id * C_o + c] : 0.f;
            },
            [&](int q, float x) {
                const int e = q >> 5, c = q & 31;
                __bf16 h, l;
                split_bf16(x, h, l);
                ssem[e * kSemRow + c] = h;
                ssem[e * kSemRow + 32 + c] = l;
            });
        for (int q = threadIdx.x; q < n; q += NT) sid[q] = vals[start + q];
        stage_hits<NT, HIT>(shh, vals, start, n, hrec, recbase);
        __syncthreads();
        const int ngrp = (n + kGrp - 1) / kGrp;
        for (int grp = ngrp - 1; grp >= 0; --grp) {
            const int j0 = grp * kGrp;
            if (start + (uint32_t)j0 >= wave_last) continue;  // beyond every pixel of this wavefront
            // S[f][p] for the group's 16 entries (rows past n hold stale data; their w is 0)
            {
                const __bf16 *row = ssem + (j0 + l16) * kSemRow + 8 * h16;
                const bf8 ah = *(const bf8 *)row, al = *(const bf8 *)(row + 32);
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) {
                    const mf4 d = mfma3(ah, al, SBh[pb], SBl[pb], mf4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                    for (int r = 0; r < 4; ++r) wb[(4 * h16 + r) * kWbStride + 16 * pb + l16] = d[r];
                }
            }
            __builtin_amdgcn_wave_barrier();
            // reverse walk over the group
            for (int jj = kGrp - 1; jj >= 0; --jj) {
                const int j = j0 + jj;
                const uint32_t entry = start + (uint32_t)j;
                const float s_sem = wb[jj * kWbStride + lane];
                float w = 0.f;
                if (j < n && entry < wave_last) {
                    const float4 r0 = srec[4 * j], r1 = srec[4 * j + 1];
                    const float dx = fx - r0.x, dy = fy - r0.y;
                    const float t1 = r0.z * dx + r0.w * dy, t2 = r1.x * dy;
                    const float G = gauss_of(t1, t2);
                    const float oG = r1.y * G;
                    const float alpha = fminf(kAlphaMax, oG);
                    const bool contrib = entry < last && alpha >= kAlphaMin;
                    if (__any(contrib)) {
                        float v[16];
                        const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
                        w = frag_adjoint(contrib, r0, r1, r2, r3, dx, dy, t1, t2, G, oG, alpha, s_sem, gR, gG, gB,
                                         gDp, gK, frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy), T, A, v);
                        const float tot = reduce_scatter<16>(v);
                        if ((lane & 3) == 0)
                            unsafeAtomicAdd(&grec[(recbase + sid[j]) * kRecFloats + (lane >> 2)], tot);
                    }
                }
                wb[jj * kWbStride + lane] = w;
            }
            __builtin_amdgcn_wave_barrier();
            // dO[f][c] += sum_p w[f][p] G[p][c]: A = w rows, split on the fly
            mf4 ad[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) ad[cb] = mf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const float *src = wb + l16 * kWbStride + 32 * kk + 8 * h16;
                const float4 x0 = *(const float4 *)src, x1 = *(const float4 *)(src + 4);
                const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                bf8 ah, al;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    __bf16 h, l;
                    split_bf16(xs[e], h, l);
                    ah[e] = h;
                    al[e] = l;
                }
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) ad[cb] = mfma3(ah, al, DBh[kk][cb], DBl[kk][cb], ad[cb]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = j0 + 4 * h16 + r;
                if (f < n) {
                    const int64_t row = (int64_t)sid[f] * C_o;
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const int c = 16 * cb + l16;
                        const float val = ad[cb][r];
                        if (c < C_o && val != 0.f) unsafeAtomicAdd(&dsem[row + c], val);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        end = start;
    }
}

// ------------------------------------------------------------------------
// Forward with the semantic blend on the matrix cores (C_o padded to 16 or 32).
// The walk is the plain kernel's, without the per-fragment channel loop: each
// lane writes its FP32 weight w_i (0 when the entry does not contribute) to a
// per-wavefront 16 x 68 LDS buffer, and after every 16 entries the wavefront
// adds O~[p][c] += sum_f w_f[p] o_f[c] with bf16 MFMAs (16x16x16) on hi/lo
// splits of both operands (three products, FP32 accumulation, as in the
// backward).  The accumulators O~ stay in the MFMA output layout until the
// end of the tile.  Colour, depth, gradient factor, T_final and n_contrib are
// computed exactly as in the plain kernel; the semantic map differs from it
// by rounding only (the matrix-core sums group the list entries per tile).
typedef short bs4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16_bits(float x, short &hi, short &lo)
{
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(short, h);
    lo = __builtin_bit_cast(short, l);
}

__device__ __forceinline__ mf4 mfma3k16(const bs4 &ah, const bs4 &al, const bs4 &bh, const bs4 &bl, mf4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    return c;
}

__host__ __device__ constexpr int fwd_semT_stride(int batch) { return batch + 4; }

__host__ __device__ constexpr size_t fwd_mfma_lds(int batch, int CO, int NW)
{
    return (size_t)batch * (64 + 4) + (size_t)2 * CO * fwd_semT_stride(batch) * 2 + (size_t)NW * kGrp * kWbStride * 4;
}

template <int TW, int TH, int CO, int DM>
__global__ void __launch_bounds__(TW *TH) render_fwd_mfma_kernel(
    const DevCam *__restrict__ cams, int V, int64_t N, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const float4 *__restrict__ rec, const float *__restrict__ sem, int C_o,
    ugs_outputs out, int batch, DevCounters *__restrict__ cnt, int count, uint32_t ntiles, int depth_mode, const float *__restrict__ hrec,
    int half_out)
{
    static_assert(CO == 16 || CO == 32, "MFMA forward: C_o padded to 16 or 32");
    constexpr int NT = TW * TH;
    constexpr int NCB = CO / 16;
    extern __shared__ float4 smem[];
    float4 *srec = smem;
    const int RS = fwd_semT_stride(batch);
    short *semh = (short *)(smem + 4 * batch);  // [CO][RS]: bf16 hi of o_f[c], transposed
    short *seml = semh + CO * RS;
    const int wave = (int)(threadIdx.x >> 6);
    float *wb = (float *)(seml + CO * RS) + wave * (kGrp * kWbStride);
    float *shh = DM == 2 ? (float *)(seml + CO * RS) + (NT / 64) * (kGrp * kWbStride) : nullptr;
    const uint32_t slot = xcd_tile(blockIdx.x, ntiles);
    if (slot >= ntiles) return;
    const TileInfo ti = tile_info<TW, TH>(cams, V, slot);
    const uint32_t tile = ti.tile;
    const uint2 range = ranges[tile];
    const float fx = (float)ti.px, fy = (float)ti.py;
    const int64_t recbase = (int64_t)ti.v * N;
    const int lane = __lane_id();
    const int l16 = lane & 15, h16 = lane >> 4;

    double T = 1.0, D = 0.0;
    float cr = 0.f, cg = 0.f, cb = 0.f, K = 0.f;
    mf4 acc[4][NCB];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int q = 0; q < NCB; ++q) acc[pb][q] = mf4{0.f, 0.f, 0.f, 0.f};
    uint32_t last = 0, n_eval = 0, n_con = 0;
    bool done = !ti.inside;
    constexpr bool HIT = DM == 2;
    constexpr float kd = DM == 1 ? 0.f : 1.f;  // depth form fixed per instantiation

    for (uint32_t start = range.x; start < range.y; start += (uint32_t)batch) {
        if (__syncthreads_count(done) == NT) break;
        const int n = (int)min((uint32_t)batch, range.y - start);
        stage_records<NT>(srec, vals, start, n, rec, recbase);
        // features, split and transposed: column f of row c (zero beyond C_o and past n)
        const int ng16 = (n + kGrp - 1) / kGrp * kGrp;
        staged_copy<NT, 4, float>(
            ng16 * CO, [&](int q) { return q / CO < n ? vals[start + q / CO] : 0u; },
            [&](int q, uint32_t id) {
                const int e = q / CO, c = q - e * CO;
                return e < n && c < C_o ? sem[(int64_t)id * C_o + c] : 0.f;
            },
            [&](int q, float x) {
                const int e = q / CO, c = q - e * CO;
                short h, l;
                split_bf16_bits(x, h, l);
                semh[c * RS + e] = h;
                seml[c * RS + e] = l;
            });
        stage_hits<NT, HIT>(shh, vals, start, n, hrec, recbase);
        __syncthreads();
        if (__all(done)) continue;  // the block may still walk this batch
        for (int j0 = 0; j0 < n; j0 += kGrp) {
            for (int jj = 0; jj < kGrp; ++jj) {
                const int j = j0 + jj;
                float wf = 0.f;
                if (j < n && !done) {
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
                            const float4 r2 = srec[4 * j + 2], r3 = srec[4 * j + 3];
                            const float kdj = frag_kd<HIT>(kd, shh, j, r2, r3, dx, dy);
                            const float B = kdj * (r2.x * dx + r2.y * dy);
                            const float Cq = kdj * (r2.z * dx * dx + 2.f * r2.w * dx * dy + r3.x * dy * dy);
                            const float d = r1.w * (1.f + B) * rcp_nr(1.f + 2.f * B + Cq);
                            const double w = (double)alpha * T;
                            wf = (float)w;
                            cr += wf * r3.y;
                            cg += wf * r3.z;
                            cb += wf * r3.w;
                            K += wf * r1.z;
                            D += w * (double)d;
                            T = tT;
                            last = start + (uint32_t)j + 1;
                            ++n_con;
                        }
                    }
                }
                wb[jj * kWbStride + lane] = wf;
            }
            __builtin_amdgcn_wave_barrier();
            // O~[p][c] += sum_f w[f][p] o[f][c] over the 16 entries
            bs4 bh[NCB], bl[NCB];
#pragma unroll
            for (int q = 0; q < NCB; ++q) {
                const int c = 16 * q + l16;
                bh[q] = *(const bs4 *)(semh + c * RS + j0 + 4 * h16);
                bl[q] = *(const bs4 *)(seml + c * RS + j0 + 4 * h16);
            }
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                bs4 ah, al;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    short h, l;
                    split_bf16_bits(wb[(4 * h16 + e) * kWbStride + 16 * pb + l16], h, l);
                    ah[e] = h;
                    al[e] = l;
                }
#pragma unroll
                for (int q = 0; q < NCB; ++q) acc[pb][q] = mfma3k16(ah, al, bh[q], bl[q], acc[pb][q]);
            }
            __builtin_amdgcn_wave_barrier();
            if (__all(done)) break;
        }
    }
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
    // O~ from the MFMA layout: acc[pb][q][r] is pixel 16 pb + 4 h16 + r, channel 16 q + l16
    {
        const int W = cams[ti.v].W, H = cams[ti.v].H;
        const int qx0 = ti.px - (lane & 7), qy0 = ti.py - (lane >> 3);
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = 16 * pb + 4 * h16 + r;
                const int x = qx0 + (pp & 7), y = qy0 + (pp >> 3);
                if (x < W && y < H) {
#pragma unroll
                    for (int q = 0; q < NCB; ++q) {
                        const int c = 16 * q + l16;
                        if (c < C_o)
                            put_out(out.sem, (int64_t)C_o * ti.off + (int64_t)c * ti.HW + (int64_t)y * W + x,
                                    acc[pb][q][r], half_out);
                    }
                }
            }
    }
    if (count) {
        unsigned long long e = n_eval, c = n_con;
        for (int o = 32; o > 0; o >>= 1) {
            e += __shfl_xor(e, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if (__lane_id() == 0) {
            atomicAdd(&cnt->n_eval, e);
            atomicAdd(&cnt->n_contrib, c);
        }
    }
}

template <int TW, int TH, int CO>
hipError_t fwd_dispatch(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                        const ugs_outputs &out, int batch, bool counters, int final_buf, hipStream_t s)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto ranges = (const uint2 *)(ws + L.ranges);
    auto vals = (const uint32_t *)(ws + (final_buf ? L.vals1 : L.vals0));
    auto rec = (const float4 *)(ws + L.rec);
    auto cnt = (DevCounters *)(ws + L.counters);
    auto hrec = (const float *)(ws + L.hrec);
    if constexpr (CO == 16 || CO == 32) {
        // whole MFMA groups per batch, at most 64 KB of LDS per workgroup
        constexpr int NW = TW * TH / 64;
        int b = (batch + kGrp - 1) / kGrp * kGrp;
        while (b > kGrp && fwd_mfma_lds(b, CO, NW) > 64 * 1024) b -= kGrp;
        auto k = pb.depth_mode == 2 ? render_fwd_mfma_kernel<TW, TH, CO, 2>
                 : pb.depth_mode == 1 ? render_fwd_mfma_kernel<TW, TH, CO, 1> : render_fwd_mfma_kernel<TW, TH, CO, 0>;
        hipLaunchKernelGGL(k, dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), fwd_mfma_lds(b, CO, NW), s, cams, pb.V,
                           pb.N, ranges, vals, rec, g.sem, pb.C_o, out, b, cnt, (int)counters,
                           (uint32_t)pb.total_tiles, pb.depth_mode, hrec, pb.half_out);
    } else {
        size_t lds = (size_t)batch * (64 + 4 * CO + 4);
        auto k = pb.depth_mode == 2 ? render_fwd_kernel<TW, TH, CO, 2>
                 : pb.depth_mode == 1 ? render_fwd_kernel<TW, TH, CO, 1> : render_fwd_kernel<TW, TH, CO, 0>;
        hipLaunchKernelGGL(k, dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), lds, s,
                           cams, pb.V, pb.N, ranges, vals, rec, g.sem, pb.C_o, out, batch, cnt, (int)counters,
                           (uint32_t)pb.total_tiles, pb.depth_mode, hrec, pb.half_out);
    }
    return hipGetLastError();
}

template <int TW, int TH, int CO>
hipError_t bwd_dispatch(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                        const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg, int batch,
                        int final_buf, hipStream_t s)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto ranges = (const uint2 *)(ws + L.ranges);
    auto vals = (const uint32_t *)(ws + (final_buf ? L.vals1 : L.vals0));
    auto rec = (const float4 *)(ws + L.rec);
    auto grec = (float *)(ws + L.grec);
    auto gd = (const float *)(ws + L.gd);
    auto hrec = (const float *)(ws + L.hrec);
    const SemSeed seed{out.sem, up.sem ? nullptr : up.sem_label, up.sem_scale};
    if constexpr (CO == 16 || CO == 32) {
        // whole MFMA groups per batch, at most 64 KB of LDS per workgroup
        constexpr int NW = TW * TH / 64;
        int b = (batch + kGrp - 1) / kGrp * kGrp;
        while (b > kGrp && bwd_mfma_lds(b, NW) > 64 * 1024) b -= kGrp;
        auto k = pb.depth_mode == 2 ? render_bwd_mfma_kernel<TW, TH, CO, 2>
                 : pb.depth_mode == 1 ? render_bwd_mfma_kernel<TW, TH, CO, 1> : render_bwd_mfma_kernel<TW, TH, CO, 0>;
        hipLaunchKernelGGL(k, dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), bwd_mfma_lds(b, NW), s, cams, pb.V, pb.N, ranges, vals, rec, g.sem, pb.C_o,
                           out.T_final, out.n_contrib, up.rgb, gd, up.kmap, up.sem, grec, dg.sem, b,
                           (uint32_t)pb.total_tiles, pb.depth_mode, hrec, seed);
    } else {
        size_t lds = (size_t)batch * (64 + 4 * CO + 4);
        auto k = pb.depth_mode == 2 ? render_bwd_kernel<TW, TH, CO, 2>
                 : pb.depth_mode == 1 ? render_bwd_kernel<TW, TH, CO, 1> : render_bwd_kernel<TW, TH, CO, 0>;
        hipLaunchKernelGGL(k, dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), lds, s,
                           cams, pb.V, pb.N, ranges, vals, rec, g.sem, pb.C_o, out.T_final, out.n_contrib, up.rgb, gd,
                           up.kmap, up.sem, grec, dg.sem, batch, (uint32_t)pb.total_tiles, pb.depth_mode, hrec, seed);
    }
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t fwd_co(int co_pad, const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                  const ugs_outputs &out, int batch, bool counters, int fb, hipStream_t s)
{
    switch (co_pad) {
    case 0: return fwd_dispatch<TW, TH, 0>(g, pb, L, ws, out, batch, counters, fb, s);
    case 8: return fwd_dispatch<TW, TH, 8>(g, pb, L, ws, out, batch, counters, fb, s);
    case 16: return fwd_dispatch<TW, TH, 16>(g, pb, L, ws, out, batch, counters, fb, s);
    default: return fwd_dispatch<TW, TH, 32>(g, pb, L, ws, out, batch, counters, fb, s);
    }
}

template <int TW, int TH>
hipError_t bwd_co(int co_pad, const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                  const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg, int batch, int fb,
                  hipStream_t s)
{
    switch (co_pad) {
    case 0: return bwd_dispatch<TW, TH, 0>(g, pb, L, ws, out, up, dg, batch, fb, s);
    case 8: return bwd_dispatch<TW, TH, 8>(g, pb, L, ws, out, up, dg, batch, fb, s);
    case 16: return bwd_dispatch<TW, TH, 16>(g, pb, L, ws, out, up, dg, batch, fb, s);
    default: return bwd_dispatch<TW, TH, 32>(g, pb, L, ws, out, up, dg, batch, fb, s);
    }
}

}  // namespace

int channel_pad(int C_o)
{
    if (C_o <= 0) return 0;
    if (C_o <= 8) return 8;
    if (C_o <= 16) return 16;
    if (C_o <= 32) return 32;
    if (C_o <= 64) return 64;
    if (C_o <= 128) return 128;
    return 256;
}

// 0..8 channels: the vector kernels; 9..32 with the split-bf16 option: the
// split-bf16 matrix-core kernels; otherwise the FP32 matrix-core kernels.
static bool use_f32_mm(const Problem &pb) { return pb.C_o > 8 && !(pb.sem_bf16x3 && pb.C_o <= 32); }

hipError_t launch_render_fwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                             const ugs_outputs &out, int batch, bool counters, int final_buf, hipStream_t s)
{
    if (pb.total_tiles == 0) return hipSuccess;
    if (use_f32_mm(pb)) return launch_render_fwd_mm(g, pb, L, ws, out, batch, counters, final_buf, s);
    int cp = channel_pad(pb.C_o);
    if (pb.tile_w == 8 && pb.tile_h == 8) return fwd_co<8, 8>(cp, g, pb, L, ws, out, batch, counters, final_buf, s);
    if (pb.tile_w == 32 && pb.tile_h == 8) return fwd_co<32, 8>(cp, g, pb, L, ws, out, batch, counters, final_buf, s);
    return fwd_co<16, 16>(cp, g, pb, L, ws, out, batch, counters, final_buf, s);
}

hipError_t launch_render_bwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                             const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg,
                             int batch, int final_buf, bool counters, hipStream_t s)
{
    if (pb.total_tiles == 0) return hipSuccess;
    if (use_f32_mm(pb)) return launch_render_bwd_mm(g, pb, L, ws, out, up, dg, batch, final_buf, counters, s);
    int cp = channel_pad(pb.C_o);
    if (pb.tile_w == 8 && pb.tile_h == 8) return bwd_co<8, 8>(cp, g, pb, L, ws, out, up, dg, batch, final_buf, s);
    if (pb.tile_w == 32 && pb.tile_h == 8) return bwd_co<32, 8>(cp, g, pb, L, ws, out, up, dg, batch, final_buf, s);
    return bwd_co<16, 16>(cp, g, pb, L, ws, out, up, dg, batch, final_buf, s);
}

}  // namespace ugs
