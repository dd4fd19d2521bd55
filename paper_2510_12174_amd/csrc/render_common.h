// Device helpers shared by the render kernels (stages S5 and S8): wavefront
// reductions, the Gaussian falloff, the fused cross-entropy seed, the per-
// fragment adjoint of Alg. backward_render, tile geometry and LDS staging.
#pragma once
#include "ugs_internal.h"

namespace ugs {
namespace {

// ---------------------------------------------------------------- wave64 sum
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_step(float x)
{
    int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xf, false);
    return x + __int_as_float(y);
}

// Sum over the 64 lanes; the result is returned (uniform) in every lane.
// All 64 lanes must be active.
__device__ __forceinline__ float wave_sum(float x)
{
    x = dpp_step<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
    x = dpp_step<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
    x = dpp_step<0x124, 0xf>(x);  // row_ror:4
    x = dpp_step<0x128, 0xf>(x);  // row_ror:8
    x = dpp_step<0x142, 0xa>(x);  // row_bcast:15
    x = dpp_step<0x143, 0xc>(x);  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Returns `s` in lane `lane` and `v` elsewhere.
__device__ __forceinline__ float put_lane(float v, float s, int lane) { return __lane_id() == lane ? s : v; }

template <int CTRL>
__device__ __forceinline__ float dpp_add_sel(float a, float b, bool take_b)
{
    const float ta = dpp_step<CTRL, 0xf>(a);
    const float tb = dpp_step<CTRL, 0xf>(b);
    return take_b ? tb : ta;
}

// One level of the transposed reduce-scatter inside a 16-lane row: registers
// k and k + N/2 are added to their DPP-permuted copies and each lane keeps the
// sum selected by its lane bit; a single register is just added (the result is
// then duplicated across the lane pair).
template <int CTRL, int N>
__device__ __forceinline__ void dpp_level(const float (&in)[N], float (&out)[N > 1 ? N / 2 : 1], bool bit)
{
    if constexpr (N > 1) {
#pragma unroll
        for (int k = 0; k < N / 2; ++k) out[k] = dpp_add_sel<CTRL>(in[k], in[k + N / 2], bit);
    } else {
        out[0] = dpp_step<CTRL, 0xf>(in[0]);
    }
}

// Transposed reduce-scatter over a wavefront: x[0..NV-1] are NV per-lane values
// (NV = 8, 16, 32 or 64); on return each lane l holds the sum over all 64 lanes
// of x[l >> (6 - log2 NV)], so value q sits in the 64/NV lanes starting at
// q * 64/NV.  Two cross-half swap levels (v_permlane32_swap, v_permlane16_swap)
// halve the register count at one swap and one add per register pair, then four
// DPP levels inside each 16-lane row (rotate by 8, half mirror, quad permutes)
// finish with a select on the lane's bit; once one register is left the
// remaining levels are plain adds.  For NV = 64 this is about 2.2 VALU
// instructions per value, against 7 for a separate DPP tree per value, and the
// cost scales with NV.  All 64 lanes must be active.
template <int NV>
__device__ __forceinline__ float reduce_scatter(const float (&x)[NV])
{
    static_assert(NV == 8 || NV == 16 || NV == 32 || NV == 64, "reduce_scatter: NV must be 8, 16, 32 or 64");
    constexpr int N1 = NV / 2, N2 = NV / 4;
    const int lane = __lane_id();
    float s[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[k]), __float_as_uint(x[k + N1]), false, false);
        s[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float u[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(s[k]), __float_as_uint(s[k + N2]), false, false);
        u[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    constexpr int N3 = N2 > 1 ? N2 / 2 : 1, N4 = N3 > 1 ? N3 / 2 : 1, N5 = N4 > 1 ? N4 / 2 : 1;
    float v[N3], w[N4], y[N5], z[1];
    dpp_level<0x128, N2>(u, v, lane & 8);  // row_ror:8
    dpp_level<0x141, N3>(v, w, lane & 4);  // row_half_mirror
    dpp_level<0x4E, N4>(w, y, lane & 2);   // quad_perm [2,3,0,1]
    dpp_level<0xB1, N5>(y, z, lane & 1);   // quad_perm [1,0,3,2]
    return z[0];
}

// exp(-(t1^2 + t2^2) / 2) as one multiply and the hardware 2^x: the constant
// -log2(e) / 2 is folded, so forward and backward evaluate the same expression.
__device__ __forceinline__ float gauss_of(float t1, float t2)
{
    return __builtin_amdgcn_exp2f((t1 * t1 + t2 * t2) * -0.72134752044448170f);
}

// 1/x: hardware reciprocal (1 ulp) refined by one Newton step.
__device__ __forceinline__ float rcp_nr(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.f), r);
}

// Fused cross-entropy seed: with no upstream semantic map, the backward forms
// dL/dO~ = scale (softmax(O~) - onehot(label)) per pixel from the rendered
// logits (a label outside [0, C_o) gives 0).
struct SemSeed {
    const float *logits;   // rendered O~, layout of ugs_outputs.sem
    const int32_t *label;  // [H][W] per view, NULL: no fused seed
    const float *scale;    // device scalar
};

// Log-sum-exp over the C_o channels of one pixel (stride HW), the label and
// the seed's scale for that pixel (0 for an out-of-range label).
__device__ __forceinline__ void seed_pixel(const SemSeed &sd, int C_o, int64_t off, int64_t HW, int64_t p,
                                           float &lse, int &lab, float &sc)
{
    const float *o = sd.logits + (int64_t)C_o * off + p;
    float m = -INFINITY, s = 0.f;
    for (int c = 0; c < C_o; ++c) {
        const float x = o[(int64_t)c * HW], mn = fmaxf(m, x);
        s = s * __expf(m - mn) + __expf(x - mn);
        m = mn;
    }
    lse = m + __logf(s);
    lab = sd.label[off + p];
    sc = (lab >= 0 && lab < C_o) ? *sd.scale : 0.f;
}

// 1/x in FP64: hardware reciprocal refined by one Newton step (x in [0.01, 1]).
__device__ __forceinline__ double rcp64(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// One reverse step of Alg. backward_render for one pixel and one list entry.
// Restores T in FP64 (T <- T / (1 - alpha), the exact inverse of the forward's
// FP64 T <- T (1 - alpha) up to one rounding), advances the running sum A of
// w_j s_j over the later fragments, and fills v[0..15] with this pixel's share
// of the entry's gradient record (mean2d 0-1, Cholesky conic 2-4, opacity 5,
// gradient factor 6, depth coefficients z0 7, beta 8-9, gamma 10-12, colour
// 13-15); returns the blending weight w = alpha T, rounded to FP32 from FP64 as
// in the forward.  s_sem is the semantic part of s_i.  The depth is
// d = z0 (1 + B) / (1 + 2B + Cq) (the ray-ellipsoid midpoint in the per-record
// quadric form); kd = 0 selects the centre depth d = z0.  Branch-free: a lane
// with contrib == false gets w = 0 and v = 0 and keeps T and A.
__device__ __forceinline__ float frag_adjoint(bool contrib, float4 r0, float4 r1, float4 r2, float4 r3, float dx,
                                              float dy, float t1, float t2, float G, float oG, float alpha,
                                              float s_sem, float gR, float gG, float gB, float gDp, float gK,
                                              float kd, double &T, float &A, float (&v)[16])
{
    const float rom = rcp_nr(1.f - alpha);
    const double Tn = contrib ? T * rcp64(1.0 - (double)alpha) : T;
    const float w = contrib ? (float)((double)alpha * Tn) : 0.f;
    const float Tf = (float)Tn;
    const float B = kd * (r2.x * dx + r2.y * dy);
    const float Cq = kd * (r2.z * dx * dx + 2.f * r2.w * dx * dy + r3.x * dy * dy);
    const float iden = __builtin_amdgcn_rcpf(1.f + 2.f * B + Cq);  // 1 ulp: feeds gradients only
    const float z0 = r1.w;
    const float d = z0 * (1.f + B) * iden;
    const float s = gR * r3.y + gG * r3.z + gB * r3.w + gDp * d + gK * r1.z + s_sem;
    const float dalpha = contrib ? Tf * s - A * rom : 0.f;
    A += w * s;
    T = Tn;
    v[13] = w * gR;
    v[14] = w * gG;
    v[15] = w * gB;
    v[6] = w * gK;
    const float dd = w * gDp;
    const float i2 = iden * iden;
    const float dB = kd * dd * z0 * (Cq - 1.f) * i2;
    const float dC = -kd * dd * z0 * (1.f + B) * i2;
    v[7] = dd * (1.f + B) * iden;
    v[8] = dB * dx;
    v[9] = dB * dy;
    v[10] = dC * dx * dx;
    v[11] = 2.f * dC * dx * dy;
    v[12] = dC * dy * dy;
    // alpha = min(0.99, o G): no gradient through the clamp
    const bool free_ = oG < kAlphaMax;
    const float dpow = free_ ? dalpha * oG : 0.f;
    v[5] = free_ ? dalpha * G : 0.f;
    v[2] = -t1 * dx * dpow;
    v[3] = -t1 * dy * dpow;
    v[4] = -t2 * dy * dpow;
    // the pixel offset is (pixel - mean2d): d/d(mean2d) = -d/d(dx, dy)
    v[0] = t1 * r0.z * dpow - (dB * r2.x + dC * 2.f * (r2.z * dx + r2.w * dy));
    v[1] = (t1 * r0.w + t2 * r1.x) * dpow - (dB * r2.y + dC * 2.f * (r2.w * dx + r3.x * dy));
    return w;
}

struct TileInfo {
    uint32_t tile;  // global tile id (row-major within its view)
    int v, px, py;
    bool inside;
    int64_t pix;  // pixel index within the view
    int64_t HW, off;
};

// The tile that workgroup slot `slot` (from xcd_tile) processes, and this
// lane's pixel in it.  (A super-tile order of the slots, 8 x 4 tiles per run
// of 32 slots on one XCD instead of a strip of one tile row, measured the same
// on the 3M- and 1M-Gaussian 16-view steps.)
template <int TW, int TH>
__device__ __forceinline__ TileInfo tile_info(const DevCam *cams, int V, uint32_t slot)
{
    TileInfo ti;
    ti.tile = slot;
    ti.v = view_of_tile(cams, V, slot);
    const DevCam &cam = cams[ti.v];
    const uint32_t lt = slot - cam.tile_base;
    const int tx = (int)(lt % (uint32_t)cam.tiles_x), ty = (int)(lt / (uint32_t)cam.tiles_x);
    // each wavefront covers a compact 8 x 8 (or 8-row) block of the tile
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
    constexpr int WX = TW / 8;  // wavefronts per tile row
    ti.px = tx * TW + (wave % WX) * 8 + (lane & 7);
    ti.py = ty * TH + (wave / WX) * 8 + (lane >> 3);
    ti.inside = ti.px < cam.W && ti.py < cam.H;
    ti.HW = (int64_t)cam.W * cam.H;
    ti.pix = (int64_t)ti.py * cam.W + ti.px;
    ti.off = cam.pix_off;
    return ti;
}

// Whether the pixel ray meets the Gaussian's ellipsoid, i.e. the quadratic of
// section 3.2 has a real root (depth_mode 2).  In the per-record quadric form
// the smallest Mahalanobis distance along the ray is h (Cq - B^2) / (1 + 2B + Cq)
// with h = z0^2 p0^T Q p0, so the ray hits where h (Cq - B^2) <= 1 + 2B + Cq.
// Non-contracting operations: the forward and backward kernels take the same
// decision bit for bit.
__device__ __forceinline__ bool ray_hits(float h, float4 r2, float4 r3, float dx, float dy)
{
    const float B = __fadd_rn(__fmul_rn(r2.x, dx), __fmul_rn(r2.y, dy));
    const float Cq = __fadd_rn(__fadd_rn(__fmul_rn(__fmul_rn(r2.z, dx), dx), __fmul_rn(__fmul_rn(__fmul_rn(2.f, r2.w), dx), dy)),
                               __fmul_rn(__fmul_rn(r3.x, dy), dy));
    return __fmul_rn(h, __fsub_rn(Cq, __fmul_rn(B, B))) <= __fadd_rn(__fadd_rn(1.f, __fmul_rn(2.f, B)), Cq);
}

// Depth-form factor of one fragment: kd (1 midpoint, 0 centre), or, with the
// staged hit constants of depth_mode 2, 1 where the ray hits and 0 where not.
template <bool HIT>
__device__ __forceinline__ float frag_kd(float kd, const float *shh, int j, float4 r2, float4 r3, float dx, float dy)
{
    if constexpr (HIT)
        return ray_hits(shh[j], r2, r3, dx, dy) ? 1.f : 0.f;
    else
        return kd;
}

// Copies `total` items to LDS, G items per lane at a time (item q = q0 + NT u
// + thread): first the G list ids idx(q), then the G data loads load(q, id),
// then the G LDS writes store(q, value), so that each group costs two round
// trips to memory.  A plain loop would wait for every item's loads in turn.
template <int NT, int G, typename T, typename Idx, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int total, Idx idx, Load load, Store store)
{
    const int t = (int)threadIdx.x;
#pragma unroll 1
    for (int q0 = 0; q0 < total; q0 += NT * G) {
        // items past the end load the last item again: no branches around
        // the loads or stores, which the compiler would otherwise sink into
        // per-item conditional blocks, one round trip each
        uint32_t id[G];
#pragma unroll
        for (int u = 0; u < G; ++u) id[u] = idx(min(q0 + NT * u + t, total - 1));
        asm volatile("" ::: "memory");  // every id load issued before the first data load
        T v[G];
#pragma unroll
        for (int u = 0; u < G; ++u) v[u] = load(min(q0 + NT * u + t, total - 1), id[u]);
        // (the extra items rewrite the last item's slot with the same value)
#pragma unroll
        for (int u = 0; u < G; ++u) store(min(q0 + NT * u + t, total - 1), v[u]);
    }
}

// Stages the hit constants of `n` list entries (depth_mode 2 only).
template <int NT, bool HIT>
__device__ __forceinline__ void stage_hits(float *shh, const uint32_t *vals, uint32_t start, int n,
                                           const float *hrec, int64_t recbase)
{
    if constexpr (HIT)
        staged_copy<NT, 4, float>(
            n, [&](int q) { return vals[start + q]; }, [&](int, uint32_t id) { return hrec[recbase + id]; },
            [&](int q, float v) { shh[q] = v; });
}

// Stages the 4 float4 records of `n` list entries [start, start+n).
template <int NT, int G = 2>
__device__ __forceinline__ void stage_records(float4 *srec, const uint32_t *vals, uint32_t start, int n,
                                              const float4 *rec, int64_t recbase)
{
    staged_copy<NT, G, float4>(
        n * 4, [&](int q) { return vals[start + (q >> 2)]; },
        [&](int q, uint32_t id) { return rec[(recbase + id) * 4 + (q & 3)]; }, [&](int q, float4 v) { srec[q] = v; });
}

// Stage `n` list entries [start, start+n) into LDS: 4 float4 of record and CO
// semantic floats (zero beyond C_o) each.
template <int NT, int CO>
__device__ __forceinline__ void stage_batch(float4 *srec, float *ssem, const uint32_t *vals, uint32_t start, int n,
                                            const float4 *rec, int64_t recbase, const float *sem, int C_o)
{
    stage_records<NT>(srec, vals, start, n, rec, recbase);
    if constexpr (CO > 0)
        staged_copy<NT, 4, float>(
            n * CO, [&](int q) { return vals[start + q / CO]; },
            [&](int q, uint32_t id) {
                const int c = q % CO;
                return c < C_o ? sem[(int64_t)id * C_o + c] : 0.f;
            },
            [&](int q, float v) { ssem[q] = v; });
}

}  // namespace
}  // namespace ugs
