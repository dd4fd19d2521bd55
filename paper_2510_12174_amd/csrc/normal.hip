// Stages S6 and S7: normals from the rendered depth (Alg. normal_estimation,
// supplementary S1.3) and the backward from normals to depth (Alg.
// normal_gradient, supplementary S1.4), for gfx950.
//
// All geometry is done in the camera frame and rotated once: the world-frame
// finite differences are R^T times the camera-frame ones, so the cross product,
// the fusion, the normalisation and the zero test are rotation invariant.  The
// finite difference of back-projected points is written in difference form,
//   D+ p+ - D- p- = (D+ - D-) p(u,v) + (D+ + D-) (g/fx, 0, 0),
// because p is linear in the pixel coordinate; D+ - D- is exact in FP32 for
// nearby depths, which keeps the normal accurate where the depths nearly cancel.
//
// The backward is a gather: the adjoints of every pixel's four finite-difference
// vectors (12 floats) are formed first, then every pixel collects the terms of
// the up to eight stencils that read it -- in LDS within one workgroup (tile
// plus a halo of the larger step) for steps up to kHaloMax, else through memory
// in two passes.  No atomics, so the result is deterministic.
#include "ugs_internal.h"

namespace ugs {
namespace {

constexpr int kNT = 256;

struct NState {
    int state;  // 0 border, 1 degenerate, 2 valid
    bool flip;
    float sgn;
    float vx[2][3], vy[2][3];
    float n0[3], nn;
};

__device__ __forceinline__ void cross3(const float *a, const float *b, float *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ float dot3(const float *a, const float *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__device__ __forceinline__ void normal_state(const float *D, const DevCam &cam, int u, int v, int s1, int s2,
                                             float lam, int orient, NState &S)
{
    const int W = cam.W, H = cam.H;
    const int gm = s1 > s2 ? s1 : s2;
    S.state = 0;
    S.flip = false;
    S.sgn = 1.f;
    if (u - gm < 0 || u + gm >= W || v - gm < 0 || v + gm >= H) return;
    const float p[3] = {((float)u - cam.cx) / cam.fx, ((float)v - cam.cy) / cam.fy, 1.f};
    const int gs[2] = {s1, s2};
    float n[2][3];
    for (int k = 0; k < 2; ++k) {
        const int g = gs[k];
        const float dxp = D[(int64_t)v * W + u + g], dxm = D[(int64_t)v * W + u - g];
        const float dyp = D[(int64_t)(v + g) * W + u], dym = D[(int64_t)(v - g) * W + u];
        const float ddx = dxp - dxm, sdx = dxp + dxm, ddy = dyp - dym, sdy = dyp + dym;
        S.vx[k][0] = ddx * p[0] + sdx * ((float)g / cam.fx);
        S.vx[k][1] = ddx * p[1];
        S.vx[k][2] = ddx;
        S.vy[k][0] = ddy * p[0];
        S.vy[k][1] = ddy * p[1] + sdy * ((float)g / cam.fy);
        S.vy[k][2] = ddy;
        cross3(S.vx[k], S.vy[k], n[k]);
    }
    S.sgn = dot3(n[0], n[1]) < 0.f ? -1.f : 1.f;
    float nf[3];
    for (int c = 0; c < 3; ++c) nf[c] = lam * n[0][c] + (1.f - lam) * S.sgn * n[1][c];
    S.nn = sqrtf(dot3(nf, nf));
    const float thr = 1e-9f * sqrtf(dot3(S.vx[0], S.vx[0])) * sqrtf(dot3(S.vy[0], S.vy[0]));
    if (!(S.nn > thr)) {
        S.state = 1;
        return;
    }
    const float inn = 1.f / S.nn;
    for (int c = 0; c < 3; ++c) S.n0[c] = nf[c] * inn;
    // N . (C - P) = -D(u,v) (n_cam . p)
    const float nd = -D[(int64_t)v * W + u] * dot3(S.n0, p);
    S.flip = (float)orient * nd < 0.f;
    S.state = 2;
}

template <int TW, int TH>
__device__ __forceinline__ bool pixel_of(const DevCam *cams, int V, uint32_t ntiles, int &view, int &u, int &v)
{
    const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
    if (tile >= ntiles) return false;
    view = view_of_tile(cams, V, tile);
    const DevCam &cam = cams[view];
    const uint32_t lt = tile - cam.tile_base;
    u = (int)(lt % (uint32_t)cam.tiles_x) * TW + (int)(threadIdx.x % TW);
    v = (int)(lt / (uint32_t)cam.tiles_x) * TH + (int)(threadIdx.x / TW);
    return u < cam.W && v < cam.H;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH) normal_fwd_kernel(const DevCam *__restrict__ cams, int V, uint32_t ntiles,
                                                           const float *__restrict__ depth, float *__restrict__ normal,
                                                           int s1, int s2, float lam, int orient, int half_out)
{
    int view, u, v;
    if (!pixel_of<TW, TH>(cams, V, ntiles, view, u, v)) return;
    const DevCam &cam = cams[view];
    const int64_t HW = (int64_t)cam.W * cam.H, p = (int64_t)v * cam.W + u;
    NState S;
    normal_state(depth + cam.pix_off, cam, u, v, s1, s2, lam, orient, S);
    float N[3] = {0.f, 0.f, 0.f};
    if (S.state == 2) {
        const float sg = S.flip ? -1.f : 1.f;
        const float *R = cam.R;
        for (int c = 0; c < 3; ++c) N[c] = sg * (R[c] * S.n0[0] + R[3 + c] * S.n0[1] + R[6 + c] * S.n0[2]);
    }
    const int64_t o = 3 * cam.pix_off;
    put_out(normal, o + p, N[0], half_out);
    put_out(normal, o + HW + p, N[1], half_out);
    put_out(normal, o + 2 * HW + p, N[2], half_out);
}

// Adjoints of pixel (u, v)'s four finite-difference vectors (vx1, vy1, vx2,
// vy2) in the camera frame, from the upstream normal gradient of the pixel (or
// the fused cosine seed, scale * N_target).  D, dn and nt point at the view's
// first pixel (dn and nt: three planes of W H).
__device__ __forceinline__ void normal_adj_at(const DevCam &cam, const float *D, const float *dn, const float *nt,
                                              float nsc, int u, int v, int s1, int s2, float lam, int orient,
                                              float (&out)[12])
{
    const int64_t HW = (int64_t)cam.W * cam.H, p = (int64_t)v * cam.W + u;
    for (int k = 0; k < 12; ++k) out[k] = 0.f;
    float gw[3] = {0.f, 0.f, 0.f};
    if (dn) {
        gw[0] = dn[p];
        gw[1] = dn[HW + p];
        gw[2] = dn[2 * HW + p];
    } else if (nt) {
        gw[0] = nsc * nt[p];
        gw[1] = nsc * nt[HW + p];
        gw[2] = nsc * nt[2 * HW + p];
    }
    if (gw[0] != 0.f || gw[1] != 0.f || gw[2] != 0.f) {
        NState S;
        normal_state(D, cam, u, v, s1, s2, lam, orient, S);
        if (S.state == 2) {
            const float *R = cam.R;
            float g[3];
            for (int c = 0; c < 3; ++c) g[c] = R[3 * c] * gw[0] + R[3 * c + 1] * gw[1] + R[3 * c + 2] * gw[2];
            if (S.flip)
                for (int c = 0; c < 3; ++c) g[c] = -g[c];
            const float pr = dot3(S.n0, g), inn = 1.f / S.nn;
            float gn[3];
            for (int c = 0; c < 3; ++c) gn[c] = (g[c] - S.n0[c] * pr) * inn;
            const float wk[2] = {lam, (1.f - lam) * S.sgn};
            for (int k = 0; k < 2; ++k) {
                float gk[3] = {wk[k] * gn[0], wk[k] * gn[1], wk[k] * gn[2]};
                cross3(S.vy[k], gk, out + 6 * k);      // d/d vx = vy x g
                cross3(gk, S.vx[k], out + 6 * k + 3);  // d/d vy = g x vx
            }
        }
    }
}

// The gather for pixel (u, v): the terms of the up to eight stencils that read
// it, adj(k, du, dv) giving adjoint k of the stencil centred at (u + du, v + dv),
// projected on dP/dD = R^T p.
template <typename A>
__device__ __forceinline__ float normal_gather_at(const DevCam &cam, int u, int v, int s1, int s2, A adj)
{
    const int W = cam.W, H = cam.H;
    float gP[3] = {0.f, 0.f, 0.f};
    const int gs[2] = {s1, s2};
    for (int k = 0; k < 2; ++k) {
        const int g = gs[k];
        // this pixel is (u+g, v) of the stencil at (u-g, v): + d/d vx
        if (u - g >= 0)
            for (int c = 0; c < 3; ++c) gP[c] += adj(6 * k + c, -g, 0);
        if (u + g < W)
            for (int c = 0; c < 3; ++c) gP[c] -= adj(6 * k + c, g, 0);
        if (v - g >= 0)
            for (int c = 0; c < 3; ++c) gP[c] += adj(6 * k + 3 + c, 0, -g);
        if (v + g < H)
            for (int c = 0; c < 3; ++c) gP[c] -= adj(6 * k + 3 + c, 0, g);
    }
    const float pp[3] = {((float)u - cam.cx) / cam.fx, ((float)v - cam.cy) / cam.fy, 1.f};
    return dot3(gP, pp);
}

// Pass 1 of the two-pass form: adjoints, planar [12][pixels].
template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH) normal_adj_kernel(const DevCam *__restrict__ cams, int V, uint32_t ntiles,
                                                           const float *__restrict__ depth,
                                                           const float *__restrict__ dnormal,
                                                           const float *__restrict__ ntgt,
                                                           const float *__restrict__ nscale, int64_t total_pix,
                                                           float *__restrict__ adj, int s1, int s2, float lam,
                                                           int orient)
{
    int view, u, v;
    if (!pixel_of<TW, TH>(cams, V, ntiles, view, u, v)) return;
    const DevCam &cam = cams[view];
    const int64_t gp = cam.pix_off + (int64_t)v * cam.W + u;
    float out[12];
    normal_adj_at(cam, depth + cam.pix_off, dnormal ? dnormal + 3 * cam.pix_off : nullptr,
                  ntgt ? ntgt + 3 * cam.pix_off : nullptr, ntgt && !dnormal ? *nscale : 0.f, u, v, s1, s2, lam,
                  orient, out);
    for (int k = 0; k < 12; ++k) adj[k * total_pix + gp] = out[k];
}

// Pass 2 of the two-pass form: gathers the stored adjoints, adds the direct
// depth gradient and writes G_D.
template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH) normal_gather_kernel(const DevCam *__restrict__ cams, int V, uint32_t ntiles,
                                                              const float *__restrict__ adj, int64_t total_pix,
                                                              const float *__restrict__ ddepth, float *__restrict__ gd,
                                                              int s1, int s2)
{
    int view, u, v;
    if (!pixel_of<TW, TH>(cams, V, ntiles, view, u, v)) return;
    const DevCam &cam = cams[view];
    const int64_t q = cam.pix_off + (int64_t)v * cam.W + u;
    float r = normal_gather_at(cam, u, v, s1, s2, [&](int k, int du, int dv) {
        return adj[k * total_pix + q + du + (int64_t)dv * cam.W];
    });
    if (ddepth) r += ddepth[q];
    gd[q] = r;
}

// One-pass form for steps up to kHaloMax: each workgroup computes the adjoints
// of its tile and of a halo of max(s1, s2) pixels into LDS (the halo's
// recomputed by the neighbouring tiles too) and gathers from there, instead of
// writing twelve planes of adjoints to memory and reading them back.
constexpr int kHaloMax = 4;

template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH) normal_bwd_fused_kernel(const DevCam *__restrict__ cams, int V,
                                                                 uint32_t ntiles, const float *__restrict__ depth,
                                                                 const float *__restrict__ dnormal,
                                                                 const float *__restrict__ ntgt,
                                                                 const float *__restrict__ nscale,
                                                                 const float *__restrict__ ddepth,
                                                                 float *__restrict__ gd, int s1, int s2, float lam,
                                                                 int orient)
{
    constexpr int NE_MAX = (TW + 2 * kHaloMax) * (TH + 2 * kHaloMax);
    __shared__ float sadj[12][NE_MAX];
    const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
    if (tile >= ntiles) return;
    const int view = view_of_tile(cams, V, tile);
    const DevCam &cam = cams[view];
    const uint32_t lt = tile - cam.tile_base;
    const int u0 = (int)(lt % (uint32_t)cam.tiles_x) * TW, v0 = (int)(lt / (uint32_t)cam.tiles_x) * TH;
    const int h = s1 > s2 ? s1 : s2;  // <= kHaloMax (checked by the launcher)
    const int EW = TW + 2 * h, NE = EW * (TH + 2 * h);
    const float *D = depth + cam.pix_off;
    const float *dn = dnormal ? dnormal + 3 * cam.pix_off : nullptr;
    const float *nt = ntgt ? ntgt + 3 * cam.pix_off : nullptr;
    const float nsc = nt && !dn ? *nscale : 0.f;
    for (int e = threadIdx.x; e < NE; e += TW * TH) {
        const int u = u0 - h + e % EW, v = v0 - h + e / EW;
        float out[12];
        if (u >= 0 && u < cam.W && v >= 0 && v < cam.H) {
            normal_adj_at(cam, D, dn, nt, nsc, u, v, s1, s2, lam, orient, out);
        } else {
            for (int k = 0; k < 12; ++k) out[k] = 0.f;
        }
        for (int k = 0; k < 12; ++k) sadj[k][e] = out[k];
    }
    __syncthreads();
    const int u = u0 + (int)(threadIdx.x % TW), v = v0 + (int)(threadIdx.x / TW);
    if (u >= cam.W || v >= cam.H) return;
    const int e0 = (v - v0 + h) * EW + (u - u0 + h);
    float r = normal_gather_at(cam, u, v, s1, s2, [&](int k, int du, int dv) { return sadj[k][e0 + du + dv * EW]; });
    const int64_t q = cam.pix_off + (int64_t)v * cam.W + u;
    if (ddepth) r += ddepth[q];
    gd[q] = r;
}

template <int TW, int TH>
hipError_t nfwd(const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out, const ugs_options &o,
                hipStream_t s)
{
    hipLaunchKernelGGL((normal_fwd_kernel<TW, TH>), dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), 0, s,
                       (const DevCam *)(ws + L.cams), pb.V, (uint32_t)pb.total_tiles, out.depth, out.normal, o.step1, o.step2, o.lambda,
                       o.orient_sign, pb.half_out);
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t nbwd(const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out, const ugs_upstream &up,
                const ugs_options &o, hipStream_t s)
{
    auto cams = (const DevCam *)(ws + L.cams);
    auto adj = (float *)(ws + L.nadj);
    auto gd = (float *)(ws + L.gd);
    if (o.step1 <= kHaloMax && o.step2 <= kHaloMax) {
        hipLaunchKernelGGL((normal_bwd_fused_kernel<TW, TH>), dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), 0, s,
                           cams, pb.V, (uint32_t)pb.total_tiles, out.depth, up.normal, up.normal_target,
                           up.normal_scale, up.depth, gd, o.step1, o.step2, o.lambda, o.orient_sign);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((normal_adj_kernel<TW, TH>), dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), 0, s, cams, pb.V,
                       (uint32_t)pb.total_tiles, out.depth, up.normal, up.normal_target, up.normal_scale, pb.total_pix, adj,
                       o.step1, o.step2, o.lambda, o.orient_sign);
    hipLaunchKernelGGL((normal_gather_kernel<TW, TH>), dim3(xcd_grid(pb.total_tiles)), dim3(TW * TH), 0, s, cams,
                       pb.V, (uint32_t)pb.total_tiles, (const float *)adj, pb.total_pix, up.depth, gd, o.step1, o.step2);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_normal_fwd(const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out,
                             const ugs_options &opt, hipStream_t s)
{
    if (pb.total_tiles == 0) return hipSuccess;
    if (pb.tile_w == 8 && pb.tile_h == 8) return nfwd<8, 8>(pb, L, ws, out, opt, s);
    if (pb.tile_w == 32 && pb.tile_h == 8) return nfwd<32, 8>(pb, L, ws, out, opt, s);
    return nfwd<16, 16>(pb, L, ws, out, opt, s);
}

hipError_t launch_normal_bwd(const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out,
                             const ugs_upstream &up, const ugs_options &opt, hipStream_t s)
{
    if (pb.total_tiles == 0) return hipSuccess;
    if (pb.tile_w == 8 && pb.tile_h == 8) return nbwd<8, 8>(pb, L, ws, out, up, opt, s);
    if (pb.tile_w == 32 && pb.tile_h == 8) return nbwd<32, 8>(pb, L, ws, out, up, opt, s);
    return nbwd<16, 16>(pb, L, ws, out, up, opt, s);
}

}  // namespace ugs
