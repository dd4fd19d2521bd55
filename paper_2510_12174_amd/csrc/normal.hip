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
// The backward is a gather: a first pass stores, per pixel, the adjoints of its
// four finite-difference vectors (12 floats); a second pass lets every pixel
// collect the terms of the up to eight stencils that read it.  No atomics, so
// the result is deterministic.
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

// Pass 1: adjoints of (vx1, vy1, vx2, vy2) in the camera frame, planar [12][pixels].
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
    const int64_t HW = (int64_t)cam.W * cam.H, p = (int64_t)v * cam.W + u, gp = cam.pix_off + p;
    float out[12];
    for (int k = 0; k < 12; ++k) out[k] = 0.f;
    float gw[3] = {0.f, 0.f, 0.f};
    if (dnormal) {
        const float *dn = dnormal + 3 * cam.pix_off;
        gw[0] = dn[p];
        gw[1] = dn[HW + p];
        gw[2] = dn[2 * HW + p];
    } else if (ntgt) {  // fused cosine seed: scale * N_target
        const float *nt = ntgt + 3 * cam.pix_off, sc = *nscale;
        gw[0] = sc * nt[p];
        gw[1] = sc * nt[HW + p];
        gw[2] = sc * nt[2 * HW + p];
    }
    if (gw[0] != 0.f || gw[1] != 0.f || gw[2] != 0.f) {
        NState S;
        normal_state(depth + cam.pix_off, cam, u, v, s1, s2, lam, orient, S);
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
    for (int k = 0; k < 12; ++k) adj[k * total_pix + gp] = out[k];
}

// Pass 2: gather the stencil adjoints that reference this pixel and project on
// dP/dD = R^T p; adds the direct depth gradient and writes G_D.
template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH) normal_gather_kernel(const DevCam *__restrict__ cams, int V, uint32_t ntiles,
                                                              const float *__restrict__ adj, int64_t total_pix,
                                                              const float *__restrict__ ddepth, float *__restrict__ gd,
                                                              int s1, int s2)
{
    int view, u, v;
    if (!pixel_of<TW, TH>(cams, V, ntiles, view, u, v)) return;
    const DevCam &cam = cams[view];
    const int W = cam.W, H = cam.H;
    const int64_t base = cam.pix_off;
    const int64_t p = (int64_t)v * W + u;
    float gP[3] = {0.f, 0.f, 0.f};
    const int gs[2] = {s1, s2};
    for (int k = 0; k < 2; ++k) {
        const int g = gs[k];
        // this pixel is (u+g, v) of the stencil at (u-g, v): + d/d vx
        if (u - g >= 0) {
            const int64_t q = base + p - g;
            for (int c = 0; c < 3; ++c) gP[c] += adj[(6 * k + c) * total_pix + q];
        }
        if (u + g < W) {
            const int64_t q = base + p + g;
            for (int c = 0; c < 3; ++c) gP[c] -= adj[(6 * k + c) * total_pix + q];
        }
        if (v - g >= 0) {
            const int64_t q = base + p - (int64_t)g * W;
            for (int c = 0; c < 3; ++c) gP[c] += adj[(6 * k + 3 + c) * total_pix + q];
        }
        if (v + g < H) {
            const int64_t q = base + p + (int64_t)g * W;
            for (int c = 0; c < 3; ++c) gP[c] -= adj[(6 * k + 3 + c) * total_pix + q];
        }
    }
    const float pp[3] = {((float)u - cam.cx) / cam.fx, ((float)v - cam.cy) / cam.fy, 1.f};
    float r = dot3(gP, pp);
    if (ddepth) r += ddepth[base + p];
    gd[base + p] = r;
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
