// Internal definitions shared by the gfx950 kernels and the C-ABI host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "unigs.h"

namespace ugs {

// Splatting constants of the 3DGS pipeline UniGS extends (section 3.4): alpha
// cut-off, alpha clamp, transmittance termination, EWA low-pass, FOV clamp.
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr double kTStop = 1e-4;
constexpr float kLowPass = 0.3f;
constexpr float kFovClamp = 1.3f;

// Per-view constants on the device.
struct DevCam {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float C[3];         // camera centre -R^T t
    float limx, limy;   // 1.3 * tan(half FOV)
    float z_near;
    int W, H;
    int tiles_x, tiles_y;
    uint32_t tile_base; // first global tile of this view
    int64_t pix_off;    // first pixel of this view in the stacked image planes
};

// Per-(view, Gaussian) render record, 4 x float4 = 64 B:
//   r0 = (mean2d.x, mean2d.y, l11, l21)
//   r1 = (l22, opacity, k, z0)
//   r2 = (beta.x, beta.y, gam.a, gam.b)
//   r3 = (gam.c, rgb.r, rgb.g, rgb.b)
// (l11, l21, l22) is the lower Cholesky factor of the conic (inverse 2D
// covariance): with (dx, dy) the pixel minus mean2d,
//   power = -0.5 ((l11 dx + l21 dy)^2 + (l22 dy)^2),
// a sum of squares that stays accurate in FP32 for thin splats.  Depth of the
// ray-ellipsoid midpoint at that pixel:
//   d = z0 (1 + B) / (1 + 2B + Cq),  B = beta . (dx, dy),
//   Cq = gam.a dx^2 + 2 gam.b dx dy + gam.c dy^2.
// The per-view gradient record has the same 16 slots:
//   g0 = (d mean2d.x, d mean2d.y, d l11, d l21)
//   g1 = (d l22, d opacity, d k, d z0)
//   g2 = (d beta.x, d beta.y, d gam.a, d gam.b)
//   g3 = (d gam.c, d rgb.r, d rgb.g, d rgb.b)
constexpr int kRecFloats = 16;

// Activity mask written by the forward for the backward (9..256 channels): one
// bit plane per wavefront slot of a tile (4 planes), bit e of a plane set when
// list entry e (a sorted pair) has at least one contributing pixel among that
// wavefront's 64 pixels.  The backward walks only those entries.
constexpr int kMaskPlanes = 4;

struct DevCounters {
    uint32_t P;          // pairs required
    uint32_t overflow;   // non-zero when P exceeded the capacity
    uint32_t R;          // visible (view, Gaussian) records
    uint32_t P_eff;      // pairs emitted and sorted (0 on overflow)
    unsigned long long n_eval, n_contrib;
    uint32_t R_gauss, pad;  // records still touched after the binning walk (<= R), listed per Gaussian
};

struct WsLayout {
    size_t cams, rec, hrec, rect, touched, voff, poff, tsorted, dkey0, dkey1, didx0, didx1, vlist, scan_part, keys0, keys1,
        vals0, vals1, hist, digit_tot, ranges, grec, gd, nadj, amask, tclk, counters, total;
    int64_t N, VN, total_tiles, total_pix, pair_cap;
    int64_t amask_words;  // 32-bit words per plane of the activity mask
    int V, nb_scan, depth_bits, tile_bits;
};

constexpr int kScanBlock = 1024;  // elements per scan block (256 threads x 4)
constexpr int kSortBlocks = 4096; // fixed radix-sort grid (one wavefront per block)
constexpr int kSortThreads = 64;

struct Problem {
    int64_t N;
    int sh_deg, C_o, V;
    int tile_w, tile_h;
    int64_t total_tiles, total_pix;
    float prune_Tk;
    int depth_mode;  // 0: ray-ellipsoid midpoint, 1: Gaussian centre, 2: midpoint on a hit, else centre
    int half_out;    // rgb, kmap, normal and sem outputs in binary16
    int sem_bf16x3;  // 9..32 channels: semantic products on split-bf16 matrix cores
};

// Stores an output value as FP32 or, for half outputs, binary16 (nearest even).
__device__ __forceinline__ void put_out(float *p, int64_t i, float v, int half)
{
    if (half)
        reinterpret_cast<_Float16 *>(p)[i] = (_Float16)v;
    else
        p[i] = v;
}

// ---- launchers (each enqueues on `s`; return the launch error) ----
hipError_t launch_project_fwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                              bool zero_grad, hipStream_t s);
hipError_t launch_project_bwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                              const ugs_gaussian_grads &dg, hipStream_t s);
hipError_t launch_binsort(const Problem &pb, const WsLayout &L, char *ws, hipStream_t s, int *final_buf);
// The records still touched after the binning (a kept tile) in (Gaussian,
// view) order into L.vlist, their count into DevCounters::R_gauss (after the
// binning; uses L.tsorted and L.poff, free by then, as scratch).
hipError_t launch_gauss_major_list(const WsLayout &L, char *ws, int V, hipStream_t s);
hipError_t launch_render_fwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                             const ugs_outputs &out, int batch, bool counters, int final_buf, hipStream_t s);
hipError_t launch_render_bwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                             const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg,
                             int batch, int final_buf, bool counters, hipStream_t s);
// 9..256 channels, semantic contractions on the FP32 matrix cores
// With `counters` set, the first (main) pass of each also writes each tile
// workgroup's start and end time (s_memrealtime, 100 MHz) to L.tclk.
hipError_t launch_render_fwd_mm(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                                const ugs_outputs &out, int batch, bool counters, int final_buf, hipStream_t s);
hipError_t launch_render_bwd_mm(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                                const ugs_outputs &out, const ugs_upstream &up, const ugs_gaussian_grads &dg,
                                int batch, int final_buf, bool counters, hipStream_t s);
hipError_t launch_normal_fwd(const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out,
                             const ugs_options &opt, hipStream_t s);
hipError_t launch_normal_bwd(const Problem &pb, const WsLayout &L, char *ws, const ugs_outputs &out,
                             const ugs_upstream &up, const ugs_options &opt, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Exclusive scan of (flags[i] > 0) over n elements into out, total to *total;
// part holds ceil(n / kScanBlock) partials.
hipError_t launch_scan_flags(const uint32_t *flags, int64_t n, uint32_t *part, uint32_t *out, uint32_t *total,
                             hipStream_t s);
// Passes of the LSD radix sorts over `bits` key bits: digits of at most 9 bits,
// the bits split evenly.
inline int radix_passes(int bits) { return (bits + 8) / 9; }
// Which record-index buffer (0: didx0, 1: didx1) holds the depth-sorted visible
// records after launch_binsort (the depth sort flips buffers once per pass).
// L.vlist holds the records that kept a tile, in (Gaussian, view) order, once
// launch_gauss_major_list has run.
inline int depth_sort_buffer(const WsLayout &L) { return radix_passes(L.depth_bits) & 1; }
int channel_pad(int C_o);

// index of the view owning a global tile (V small: linear scan over tile_base)
__device__ __forceinline__ int view_of_tile(const DevCam *cams, int V, uint32_t tile)
{
    int v = 0;
    for (int k = 1; k < V; ++k)
        if (tile >= cams[k].tile_base) v = k;
    return v;
}

// Workgroups are dealt to the 8 XCDs round-robin by workgroup id.  Tile kernels
// map workgroup b so that each XCD (with its own L2) works through runs of
// kXcdChunk consecutive tiles (a few tile rows, which share most of their
// Gaussians), while the runs themselves alternate between XCDs so that every
// XCD gets a similar share of every view:
//   xcd = b % 8, k = b / 8, tile = ((k / C) * 8 + xcd) * C + k % C.
// The grid is rounded up to a whole number of 8 * C blocks; ids at or beyond T
// return at once.
constexpr int kXcds = 8;
constexpr uint32_t kXcdChunk = 32;
inline unsigned xcd_grid(int64_t tiles)
{
    const int64_t g = (int64_t)kXcds * kXcdChunk;
    return (unsigned)(g * ((tiles + g - 1) / g));
}
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t tiles)
{
    const uint32_t xcd = b % kXcds, k = b / kXcds;
    return ((k / kXcdChunk) * kXcds + xcd) * kXcdChunk + k % kXcdChunk;
}

// Tile culling by the alpha >= 1/255 ellipse.  A (view, Gaussian) record
// covers tile [x0, x1] x [y0, y1] (pixel centres, clipped to the image) when
// the minimum over the box of q(d) = (l11 dx + l21 dy)^2 + (l22 dy)^2 (d the
// offset from mean2d; power = -q/2) is at most 2 ln(255 o), inflated by 1e-3
// relative and absolute so that no pixel whose FP32 alpha reaches 1/255 is
// ever culled.  Evaluated from the FP32 record with non-contracting IEEE
// operations only, by one routine shared by the counting and the emission
// pass, so the two take bit-identical decisions.  Rectangles of more than
// kCullMaxTiles tiles are not tested (every tile kept).
constexpr int kCullMaxTiles = 1024;

struct CullGeom {
    float mx, my, l11, l21, l22;
    float thr;  // inflated 2 ln(255 o)
    float kb;   // l11 l21 / (l21^2 + l22^2): stationary dy = -kb dx on a vertical edge
    float kl;   // l21 / l11: stationary dx = -kl dy on a horizontal edge
};

__device__ __forceinline__ CullGeom cull_geom(float4 r0, float4 r1)
{
    CullGeom c;
    c.mx = r0.x;
    c.my = r0.y;
    c.l11 = r0.z;
    c.l21 = r0.w;
    c.l22 = r1.x;
    const float thr = __fmul_rn(2.0f, logf(__fmul_rn(255.0f, r1.y)));
    c.thr = __fadd_rn(__fmul_rn(thr, 1.001f), 1e-3f);
    c.kb = __fdiv_rn(__fmul_rn(c.l11, c.l21), __fadd_rn(__fmul_rn(c.l21, c.l21), __fmul_rn(c.l22, c.l22)));
    c.kl = __fdiv_rn(c.l21, c.l11);
    return c;
}

__device__ __forceinline__ float cull_q(const CullGeom &c, float dx, float dy)
{
    // (l11 dx + l21 dy)^2 + (l22 dy)^2, the factored form the renderer uses (an
    // expanded quadratic would cancel badly for thin splats)
    const float t1 = __fadd_rn(__fmul_rn(c.l11, dx), __fmul_rn(c.l21, dy));
    const float t2 = __fmul_rn(c.l22, dy);
    return __fadd_rn(__fmul_rn(t1, t1), __fmul_rn(t2, t2));
}

__device__ __forceinline__ bool cull_hits(const CullGeom &c, int x0, int x1, int y0, int y1)
{
    const float fx0 = (float)x0, fx1 = (float)x1, fy0 = (float)y0, fy1 = (float)y1;
    if (c.mx >= fx0 && c.mx <= fx1 && c.my >= fy0 && c.my <= fy1) return true;
    const float ex0 = __fsub_rn(fx0, c.mx), ex1 = __fsub_rn(fx1, c.mx);
    const float ey0 = __fsub_rn(fy0, c.my), ey1 = __fsub_rn(fy1, c.my);
    float qmin = INFINITY;
    for (int k = 0; k < 2; ++k) {
        const float dx = k ? ex1 : ex0;
        const float dy = fminf(fmaxf(-__fmul_rn(c.kb, dx), ey0), ey1);
        qmin = fminf(qmin, cull_q(c, dx, dy));
    }
    for (int k = 0; k < 2; ++k) {
        const float dy = k ? ey1 : ey0;
        const float dx = fminf(fmaxf(-__fmul_rn(c.kl, dy), ex0), ex1);
        qmin = fminf(qmin, cull_q(c, dx, dy));
    }
    return qmin <= c.thr;
}

// Pixel box of tile (tx, ty), clipped to a W x H image.
__device__ __forceinline__ void tile_box(int tx, int ty, int tw, int th, int W, int H, int &x0, int &x1, int &y0,
                                         int &y1)
{
    x0 = tx * tw;
    y0 = ty * th;
    x1 = min(x0 + tw, W) - 1;
    y1 = min(y0 + th, H) - 1;
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }

}  // namespace ugs
