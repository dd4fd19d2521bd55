// The training loss of section 3.4 on the rendered maps and its gradient, the
// upstream of the rasterizer's backward.  Five launches over all views at once,
// asynchronous and free of atomics (graph-capturable, and the loss values are
// the same from run to run: every block writes its own partial sums, which one
// block adds up in a fixed order):
//   pix_fwd    per-pixel terms, one block per 1024 pixels of a view: |C - C_gt|,
//              N . N_gt, |D - D_gt|, the cross-entropy (one online-softmax
//              pass over the channels; the log-sum-exp is kept for the
//              gradient) and |K - 1|;
//   ssim_fwd   one block per 64x16 tile and colour channel: the five
//              Gaussian-window moments from an LDS tile with a 5-pixel halo
//              (separable, zero outside the image), SSIM and its partials with
//              respect to the mean, E[x^2] and E[xy] of the rendered image;
//   finalize   the loss values, the balancing ratios |L_l1| / |L_x| and the
//              per-term gradient coefficients;
//   grad_pix   the depth, K, normal and logit gradients per pixel;
//   ssim_bwd   the colour gradient: the L1 sign term plus the three partial
//              maps correlated with the same window (a tile with halo again).
#include "ugs_internal.h"

namespace ugs {
namespace {

constexpr int kR = 5;              // window radius (11 x 11)
constexpr int kChunk = 1024;       // pixels per per-pixel work item
constexpr size_t kHeaderBytes = 256;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct ViewTable {
    int V;
    int W[UGS_MAX_VIEWS], H[UGS_MAX_VIEWS];
    int64_t off[UGS_MAX_VIEWS];        // first pixel of the view in the stacked planes
    int chunk0[UGS_MAX_VIEWS + 1];     // prefix of per-view pixel chunks
    int tile0[UGS_MAX_VIEWS + 1];      // prefix of per-view SSIM tiles
};

struct LossHeader {
    float coef[8];  // 0 l1 (per colour value), 1 ssim, 2 normal, 3 depth, 4 seg, 5 K
};

__device__ __forceinline__ int find_view(const int *pre, int V, int item)
{
    int v = 0;
    while (v + 1 < V && pre[v + 1] <= item) ++v;
    return v;
}

__device__ __forceinline__ float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// Block sum of a double in a fixed order (shuffle tree, then waves in order).
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lds[w];
    return t;
}

// NP consecutive pixels per thread: 4 (16-byte loads and stores) when every
// plane starts 16-byte aligned, else 1.
template <int NP>
struct Px {
    float v[NP];
};

template <int NP>
__device__ __forceinline__ Px<NP> ld(const float *p)
{
    Px<NP> r;
    if constexpr (NP == 4) {
        const float4 f = *reinterpret_cast<const float4 *>(p);
        r.v[0] = f.x, r.v[1] = f.y, r.v[2] = f.z, r.v[3] = f.w;
    } else {
        r.v[0] = *p;
    }
    return r;
}

template <int NP>
__device__ __forceinline__ void st(float *p, const Px<NP> &x)
{
    if constexpr (NP == 4)
        *reinterpret_cast<float4 *>(p) = make_float4(x.v[0], x.v[1], x.v[2], x.v[3]);
    else
        *p = x.v[0];
}

template <int NP>
__device__ __forceinline__ void ld_label(const int32_t *p, int (&l)[NP])
{
    if constexpr (NP == 4) {
        const int4 f = *reinterpret_cast<const int4 *>(p);
        l[0] = f.x, l[1] = f.y, l[2] = f.z, l[3] = f.w;
    } else {
        l[0] = *p;
    }
}

// Online softmax over the channels of NP pixels: the log-sum-exp of each, and
// the logit of each pixel's label channel picked on the way (0 when the label
// is out of range), so that no second read of that channel is needed.
template <int NP>
__device__ __forceinline__ Px<NP> logsumexp(const float *o, int64_t HW, int C, const int (&lab)[NP],
                                            float (&picked)[NP])
{
    constexpr int U = NP == 4 ? 4 : 8;  // channels in flight
    float m[NP], s[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) m[i] = -INFINITY, s[i] = 0.f, picked[i] = 0.f;
    int c = 0;
    for (; c + U <= C; c += U) {
        Px<NP> x[U];
#pragma unroll
        for (int j = 0; j < U; ++j) x[j] = ld<NP>(o + (int64_t)(c + j) * HW);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
#pragma unroll
            for (int j = 0; j < U; ++j) picked[i] = c + j == lab[i] ? x[j].v[i] : picked[i];
            float mb = x[0].v[i];
#pragma unroll
            for (int j = 1; j < U; ++j) mb = fmaxf(mb, x[j].v[i]);
            const float mn = fmaxf(m[i], mb);
            float sb = 0.f;
#pragma unroll
            for (int j = 0; j < U; ++j) sb += __expf(x[j].v[i] - mn);
            s[i] = s[i] * __expf(m[i] - mn) + sb;
            m[i] = mn;
        }
    }
    for (; c < C; ++c) {
        const Px<NP> x = ld<NP>(o + (int64_t)c * HW);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            picked[i] = c == lab[i] ? x.v[i] : picked[i];
            const float mn = fmaxf(m[i], x.v[i]);
            s[i] = s[i] * __expf(m[i] - mn) + __expf(x.v[i] - mn);
            m[i] = mn;
        }
    }
    Px<NP> r;
#pragma unroll
    for (int i = 0; i < NP; ++i) r.v[i] = m[i] + __logf(s[i]);
    return r;
}

template <int NP>
__global__ void __launch_bounds__(256) pix_fwd(ViewTable vt, ugs_outputs out, ugs_targets gt, int C_o,
                                               float *__restrict__ lse, double *__restrict__ part)
{
    __shared__ double lds[4];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    {
        const int item = blockIdx.x;  // one chunk per block
        const int v = find_view(vt.chunk0, vt.V, item);
        const int64_t HW = (int64_t)vt.W[v] * vt.H[v], off = vt.off[v];
        const int64_t base = (int64_t)(item - vt.chunk0[v]) * kChunk;
        for (int j = 0; j < kChunk / (256 * NP); ++j) {
            const int64_t p = base + (int64_t)(j * 256 + threadIdx.x) * NP;
            if (p >= HW) break;  // NP divides HW
            for (int c = 0; c < 3; ++c) {
                const int64_t q = 3 * off + c * HW + p;
                const Px<NP> x = ld<NP>(out.rgb + q), y = ld<NP>(gt.rgb + q);
#pragma unroll
                for (int i = 0; i < NP; ++i) a[0] += fabs((double)x.v[i] - (double)y.v[i]);
                if (gt.normal) {
                    const Px<NP> n = ld<NP>(out.normal + q), ng = ld<NP>(gt.normal + q);
#pragma unroll
                    for (int i = 0; i < NP; ++i) a[1] += (double)n.v[i] * (double)ng.v[i];
                }
            }
            if (gt.depth) {
                const Px<NP> d = ld<NP>(out.depth + off + p), dg = ld<NP>(gt.depth + off + p);
#pragma unroll
                for (int i = 0; i < NP; ++i) a[2] += fabs((double)d.v[i] - (double)dg.v[i]);
            }
            if (gt.label) {
                const float *o = out.sem + (int64_t)C_o * off + p;
                int lab[NP];
                ld_label<NP>(gt.label + off + p, lab);
                float picked[NP];
                const Px<NP> l = logsumexp<NP>(o, HW, C_o, lab, picked);
                st<NP>(lse + off + p, l);
#pragma unroll
                for (int i = 0; i < NP; ++i)
                    if (lab[i] >= 0 && lab[i] < C_o) a[3] += (double)(l.v[i] - picked[i]);
            }
            const Px<NP> k = ld<NP>(out.kmap + off + p);
#pragma unroll
            for (int i = 0; i < NP; ++i) a[4] += fabs((double)k.v[i] - 1.0);
        }
    }
    for (int k = 0; k < 5; ++k) {
        const double t = block_sum(a[k], lds);
        if (threadIdx.x == 0) part[(size_t)k * gridDim.x + blockIdx.x] = t;
    }
}

// SSIM tiles: 64 x 16 outputs per work item, read with a 5-pixel halo
// (74 x 26 values, rows padded to 76 floats for 16-byte LDS reads).  The
// horizontal pass gives each of 208 threads eight consecutive outputs of one
// halo row (18 inputs, read as float4); the vertical pass gives each of the 256
// threads four consecutive rows of one column (14 inputs).
constexpr int kSW = 64, kSH = 16;
constexpr int kXW = kSW + 2 * kR, kXH = kSH + 2 * kR, kXS = 76;
constexpr int kHSeg = 8;                  // horizontal outputs per thread
constexpr int kHTasks = kXH * (kSW / kHSeg);  // 208
constexpr int kVRows = 4;                 // vertical outputs per thread
static_assert(kSW * kSH == 256 * kVRows, "one vertical task per thread");
static_assert(kHSeg * (kSW / kHSeg - 1) + 20 <= kXS, "float4 reads stay inside the padded row");

// The normalised 1-D Gaussian window (computed on the host, in double).
struct Window {
    float g[2 * kR + 1];
};

struct TileItem {
    int c, x0, y0, W, H;
    int64_t plane;  // first value of the channel plane in the stacked colour maps
};

__device__ __forceinline__ TileItem tile_item(const ViewTable &vt, int item)
{
    TileItem t;
    const int ti = item / 3;
    t.c = item - 3 * ti;
    const int v = find_view(vt.tile0, vt.V, ti);
    t.W = vt.W[v];
    t.H = vt.H[v];
    const int tx = (t.W + kSW - 1) / kSW, k = ti - vt.tile0[v];
    t.y0 = (k / tx) * kSH;
    t.x0 = (k - (k / tx) * tx) * kSW;
    t.plane = 3 * vt.off[v] + (int64_t)t.c * t.W * t.H;
    return t;
}

// Loads NM channel planes' tile with halo into lds[NM][kXH][kXS] (zero outside
// the image).  All global loads of a thread are issued before the first LDS
// store, so their latencies overlap.
template <int NM>
__device__ __forceinline__ void load_halo(float *lds, const float *const (&src)[NM], const TileItem &t)
{
    constexpr int kIt = (kXH * kXW + 255) / 256;
    float v[kIt][NM];
    int dst[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
        const int q = i * 256 + threadIdx.x;
        const int r = q / kXW, c = q - r * kXW;
        const int y = t.y0 - kR + r, x = t.x0 - kR + c;
        const bool in = q < kXH * kXW && x >= 0 && x < t.W && y >= 0 && y < t.H;
        const int64_t a = t.plane + (int64_t)y * t.W + x;
        dst[i] = q < kXH * kXW ? r * kXS + c : -1;
#pragma unroll
        for (int m = 0; m < NM; ++m) v[i][m] = in ? src[m][a] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kIt; ++i)
        if (dst[i] >= 0)
#pragma unroll
            for (int m = 0; m < NM; ++m) lds[m * kXH * kXS + dst[i]] = v[i][m];
}

__device__ __forceinline__ void read20(const float *row, float (&v)[20])
{
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float4 f = r4[i];
        v[4 * i] = f.x;
        v[4 * i + 1] = f.y;
        v[4 * i + 2] = f.z;
        v[4 * i + 3] = f.w;
    }
}

__device__ __forceinline__ void write8(float *dst, const float (&v)[kHSeg])
{
    float4 *d4 = reinterpret_cast<float4 *>(dst);
    d4[0] = make_float4(v[0], v[1], v[2], v[3]);
    d4[1] = make_float4(v[4], v[5], v[6], v[7]);
}

__global__ void __launch_bounds__(256) ssim_fwd(ViewTable vt, Window win, const float *__restrict__ img,
                                                const float *__restrict__ ref, float *__restrict__ dmu,
                                                float *__restrict__ dxx, float *__restrict__ dxy,
                                                double *__restrict__ part)
{
    __shared__ __align__(16) float xy[2 * kXH * kXS];
    __shared__ __align__(16) float hm[5 * kXH * kSW];
    __shared__ double lds[4];
    const float *g = win.g;
    const int col = threadIdx.x & (kSW - 1), r0 = (threadIdx.x / kSW) * kVRows;
    double s_sum = 0.0;
    for (int item = blockIdx.x; item < 3 * vt.tile0[vt.V]; item += gridDim.x) {  // tile and channel
        const TileItem t = tile_item(vt, item);
        __syncthreads();
        load_halo<2>(xy, {img, ref}, t);
        __syncthreads();
        if (threadIdx.x < kHTasks) {  // horizontal pass
            const int r = threadIdx.x / (kSW / kHSeg), c0 = (threadIdx.x % (kSW / kHSeg)) * kHSeg;
            float a[20], b[20];
            read20(&xy[r * kXS + c0], a);
            read20(&xy[(kXH + r) * kXS + c0], b);
            float m[5][kHSeg];
#pragma unroll
            for (int o = 0; o < kHSeg; ++o) {
#pragma unroll
                for (int j = 0; j < 5; ++j) m[j][o] = 0.f;
#pragma unroll
                for (int k = 0; k < 2 * kR + 1; ++k) {
                    const float x = a[o + k], y = b[o + k], wx = g[k] * x, wy = g[k] * y;
                    m[0][o] += wx;
                    m[1][o] += wy;
                    m[2][o] += wx * x;
                    m[3][o] += wy * y;
                    m[4][o] += wx * y;
                }
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) write8(&hm[(j * kXH + r) * kSW + c0], m[j]);
        }
        __syncthreads();
        float v[5][kVRows + 2 * kR];
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
            for (int i = 0; i < kVRows + 2 * kR; ++i) v[j][i] = hm[(j * kXH + r0 + i) * kSW + col];
        const int x = t.x0 + col;
#pragma unroll
        for (int i = 0; i < kVRows; ++i) {
            const int y = t.y0 + r0 + i;
            if (x >= t.W || y >= t.H) continue;
            float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 2 * kR + 1; ++k)
#pragma unroll
                for (int j = 0; j < 5; ++j) m[j] += g[k] * v[j][i + k];
            const float mx = m[0], my = m[1];
            const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
            const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
            const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
            const float iB = 1.f / (B1 * B2);
            const float S = A1 * A2 * iB;
            const float dA1 = A2 * iB, dA2 = A1 * iB, dB1 = -S * (B2 * iB), dB2 = -S * (B1 * iB);
            const int64_t p = t.plane + (int64_t)y * t.W + x;
            dmu[p] = 2.f * my * (dA1 - dA2) + 2.f * mx * (dB1 - dB2);
            dxx[p] = dB2;
            dxy[p] = 2.f * dA2;
            s_sum += (double)S;
        }
    }
    const double tsum = block_sum(s_sum, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tsum;
}

// Adds the partial sums in a fixed order, then derives losses and coefficients.
__global__ void __launch_bounds__(1024) finalize(const double *__restrict__ part_pix, int n_pix,
                                                 const double *__restrict__ part_ssim, int n_ssim, int64_t P,
                                                 ugs_loss_options opt, int has_n, int has_d, int has_s,
                                                 LossHeader *h, float *losses)
{
    __shared__ double lds[16];
    double sums[6];
    for (int k = 0; k < 6; ++k) {
        const double *src = k < 5 ? part_pix + (size_t)k * n_pix : part_ssim;
        const int n = k < 5 ? n_pix : n_ssim;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        int i = threadIdx.x;
        for (; i + 3 * 1024 < n; i += 4 * 1024)
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += src[i + u * 1024];
        for (; i < n; i += 1024) a[0] += src[i];
        sums[k] = block_sum((a[0] + a[1]) + (a[2] + a[3]), lds);
    }
    if (threadIdx.x != 0) return;
    const double n3 = 3.0 * (double)P, n1 = (double)P;
    const double L_l1 = sums[0] / n3, L_ssim = 1.0 - sums[5] / n3;
    const double L_n = has_n ? 1.0 - sums[1] / n1 : 0.0, L_d = has_d ? sums[2] / n1 : 0.0;
    const double L_s = has_s ? sums[3] / n1 : 0.0, L_k = sums[4] / n1;
    const double L[6] = {L_l1, L_ssim, L_n, L_d, L_s, L_k};
    const int on[6] = {1, 1, has_n, has_d, has_s, 1};
    double w[6], all = 0.0;
    for (int k = 0; k < 6; ++k) {
        w[k] = (k == 0 || !opt.balance) ? 1.0 : (fabs(L[k]) > 0.0 ? fabs(L_l1) / fabs(L[k]) : 0.0);
        if (!on[k]) w[k] = 0.0;
        all += (double)opt.lambda[k] * w[k] * L[k];
    }
    for (int k = 0; k < 6; ++k) losses[k] = (float)L[k];
    losses[6] = (float)all;
    losses[7] = (float)(sums[5] / n3);
    h->coef[0] = (float)(opt.lambda[0] * w[0] / n3);
    h->coef[1] = (float)(-opt.lambda[1] * w[1] / n3);  // d(1 - mean SSIM)
    h->coef[2] = (float)(-opt.lambda[2] * w[2] / n1);  // d(1 - mean N . N_gt)
    h->coef[3] = (float)(opt.lambda[3] * w[3] / n1);
    h->coef[4] = (float)(opt.lambda[4] * w[4] / n1);
    h->coef[5] = (float)(opt.lambda[5] * w[5] / n1);
    for (int k = 0; k < 6; ++k) losses[8 + k] = h->coef[k];
}

template <int NP>
__global__ void __launch_bounds__(256) grad_pix(ViewTable vt, ugs_outputs out, ugs_targets gt, int C_o,
                                                const float *__restrict__ lse, const LossHeader *__restrict__ h,
                                                ugs_upstream grad)
{
    float *gK = const_cast<float *>(grad.kmap), *gD = const_cast<float *>(grad.depth);
    float *gN = const_cast<float *>(grad.normal), *gS = const_cast<float *>(grad.sem);
    const float cn = h->coef[2], cd = h->coef[3], cs = h->coef[4], ck = h->coef[5];
    {
        const int item = blockIdx.x;  // one chunk per block
        const int v = find_view(vt.chunk0, vt.V, item);
        const int64_t HW = (int64_t)vt.W[v] * vt.H[v], off = vt.off[v];
        const int64_t base = (int64_t)(item - vt.chunk0[v]) * kChunk;
        for (int j = 0; j < kChunk / (256 * NP); ++j) {
            const int64_t p = base + (int64_t)(j * 256 + threadIdx.x) * NP;
            if (p >= HW) break;
            Px<NP> r = ld<NP>(out.kmap + off + p);
#pragma unroll
            for (int i = 0; i < NP; ++i) r.v[i] = ck * sgn(r.v[i] - 1.f);
            st<NP>(gK + off + p, r);
            if (gD) {
                if (gt.depth) {
                    const Px<NP> d = ld<NP>(out.depth + off + p), dg = ld<NP>(gt.depth + off + p);
#pragma unroll
                    for (int i = 0; i < NP; ++i) r.v[i] = cd * sgn(d.v[i] - dg.v[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < NP; ++i) r.v[i] = 0.f;
                }
                st<NP>(gD + off + p, r);
            }
            if (gN)
                for (int c = 0; c < 3; ++c) {
                    const int64_t q = 3 * off + c * HW + p;
                    if (gt.normal) {
                        r = ld<NP>(gt.normal + q);
#pragma unroll
                        for (int i = 0; i < NP; ++i) r.v[i] *= cn;
                    } else {
#pragma unroll
                        for (int i = 0; i < NP; ++i) r.v[i] = 0.f;
                    }
                    st<NP>(gN + q, r);
                }
            if (gS && C_o > 0) {
                float *gs = gS + (int64_t)C_o * off + p;
                if (gt.label) {
                    const float *o = out.sem + (int64_t)C_o * off + p;
                    const Px<NP> l = ld<NP>(lse + off + p);
                    int lab[NP];
                    ld_label<NP>(gt.label + off + p, lab);
                    float cl[NP];
#pragma unroll
                    for (int i = 0; i < NP; ++i) cl[i] = (lab[i] >= 0 && lab[i] < C_o) ? cs : 0.f;  // ignored label
                    constexpr int U = NP == 4 ? 4 : 8;
                    int c = 0;
                    for (; c + U <= C_o; c += U) {
                        Px<NP> x[U];
#pragma unroll
                        for (int k = 0; k < U; ++k) x[k] = ld<NP>(o + (int64_t)(c + k) * HW);
#pragma unroll
                        for (int k = 0; k < U; ++k) {
#pragma unroll
                            for (int i = 0; i < NP; ++i)
                                x[k].v[i] = cl[i] * (__expf(x[k].v[i] - l.v[i]) - (c + k == lab[i] ? 1.f : 0.f));
                            st<NP>(gs + (int64_t)(c + k) * HW, x[k]);
                        }
                    }
                    for (; c < C_o; ++c) {
                        Px<NP> x = ld<NP>(o + (int64_t)c * HW);
#pragma unroll
                        for (int i = 0; i < NP; ++i)
                            x.v[i] = cl[i] * (__expf(x.v[i] - l.v[i]) - (c == lab[i] ? 1.f : 0.f));
                        st<NP>(gs + (int64_t)c * HW, x);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < NP; ++i) r.v[i] = 0.f;
                    for (int c = 0; c < C_o; ++c) st<NP>(gs + (int64_t)c * HW, r);
                }
            }
        }
    }
}

// dL/dx(q) = coef_l1 sign(x - y) + coef_ssim (G * dmu + 2 x G * dxx + y G * dxy)(q).
__global__ void __launch_bounds__(256) ssim_bwd(ViewTable vt, Window win, const float *__restrict__ img,
                                                const float *__restrict__ ref, const float *__restrict__ dmu,
                                                const float *__restrict__ dxx, const float *__restrict__ dxy,
                                                const LossHeader *__restrict__ h, float *__restrict__ grad)
{
    __shared__ __align__(16) float ps[3 * kXH * kXS];
    __shared__ __align__(16) float hm[3 * kXH * kSW];
    const float *g = win.g;
    const float c0 = h->coef[0], c1 = h->coef[1];
    const int col = threadIdx.x & (kSW - 1), r0 = (threadIdx.x / kSW) * kVRows;
    for (int item = blockIdx.x; item < 3 * vt.tile0[vt.V]; item += gridDim.x) {  // tile and channel
        const TileItem t = tile_item(vt, item);
        __syncthreads();
        load_halo<3>(ps, {dmu, dxx, dxy}, t);
        __syncthreads();
        if (threadIdx.x < kHTasks) {
            const int r = threadIdx.x / (kSW / kHSeg), cs = (threadIdx.x % (kSW / kHSeg)) * kHSeg;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float a[20], m[kHSeg];
                read20(&ps[(j * kXH + r) * kXS + cs], a);
#pragma unroll
                for (int o = 0; o < kHSeg; ++o) {
                    m[o] = 0.f;
#pragma unroll
                    for (int k = 0; k < 2 * kR + 1; ++k) m[o] += g[k] * a[o + k];
                }
                write8(&hm[(j * kXH + r) * kSW + cs], m);
            }
        }
        __syncthreads();
        float v[3][kVRows + 2 * kR];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < kVRows + 2 * kR; ++i) v[j][i] = hm[(j * kXH + r0 + i) * kSW + col];
        const int x = t.x0 + col;
#pragma unroll
        for (int i = 0; i < kVRows; ++i) {
            const int y = t.y0 + r0 + i;
            if (x >= t.W || y >= t.H) continue;
            float m[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 2 * kR + 1; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j) m[j] += g[k] * v[j][i + k];
            const int64_t p = t.plane + (int64_t)y * t.W + x;
            const float a = img[p], b = ref[p];
            grad[p] = c0 * sgn(a - b) + c1 * (m[0] + 2.f * a * m[1] + b * m[2]);
        }
    }
}

bool al(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int view_table(const ugs_camera *cams, int V, ViewTable *vt, int64_t *P)
{
    if (!cams || V < 1 || V > UGS_MAX_VIEWS) return UGS_ERR_INVALID_ARG;
    int64_t off = 0, ch = 0, tl = 0;
    vt->V = V;
    for (int v = 0; v < V; ++v) {
        const int W = cams[v].W, H = cams[v].H;
        if (W < 1 || H < 1 || W > 16384 || H > 16384) return UGS_ERR_INVALID_ARG;
        const int64_t HW = (int64_t)W * H;
        vt->W[v] = W;
        vt->H[v] = H;
        vt->off[v] = off;
        vt->chunk0[v] = (int)ch;
        vt->tile0[v] = (int)tl;
        off += HW;
        ch += (HW + kChunk - 1) / kChunk;
        tl += (int64_t)((W + kSW - 1) / kSW) * ((H + kSH - 1) / kSH);
    }
    if (3 * tl > INT32_MAX / 2) return UGS_ERR_INVALID_ARG;
    vt->chunk0[V] = (int)ch;
    vt->tile0[V] = (int)tl;
    *P = off;
    return UGS_OK;
}

// Scratch: header, per-block partial sums (5 per pixel chunk, 1 per SSIM
// item, 256-byte rounded), then dmu, dxx, dxy (3 x 3P) and lse (P) floats.
size_t part_bytes(const ViewTable &vt)
{
    return ((size_t)(5 * vt.chunk0[vt.V] + 3 * vt.tile0[vt.V]) * sizeof(double) + 255) & ~(size_t)255;
}

size_t loss_scratch_bytes(const ViewTable &vt, int64_t P) { return kHeaderBytes + part_bytes(vt) + (size_t)40 * P; }

}  // namespace
}  // namespace ugs

using namespace ugs;

extern "C" {

void ugs_default_loss_options(ugs_loss_options *o)
{
    if (!o) return;
    o->lambda[0] = 1.f;
    for (int k = 1; k < 6; ++k) o->lambda[k] = 0.1f;
    o->balance = 1;
}

int ugs_loss_scratch_size(const ugs_camera *cams, int V, size_t *bytes)
{
    ViewTable vt;
    int64_t P;
    if (!bytes || view_table(cams, V, &vt, &P) != UGS_OK) return UGS_ERR_INVALID_ARG;
    *bytes = loss_scratch_bytes(vt, P);
    return UGS_OK;
}

int ugs_loss(const ugs_camera *cams, int V, int C_o, const ugs_outputs *out, const ugs_targets *gt,
             const ugs_loss_options *opt, const ugs_upstream *grad, float *losses, void *scratch,
             size_t scratch_bytes, void *stream)
{
    ViewTable vt;
    int64_t P;
    if (view_table(cams, V, &vt, &P) != UGS_OK) return UGS_ERR_INVALID_ARG;
    const size_t need = loss_scratch_bytes(vt, P);
    if (!out || !gt || !opt || !grad || !losses || !scratch || scratch_bytes < need || !al(scratch, 256))
        return UGS_ERR_INVALID_ARG;
    if (C_o < 0 || C_o > UGS_MAX_CHANNELS || (gt->label && (C_o < 1 || !out->sem))) return UGS_ERR_INVALID_ARG;
    if (!out->rgb || !out->kmap || !gt->rgb || !grad->rgb || !grad->kmap) return UGS_ERR_INVALID_ARG;
    if ((gt->depth && !out->depth) || (gt->normal && !out->normal)) return UGS_ERR_INVALID_ARG;
    const void *ps[] = {out->rgb, out->kmap, out->depth, out->normal, out->sem, gt->rgb, gt->depth, gt->normal,
                        gt->label, grad->rgb, grad->kmap, grad->depth, grad->normal, grad->sem, losses};
    for (auto p : ps)
        if (p && !al(p, 4)) return UGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)scratch;
    LossHeader *h = (LossHeader *)base;
    double *part_pix = (double *)(base + kHeaderBytes);
    const int nb_pix = vt.chunk0[V];
    double *part_ssim = part_pix + (size_t)5 * nb_pix;
    // SSIM blocks: as many as are resident at once (each loops over items)
    int dev = 0, cus = 0, occ_f = 0, occ_b = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, ssim_fwd, 256, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_b, ssim_bwd, 256, 0) != hipSuccess)
        return UGS_ERR_HIP;
    const int items = 3 * vt.tile0[V];
    const int nb_sf = std::max(1, std::min(items, cus * std::max(occ_f, 1)));
    const int nb_sb = std::max(1, std::min(items, cus * std::max(occ_b, 1)));
    Window win;
    {
        double w[2 * kR + 1], sum = 0.0;
        for (int k = 0; k <= 2 * kR; ++k) sum += (w[k] = std::exp(-(double)((k - kR) * (k - kR)) / (2.0 * 1.5 * 1.5)));
        for (int k = 0; k <= 2 * kR; ++k) win.g[k] = (float)(w[k] / sum);
    }
    float *dmu = (float *)(base + kHeaderBytes + part_bytes(vt)), *dxx = dmu + 3 * P, *dxy = dmu + 6 * P;
    float *lse = dmu + 9 * P;
    // four pixels per thread when every plane start is a multiple of 4 values
    // and every map 16-byte aligned
    bool v4 = true;
    for (int v = 0; v < V; ++v) v4 = v4 && ((int64_t)vt.W[v] * vt.H[v]) % 4 == 0;
    for (auto p : ps)
        v4 = v4 && (!p || al(p, 16));
    if (v4)
        hipLaunchKernelGGL(pix_fwd<4>, dim3(nb_pix), dim3(256), 0, s, vt, *out, *gt, C_o, lse, part_pix);
    else
        hipLaunchKernelGGL(pix_fwd<1>, dim3(nb_pix), dim3(256), 0, s, vt, *out, *gt, C_o, lse, part_pix);
    hipLaunchKernelGGL(ssim_fwd, dim3(nb_sf), dim3(256), 0, s, vt, win, out->rgb, gt->rgb, dmu, dxx, dxy,
                       part_ssim);
    hipLaunchKernelGGL(finalize, dim3(1), dim3(1024), 0, s, (const double *)part_pix, nb_pix,
                       (const double *)part_ssim, nb_sf, P, *opt, gt->normal ? 1 : 0, gt->depth ? 1 : 0,
                       gt->label ? 1 : 0, h, losses);
    if (v4)
        hipLaunchKernelGGL(grad_pix<4>, dim3(nb_pix), dim3(256), 0, s, vt, *out, *gt, C_o, (const float *)lse,
                           (const LossHeader *)h, *grad);
    else
        hipLaunchKernelGGL(grad_pix<1>, dim3(nb_pix), dim3(256), 0, s, vt, *out, *gt, C_o, (const float *)lse,
                           (const LossHeader *)h, *grad);
    hipLaunchKernelGGL(ssim_bwd, dim3(nb_sb), dim3(256), 0, s, vt, win, out->rgb, gt->rgb, (const float *)dmu,
                       (const float *)dxx, (const float *)dxy, (const LossHeader *)h, const_cast<float *>(grad->rgb));
    return hipGetLastError() == hipSuccess ? UGS_OK : UGS_ERR_HIP;
}

}  // extern "C"
