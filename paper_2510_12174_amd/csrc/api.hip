// C ABI of the gfx950 multimodal Gaussian rasterizer: argument checking,
// workspace layout, stage sequencing, HIP-graph capture of the batched step and
// the tile/batch autotuner.  See include/unigs.h for the contract.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ugs_internal.h"

using namespace ugs;

struct ugs_ctx {
    ugs_options opt;
    Problem pb;
    WsLayout L;
    bool have_problem = false;
    bool sorted = false;
    // set once the gradient records of the current projection have been
    // consumed by a backward (eager, replayed or autotuned); cleared by the
    // next projection
    bool bwd_done = false;
    // set by a forward that kept the backward's per-pixel state (T_final,
    // n_contrib) and, with it, the activity mask the backward walks
    bool fwd_state = false;
    int final_buf = 0;
    bool counters = false;
    char *ws = nullptr;
    // captured step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
    uint32_t *host_flag = nullptr;  // mapped pinned memory written by the graph
    uint32_t *host_flag_dev = nullptr;
    char err[256] = {0};
    int timed_stage = 0;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

namespace {

constexpr size_t kAlign = 256;

// Records an event on an eager stream.  While a step is being captured the
// stage is bracketed by event-record nodes of the graph instead (see
// ugs_step_capture), so nothing is recorded here.
void record_event(hipEvent_t e, hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    hipStreamIsCapturing(s, &st);
    if (st == hipStreamCaptureStatusNone) hipEventRecord(e, s);
}

// Brackets the launches of one stage with the context's timing events.
struct StageTimer {
    ugs_ctx *c;
    int st;
    hipStream_t s;
    StageTimer(ugs_ctx *c_, int st_, hipStream_t s_) : c(c_), st(st_), s(s_)
    {
        if (c->timed_stage == st) record_event(c->ev_start, s);
    }
    ~StageTimer()
    {
        if (c->timed_stage == st) record_event(c->ev_stop, s);
    }
};

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int hip_fail(ugs_ctx *ctx, hipError_t e, const char *what)
{
    if (ctx) snprintf(ctx->err, sizeof(ctx->err), "%s: %s", what, hipGetErrorString(e));
    return UGS_ERR_HIP;
}

#define HIPCHK(ctx, call)                                          \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
    } while (0)

bool valid_tile(int w, int h) { return (w == 16 && h == 16) || (w == 8 && h == 8) || (w == 32 && h == 8); }

int check_options(const ugs_options *o)
{
    if (!o) return UGS_ERR_INVALID_ARG;
    if (!valid_tile(o->tile_w, o->tile_h)) return UGS_ERR_UNSUPPORTED;
    if (o->batch < 0 || o->batch > 1024) return UGS_ERR_INVALID_ARG;
    if (o->step1 < 1 || o->step2 < 1 || o->step1 > 64 || o->step2 > 64) return UGS_ERR_INVALID_ARG;
    if (!(o->lambda >= 0.f && o->lambda <= 1.f)) return UGS_ERR_INVALID_ARG;
    if (o->orient_sign != 1 && o->orient_sign != -1) return UGS_ERR_INVALID_ARG;
    if (!(o->prune_Tk >= 0.f)) return UGS_ERR_INVALID_ARG;
    if (o->depth_mode < 0 || o->depth_mode > 2) return UGS_ERR_INVALID_ARG;
    if (o->half_outputs != 0 && o->half_outputs != 1) return UGS_ERR_INVALID_ARG;
    if (o->sem_bf16x3 != 0 && o->sem_bf16x3 != 1) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

int check_cams(const ugs_camera *cams, int V)
{
    if (V < 1 || V > UGS_MAX_VIEWS || !cams) return UGS_ERR_INVALID_ARG;
    for (int v = 0; v < V; ++v) {
        const ugs_camera &c = cams[v];
        if (c.W < 1 || c.H < 1 || c.W > 16384 || c.H > 16384) return UGS_ERR_INVALID_ARG;
        if (!(c.fx > 0.f) || !(c.fy > 0.f) || !isfinite(c.cx) || !isfinite(c.cy)) return UGS_ERR_INVALID_ARG;
        if (!(c.z_near > 0.f)) return UGS_ERR_INVALID_ARG;
        for (int k = 0; k < 9; ++k)
            if (!isfinite(c.R[k])) return UGS_ERR_INVALID_ARG;
        for (int k = 0; k < 3; ++k)
            if (!isfinite(c.t[k])) return UGS_ERR_INVALID_ARG;
    }
    return UGS_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_gaussians(const ugs_gaussians *g)
{
    if (!g || g->N < 0 || g->N > (int64_t)0x7fffffff) return UGS_ERR_INVALID_ARG;
    if (g->sh_deg < 0 || g->sh_deg > 3) return UGS_ERR_UNSUPPORTED;
    if (g->C_o < 0 || g->C_o > UGS_MAX_CHANNELS) return UGS_ERR_UNSUPPORTED;
    if (g->N == 0) return UGS_OK;
    const float *ps[] = {g->mean, g->quat, g->log_scale, g->opacity_logit, g->mask_logit, g->sh};
    for (auto p : ps)
        if (!p || !aligned(p, 4)) return UGS_ERR_INVALID_ARG;
    if (g->C_o > 0 && (!g->sem || !aligned(g->sem, 4))) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

int check_grads(const ugs_gaussian_grads *d, int C_o)
{
    if (!d) return UGS_ERR_INVALID_ARG;
    float *ps[] = {d->mean, d->quat, d->log_scale, d->opacity_logit, d->mask_logit, d->sh};
    for (auto p : ps)
        if (!p || !aligned(p, 4)) return UGS_ERR_INVALID_ARG;
    if (C_o > 0 && (!d->sem || !aligned(d->sem, 4))) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

// The forward needs the image planes; T_final and n_contrib are optional for
// it (forward-only use) and required by the backward.  Binary16 maps need
// 2-byte alignment, FP32 ones 4.
int check_outputs(const ugs_outputs *o, int C_o, bool need_state, bool half)
{
    if (!o) return UGS_ERR_INVALID_ARG;
    const size_t a = half ? 2 : 4;
    const void *ps[] = {o->rgb, o->kmap, o->normal};
    for (auto p : ps)
        if (!p || !aligned(p, a)) return UGS_ERR_INVALID_ARG;
    if (!o->depth || !aligned(o->depth, 4)) return UGS_ERR_INVALID_ARG;
    const void *st[] = {o->T_final, o->n_contrib};
    for (auto p : st) {
        if (need_state && !p) return UGS_ERR_INVALID_ARG;
        if (p && !aligned(p, 4)) return UGS_ERR_INVALID_ARG;
    }
    if (C_o > 0 && (!o->sem || !aligned(o->sem, a))) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

int bit_length(uint64_t x)
{
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

void make_problem(const ugs_options &o, int64_t N, int C_o, int sh_deg, const ugs_camera *cams, int V, Problem &pb,
                  std::vector<DevCam> *dcs)
{
    pb.N = N;
    pb.C_o = C_o;
    pb.sh_deg = sh_deg;
    pb.V = V;
    pb.tile_w = o.tile_w;
    pb.tile_h = o.tile_h;
    pb.prune_Tk = o.prune_Tk;
    pb.depth_mode = o.depth_mode;
    pb.half_out = o.half_outputs;
    pb.sem_bf16x3 = o.sem_bf16x3;
    int64_t tiles = 0, pix = 0;
    for (int v = 0; v < V; ++v) {
        const ugs_camera &c = cams[v];
        int tx = (c.W + o.tile_w - 1) / o.tile_w, ty = (c.H + o.tile_h - 1) / o.tile_h;
        if (dcs) {
            DevCam d;
            memset(&d, 0, sizeof(d));
            memcpy(d.R, c.R, sizeof(d.R));
            memcpy(d.t, c.t, sizeof(d.t));
            d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
            for (int i = 0; i < 3; ++i)
                d.C[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
            d.limx = kFovClamp * (float)c.W / (2.f * c.fx);
            d.limy = kFovClamp * (float)c.H / (2.f * c.fy);
            d.z_near = c.z_near;
            d.W = c.W; d.H = c.H;
            d.tiles_x = tx; d.tiles_y = ty;
            d.tile_base = (uint32_t)tiles;
            d.pix_off = pix;
            dcs->push_back(d);
        }
        tiles += (int64_t)tx * ty;
        pix += (int64_t)c.W * c.H;
    }
    pb.total_tiles = tiles;
    pb.total_pix = pix;
}

WsLayout make_layout(const Problem &pb, int64_t pair_cap)
{
    WsLayout L;
    memset(&L, 0, sizeof(L));
    L.N = pb.N;
    L.V = pb.V;
    L.VN = pb.N * pb.V;
    L.total_tiles = pb.total_tiles;
    L.total_pix = pb.total_pix;
    L.pair_cap = pair_cap;
    L.nb_scan = (int)((L.VN + kScanBlock - 1) / kScanBlock);
    if (L.nb_scan < 1) L.nb_scan = 1;
    L.depth_bits = 32;
    L.tile_bits = bit_length((uint64_t)(pb.total_tiles > 0 ? pb.total_tiles - 1 : 0));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    const size_t VN = (size_t)L.VN, P = (size_t)pair_cap, pix = (size_t)pb.total_pix;
    L.counters = take(sizeof(DevCounters) + 64);
    L.cams = take(sizeof(DevCam) * pb.V);
    L.rec = take(VN * 64);
    L.hrec = take(VN * 4);
    L.grec = take(VN * 64);
    L.rect = take(VN * 8);
    L.touched = take(VN * 4);
    L.voff = take(VN * 4);
    L.poff = take(VN * 4);
    L.tsorted = take(VN * 4);
    L.dkey0 = take(VN * 4);
    L.dkey1 = take(VN * 4);
    L.didx0 = take(VN * 4);
    L.vlist = take(VN * 4);
    L.didx1 = take(VN * 4);
    L.scan_part = take((size_t)L.nb_scan * 4);
    L.keys0 = take(P * 4);
    L.keys1 = take(P * 4);
    L.vals0 = take(P * 4);
    L.vals1 = take(P * 4);
    L.hist = take((size_t)512 * kSortBlocks * 4);  // one row per digit of a 9-bit sort pass
    L.digit_tot = take(512 * 4);
    L.ranges = take((size_t)pb.total_tiles * 8);
    L.gd = take(pix * 4);
    L.nadj = take(pix * 12 * 4);
    L.amask_words = (int64_t)(P / 32 + 4);
    L.amask = take((size_t)kMaskPlanes * L.amask_words * 4);
    L.tclk = take((size_t)pb.total_tiles * 4 * 8);  // forward, backward: start and end per tile
    L.total = o;
    return L;
}

int auto_batch(const ugs_options &o, int C_o)
{
    if (o.batch > 0) return o.batch;
    const int nt = o.tile_w * o.tile_h, cp = channel_pad(C_o);
    // FP32 matrix-core kernels (9..256 channels): 64 entries per batch (32 for
    // single-wavefront tiles); the kernels shrink it to what their LDS holds
    if (C_o > 8 && !(o.sem_bf16x3 && cp <= 32)) return nt >= 256 ? 64 : 32;
    // otherwise the largest power of two up to the tile's pixel count whose LDS
    // staging fits 32 KB per workgroup; the split-bf16 kernels (16 or 32 padded
    // channels) also hold a 16 x 68 FP32 buffer per wavefront and 216 B per entry
    const bool mfma = cp == 16 || cp == 32;
    const size_t per = mfma ? 216 : (size_t)(68 + 4 * cp);
    const size_t fixed = mfma ? (size_t)(nt / 64) * 16 * 68 * 4 : 0;
    int b = nt;
    while (b > 16 && fixed + (size_t)b * per > 32 * 1024) b /= 2;
    return b;
}

// Writes up to 16 cameras per launch through kernel arguments (graph-safe, no
// host staging buffer).
struct CamBatch {
    int first, count;
    DevCam c[16];
};

__global__ void write_cams(CamBatch b, DevCam *dst)
{
    int i = threadIdx.x;
    if (i < b.count) dst[b.first + i] = b.c[i];
}

__global__ void report_flag(const DevCounters *cnt, uint32_t *flag)
{
    if (threadIdx.x == 0) flag[0] = cnt->overflow ? (cnt->P ? cnt->P : 1u) : 0u;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// Order-independent fingerprint of a float array: XOR of mix(index, bits).
__global__ void hash_floats(const float *p, int64_t n, unsigned long long salt, unsigned long long *out)
{
    unsigned long long h = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        h ^= mix64(((unsigned long long)i << 32) ^ (unsigned long long)__float_as_uint(p[i]) ^ salt);
    for (int o = 32; o > 0; o >>= 1) h ^= __shfl_xor(h, o, 64);
    if (__lane_id() == 0 && h) atomicXor(out, h);
}

__global__ void zero_u64(unsigned long long *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Sum and absolute sum (FP64) of n floats: a rounding-tolerant fingerprint.
__global__ void sum_floats(const float *p, int64_t n, double *out)
{
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        a += (double)p[i];
        b += fabs((double)p[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (__lane_id() == 0) {
        atomicAdd(&out[0], a);
        atomicAdd(&out[1], b);
    }
}

int upload_cams(ugs_ctx *ctx, const std::vector<DevCam> &dcs, hipStream_t s)
{
    for (size_t f = 0; f < dcs.size(); f += 16) {
        CamBatch b;
        memset(&b, 0, sizeof(b));
        b.first = (int)f;
        b.count = (int)std::min<size_t>(16, dcs.size() - f);
        for (int i = 0; i < b.count; ++i) b.c[i] = dcs[f + i];
        hipLaunchKernelGGL(write_cams, dim3(1), dim3(16), 0, s, b, (DevCam *)(ctx->ws + ctx->L.cams));
    }
    HIPCHK(ctx, hipGetLastError());
    return UGS_OK;
}

int do_project(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws, size_t ws_bytes,
               hipStream_t s, bool zero_grec = true)
{
    int rc;
    if ((rc = check_gaussians(g)) || (rc = check_cams(cams, V))) return rc;
    if (!ws || !aligned(ws, 256)) return UGS_ERR_INVALID_ARG;
    std::vector<DevCam> dcs;
    Problem pb;
    make_problem(ctx->opt, g->N, g->C_o, g->sh_deg, cams, V, pb, &dcs);
    if (pb.total_tiles >= ((int64_t)1 << 31)) return UGS_ERR_UNSUPPORTED;
    // pair capacity: what fits in the rest of the workspace
    WsLayout L0 = make_layout(pb, 0);
    if (ws_bytes < L0.total) return UGS_ERR_INVALID_ARG;
    // 16 B of keys and values per pair plus its activity-mask bits
    int64_t cap = (int64_t)((ws_bytes - L0.total) * 8 / (128 + kMaskPlanes));
    while (cap > 0 && make_layout(pb, cap).total > ws_bytes) cap -= 64;
    if (cap < 0) cap = 0;
    if (cap > 0x7fffffffll) cap = 0x7fffffffll;
    ctx->pb = pb;
    ctx->L = make_layout(pb, cap);
    ctx->ws = (char *)ws;
    ctx->have_problem = true;
    ctx->sorted = false;
    ctx->bwd_done = false;
    ctx->fwd_state = false;
    if ((rc = upload_cams(ctx, dcs, s))) return rc;
    StageTimer tm(ctx, 1, s);
    HIPCHK(ctx, launch_project_fwd(*g, ctx->pb, ctx->L, ctx->ws, zero_grec, s));
    return UGS_OK;
}

int read_counters(ugs_ctx *ctx, void *ws, hipStream_t s, DevCounters *c)
{
    HIPCHK(ctx, hipMemcpyAsync(c, (char *)ws + ctx->L.counters, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return UGS_OK;
}

int do_bin_sort(ugs_ctx *ctx, void *ws, hipStream_t s, int64_t *P_out)
{
    if (!ctx->have_problem || ws != ctx->ws) return UGS_ERR_STATE;
    int fb = 0;
    {
        StageTimer tm(ctx, 2, s);
        HIPCHK(ctx, launch_binsort(ctx->pb, ctx->L, ctx->ws, s, &fb));
    }
    ctx->final_buf = fb;
    ctx->sorted = true;
    if (P_out) {
        DevCounters c;
        int rc = read_counters(ctx, ws, s, &c);
        if (rc) return rc;
        *P_out = (int64_t)c.P;
        if (c.overflow) return UGS_ERR_CAPACITY;
    }
    return UGS_OK;
}

int check_fwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out)
{
    int rc;
    if (!ctx->sorted || ws != ctx->ws) return UGS_ERR_STATE;
    if ((rc = check_gaussians(g)) || (rc = check_outputs(out, g->C_o, false, ctx->opt.half_outputs))) return rc;
    if (g->N != ctx->pb.N || g->C_o != ctx->pb.C_o || g->sh_deg != ctx->pb.sh_deg) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

int check_bwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out, const ugs_upstream *up,
              const ugs_gaussian_grads *dg)
{
    int rc;
    if ((rc = check_fwd(ctx, g, ws, out))) return rc;
    // the projection zeroes the per-view gradient records and one backward
    // accumulates into them: a second backward needs a new projection
    if (ctx->bwd_done || !ctx->fwd_state) return UGS_ERR_STATE;
    if (ctx->opt.half_outputs) return UGS_ERR_INVALID_ARG;  // half outputs are for forward-only use
    if ((rc = check_outputs(out, g->C_o, true, false))) return rc;
    if ((rc = check_grads(dg, g->C_o))) return rc;
    if (!up || (!up->normal && up->normal_target && !up->normal_scale)) return UGS_ERR_INVALID_ARG;
    if (!up->sem && up->sem_label && (!up->sem_scale || g->C_o < 1 || !out->sem)) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

// Stages of one step: 0 zero gradients, 1 project, 2 bin+sort, 3 compositing
// forward, 4 normals, 5 normal backward, 6 compositing backward, 7 projection
// backward, 8 overflow report (captured steps only).
struct StepArgs {
    const ugs_gaussians *g;
    const ugs_camera *cams;
    int V;
    void *ws;
    size_t ws_bytes;
    const ugs_outputs *out;
    const ugs_upstream *up;
    const ugs_gaussian_grads *dg;
};

int zero_grads(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_gaussian_grads *dg, hipStream_t s);

int step_stage(ugs_ctx *ctx, const StepArgs &a, int st, hipStream_t s)
{
    int rc;
    // a step without gradients (forward only) has no backward stages
    if (!a.dg && (st == 0 || (st >= 5 && st <= 7))) return UGS_OK;
    switch (st) {
    case 0: return zero_grads(ctx, a.g, a.dg, s);
    case 1: return do_project(ctx, a.g, a.cams, a.V, a.ws, a.ws_bytes, s, a.dg != nullptr);
    case 2: return do_bin_sort(ctx, a.ws, s, nullptr);
    case 3: {
        if ((rc = check_fwd(ctx, a.g, a.ws, a.out))) return rc;
        StageTimer tm(ctx, 3, s);
        HIPCHK(ctx, launch_render_fwd(*a.g, ctx->pb, ctx->L, ctx->ws, *a.out, auto_batch(ctx->opt, a.g->C_o),
                                      ctx->counters, ctx->final_buf, s));
        ctx->fwd_state = a.out->T_final && a.out->n_contrib;
        return UGS_OK;
    }
    case 4: {
        if ((rc = check_fwd(ctx, a.g, a.ws, a.out))) return rc;
        StageTimer tm(ctx, 4, s);
        HIPCHK(ctx, launch_normal_fwd(ctx->pb, ctx->L, ctx->ws, *a.out, ctx->opt, s));
        return UGS_OK;
    }
    case 5: {
        if ((rc = check_bwd(ctx, a.g, a.ws, a.out, a.up, a.dg))) return rc;
        StageTimer tm(ctx, 5, s);
        HIPCHK(ctx, launch_normal_bwd(ctx->pb, ctx->L, ctx->ws, *a.out, *a.up, ctx->opt, s));
        return UGS_OK;
    }
    case 6: {
        if ((rc = check_bwd(ctx, a.g, a.ws, a.out, a.up, a.dg))) return rc;
        StageTimer tm(ctx, 6, s);
        HIPCHK(ctx, launch_render_bwd(*a.g, ctx->pb, ctx->L, ctx->ws, *a.out, *a.up, *a.dg,
                                      auto_batch(ctx->opt, a.g->C_o), ctx->final_buf, ctx->counters, s));
        return UGS_OK;
    }
    case 7: {
        if ((rc = check_bwd(ctx, a.g, a.ws, a.out, a.up, a.dg))) return rc;
        StageTimer tm(ctx, 7, s);
        HIPCHK(ctx, launch_project_bwd(*a.g, ctx->pb, ctx->L, ctx->ws, *a.dg, s));
        return UGS_OK;
    }
    case 8:
        hipLaunchKernelGGL(report_flag, dim3(1), dim3(64), 0, s, (const DevCounters *)(ctx->ws + ctx->L.counters),
                           ctx->host_flag_dev);
        HIPCHK(ctx, hipGetLastError());
        return UGS_OK;
    default: return UGS_ERR_INVALID_ARG;
    }
}

int run_stages(ugs_ctx *ctx, const StepArgs &a, int first, int last, hipStream_t s)
{
    for (int st = first; st <= last; ++st) {
        int rc = step_stage(ctx, a, st, s);
        if (rc) return rc;
    }
    return UGS_OK;
}

int do_render_fwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out, hipStream_t s)
{
    StepArgs a{g, nullptr, 0, ws, 0, out, nullptr, nullptr};
    return run_stages(ctx, a, 3, 4, s);
}

int do_render_bwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out, const ugs_upstream *up,
                  const ugs_gaussian_grads *dg, hipStream_t s)
{
    StepArgs a{g, nullptr, 0, ws, 0, out, up, dg};
    int rc = run_stages(ctx, a, 5, 7, s);
    if (rc == UGS_OK) ctx->bwd_done = true;
    return rc;
}

int zero_grads(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_gaussian_grads *dg, hipStream_t s)
{
    const int64_t N = g->N;
    const int nc = (g->sh_deg + 1) * (g->sh_deg + 1);
    HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->mean, 0u, 3 * N, s));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->quat, 0u, 4 * N, s));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->log_scale, 0u, 3 * N, s));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->opacity_logit, 0u, N, s));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->mask_logit, 0u, N, s));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->sh, 0u, (int64_t)nc * 3 * N, s));
    if (g->C_o > 0) HIPCHK(ctx, launch_fill_u32((uint32_t *)dg->sem, 0u, (int64_t)g->C_o * N, s));
    return UGS_OK;
}

int full_step(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws, size_t ws_bytes,
              const ugs_outputs *out, const ugs_upstream *up, const ugs_gaussian_grads *dg, hipStream_t s,
              bool zero)
{
    int rc;
    if ((rc = check_grads(dg, g ? g->C_o : 0))) return rc;
    StepArgs a{g, cams, V, ws, ws_bytes, out, up, dg};
    return run_stages(ctx, a, zero ? 0 : 1, 7, s);
}

// Captures stages [first, last] of a step into a new graph.
int capture_stages(ugs_ctx *ctx, const StepArgs &a, int first, int last, hipStream_t s, hipGraph_t *graph)
{
    *graph = nullptr;
    HIPCHK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = run_stages(ctx, a, first, last, s);
    hipError_t e = hipStreamEndCapture(s, graph);
    if (rc != UGS_OK) {
        if (*graph) hipGraphDestroy(*graph);
        *graph = nullptr;
        return rc;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
    return UGS_OK;
}

void release_graph(ugs_ctx *ctx)
{
    if (ctx->exec) hipGraphExecDestroy(ctx->exec);
    if (ctx->graph) hipGraphDestroy(ctx->graph);
    ctx->exec = nullptr;
    ctx->graph = nullptr;
    ctx->captured = false;
}

}  // namespace

extern "C" {

void ugs_default_options(ugs_options *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->tile_w = 16;
    o->tile_h = 16;
    o->batch = 0;
    o->step1 = 1;
    o->step2 = 2;
    o->lambda = 0.5f;
    o->orient_sign = 1;
    o->prune_Tk = 0.f;
    o->depth_mode = 0;
    o->half_outputs = 0;
    o->sem_bf16x3 = 0;
}

int ugs_create(ugs_ctx **out, const ugs_options *opt)
{
    if (!out) return UGS_ERR_INVALID_ARG;
    ugs_options o;
    if (opt) o = *opt;
    else ugs_default_options(&o);
    int rc = check_options(&o);
    if (rc) return rc;
    ugs_ctx *c = new (std::nothrow) ugs_ctx();
    if (!c) return UGS_ERR_INVALID_ARG;
    c->opt = o;
    *out = c;
    return UGS_OK;
}

void ugs_destroy(ugs_ctx *ctx)
{
    if (!ctx) return;
    release_graph(ctx);
    if (ctx->host_flag) hipHostFree(ctx->host_flag);
    delete ctx;
}

int ugs_set_options(ugs_ctx *ctx, const ugs_options *opt)
{
    if (!ctx) return UGS_ERR_INVALID_ARG;
    int rc = check_options(opt);
    if (rc) return rc;
    ctx->opt = *opt;
    ctx->have_problem = false;
    ctx->sorted = false;
    release_graph(ctx);
    return UGS_OK;
}

int ugs_workspace_size(const ugs_ctx *ctx, int64_t N, int C_o, int sh_deg, const ugs_camera *cams, int V,
                       int64_t pair_capacity, size_t *bytes)
{
    if (!ctx || !bytes || N < 0 || pair_capacity < 0 || pair_capacity > 0x7fffffffll) return UGS_ERR_INVALID_ARG;
    if (C_o < 0 || C_o > UGS_MAX_CHANNELS || sh_deg < 0 || sh_deg > 3) return UGS_ERR_UNSUPPORTED;
    int rc = check_cams(cams, V);
    if (rc) return rc;
    Problem pb;
    make_problem(ctx->opt, N, C_o, sh_deg, cams, V, pb, nullptr);
    *bytes = make_layout(pb, pair_capacity).total;
    return UGS_OK;
}

int ugs_project(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws, size_t ws_bytes,
                void *stream)
{
    if (!ctx) return UGS_ERR_INVALID_ARG;
    return do_project(ctx, g, cams, V, ws, ws_bytes, (hipStream_t)stream);
}

int ugs_bin_sort(ugs_ctx *ctx, void *ws, void *stream, int64_t *P_out)
{
    if (!ctx || !ws) return UGS_ERR_INVALID_ARG;
    return do_bin_sort(ctx, ws, (hipStream_t)stream, P_out);
}

int ugs_check_overflow(ugs_ctx *ctx, void *ws, void *stream, int64_t *P_required)
{
    if (!ctx || !ws) return UGS_ERR_INVALID_ARG;
    if (!ctx->have_problem || ws != ctx->ws) return UGS_ERR_STATE;
    DevCounters c;
    int rc = read_counters(ctx, ws, (hipStream_t)stream, &c);
    if (rc) return rc;
    if (P_required) *P_required = (int64_t)c.P;
    return c.overflow ? UGS_ERR_CAPACITY : UGS_OK;
}

int ugs_pair_count(ugs_ctx *ctx, void *ws, void *stream, int64_t *P)
{
    if (!ctx || !ws || !P) return UGS_ERR_INVALID_ARG;
    if (!ctx->have_problem || ws != ctx->ws) return UGS_ERR_STATE;
    DevCounters c;
    int rc = read_counters(ctx, ws, (hipStream_t)stream, &c);
    if (rc) return rc;
    *P = (int64_t)c.P;
    return UGS_OK;
}

int ugs_render_fwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out, void *stream)
{
    if (!ctx || !ws) return UGS_ERR_INVALID_ARG;
    return do_render_fwd(ctx, g, ws, out, (hipStream_t)stream);
}

int ugs_render_bwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out,
                   const ugs_upstream *dout, const ugs_gaussian_grads *dg, void *stream)
{
    if (!ctx || !ws) return UGS_ERR_INVALID_ARG;
    return do_render_bwd(ctx, g, ws, out, dout, dg, (hipStream_t)stream);
}

int ugs_step_capture(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws,
                     size_t ws_bytes, const ugs_outputs *out, const ugs_upstream *dout,
                     const ugs_gaussian_grads *dg, void *stream)
{
    if (!ctx) return UGS_ERR_INVALID_ARG;
    int rc;
    // dout and dg both NULL: a forward-only step (project, bin_sort, render_fwd, normals)
    const bool fwd_only = !dout && !dg;
    if ((rc = check_gaussians(g)) || (rc = check_cams(cams, V)) || (rc = check_outputs(out, g->C_o, !fwd_only, ctx->opt.half_outputs)) ||
        (!fwd_only && (rc = check_grads(dg, g->C_o))))
        return rc;
    if ((!fwd_only && !dout) || !ws) return UGS_ERR_INVALID_ARG;
    if (fwd_only && ctx->timed_stage >= 5) return UGS_ERR_INVALID_ARG;
    if (!fwd_only && ctx->opt.half_outputs) return UGS_ERR_INVALID_ARG;  // training steps need FP32 maps
    release_graph(ctx);
    hipStream_t s = (hipStream_t)stream;
    if (!ctx->host_flag) {
        HIPCHK(ctx, hipHostMalloc((void **)&ctx->host_flag, 64, hipHostMallocMapped));
        HIPCHK(ctx, hipHostGetDevicePointer((void **)&ctx->host_flag_dev, ctx->host_flag, 0));
    }
    ctx->host_flag[0] = 0;
    StepArgs a{g, cams, V, ws, ws_bytes, out, dout, dg};
    hipGraph_t graph = nullptr;
    const int T = ctx->timed_stage;
    if (T == 0) {
        if ((rc = capture_stages(ctx, a, 0, 8, s, &graph))) return rc;
    } else {
        // before -> event -> timed stage -> event -> after, as child graphs of one graph
        hipGraph_t parts[3] = {nullptr, nullptr, nullptr};
        if ((rc = capture_stages(ctx, a, 0, T - 1, s, &parts[0])) || (rc = capture_stages(ctx, a, T, T, s, &parts[1])) ||
            (rc = capture_stages(ctx, a, T + 1, 8, s, &parts[2]))) {
            for (auto p : parts)
                if (p) hipGraphDestroy(p);
            return rc;
        }
        hipError_t e = hipGraphCreate(&graph, 0);
        hipGraphNode_t n0, e0, n1, e1, n2;
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&n0, graph, nullptr, 0, parts[0]);
        if (e == hipSuccess) e = hipGraphAddEventRecordNode(&e0, graph, &n0, 1, ctx->ev_start);
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&n1, graph, &e0, 1, parts[1]);
        if (e == hipSuccess) e = hipGraphAddEventRecordNode(&e1, graph, &n1, 1, ctx->ev_stop);
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&n2, graph, &e1, 1, parts[2]);
        for (auto p : parts) hipGraphDestroy(p);  // child nodes hold their own copies
        if (e != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return hip_fail(ctx, e, "assembling the timed step graph");
        }
    }
    ctx->graph = graph;
    hipError_t e = hipGraphInstantiate(&ctx->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        release_graph(ctx);
        return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    ctx->captured = true;
    return UGS_OK;
}

int ugs_step_replay(ugs_ctx *ctx, void *stream)
{
    if (!ctx) return UGS_ERR_INVALID_ARG;
    if (!ctx->captured) return UGS_ERR_NOT_CAPTURED;
    if (ctx->host_flag && __atomic_load_n(&ctx->host_flag[0], __ATOMIC_ACQUIRE)) return UGS_ERR_CAPACITY;
    HIPCHK(ctx, hipGraphLaunch(ctx->exec, (hipStream_t)stream));
    ctx->bwd_done = true;  // a replayed training step consumes its gradient records
    return UGS_OK;
}

int ugs_autotune(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws, size_t ws_bytes,
                 const ugs_outputs *out, const ugs_upstream *dout, const ugs_gaussian_grads *dg, void *stream,
                 ugs_options *chosen, float *ms)
{
    if (!ctx || !g || !out || !dout || !dg || ctx->opt.half_outputs) return UGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const ugs_options base = ctx->opt;
    struct Cand { int tw, th, batch; };
    std::vector<Cand> cands;
    const int tiles[3][2] = {{16, 16}, {8, 8}, {32, 8}};
    for (auto &t : tiles) {
        ugs_options o = base;
        o.tile_w = t[0];
        o.tile_h = t[1];
        o.batch = 0;
        int b = auto_batch(o, g->C_o);
        cands.push_back({t[0], t[1], b});
        // twice the default batch: fewer barriers, more LDS (at most 64 KB,
        // since the default fits in 32 KB)
        if (2 * b <= 1024) cands.push_back({t[0], t[1], 2 * b});
        // one and a half times (a multiple of 16): the 3M-Gaussian 128-channel
        // step takes its forward passes fastest at 96 with a default of 64
        const int b3 = (3 * b / 2 + 15) / 16 * 16;
        if (b3 > b && b3 < 2 * b) cands.push_back({t[0], t[1], b3});
        if (b / 2 >= 16) cands.push_back({t[0], t[1], b / 2});
        if (b / 4 >= 16) cands.push_back({t[0], t[1], b / 4});
    }
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    unsigned long long ref_hash = 0;
    double ref_sum = 0.0, ref_abs = 0.0;
    float best = 1e30f;
    ugs_options best_opt = base;
    int rc = UGS_OK;
    bool mismatch = false, have_ref = false;
    size_t skipped = 0;
    for (size_t ci = 0; ci < cands.size() && rc == UGS_OK; ++ci) {
        ugs_options o = base;
        o.tile_w = cands[ci].tw;
        o.tile_h = cands[ci].th;
        o.batch = cands[ci].batch;
        ctx->opt = o;
        release_graph(ctx);
        // warm-up and capacity check
        if ((rc = full_step(ctx, g, cams, V, ws, ws_bytes, out, dout, dg, s, true))) break;
        int64_t Preq = 0;
        rc = ugs_check_overflow(ctx, ws, s, &Preq);
        if (rc == UGS_ERR_CAPACITY) {  // this tile shape needs more pairs than the workspace holds
            rc = UGS_OK;
            ++skipped;
            continue;
        }
        if (rc) break;
        float tmin = 1e30f;
        for (int r = 0; r < 2 && rc == UGS_OK; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = UGS_ERR_HIP; break; }
            rc = full_step(ctx, g, cams, V, ws, ws_bytes, out, dout, dg, s, true);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = UGS_ERR_HIP; break; }
            float t = 0.f;
            hipEventElapsedTime(&t, e0, e1);
            tmin = std::min(tmin, t);
        }
        if (rc) break;
        // fingerprint the tile-independent forward outputs: bit for bit, except
        // the semantic map, whose matrix-core sums group list entries per tile
        // (compared by its FP64 sum, to 1e-6 of its absolute sum)
        auto hp = (unsigned long long *)(ctx->ws + ctx->L.counters + sizeof(DevCounters));
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, hp, 3);
        const int64_t P = ctx->pb.total_pix;
        struct { const float *p; int64_t n; } maps[] = {{out->rgb, 3 * P}, {out->depth, P}, {out->kmap, P},
                                                         {out->normal, 3 * P}, {out->T_final, P}};
        unsigned long long salt = 1;
        for (auto &m : maps) {
            if (m.n > 0 && m.p) hipLaunchKernelGGL(hash_floats, dim3(1024), dim3(256), 0, s, m.p, m.n, salt * 0x9e3779b97f4a7c15ull, hp);
            ++salt;
        }
        if (g->C_o > 0 && out->sem)
            hipLaunchKernelGGL(sum_floats, dim3(1024), dim3(256), 0, s, out->sem, (int64_t)g->C_o * P, (double *)(hp + 1));
        unsigned long long hs[3] = {0, 0, 0};
        if (hipMemcpyAsync(hs, hp, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            rc = UGS_ERR_HIP;
            break;
        }
        const unsigned long long h = hs[0];
        double ssum, sabs;
        memcpy(&ssum, &hs[1], 8);
        memcpy(&sabs, &hs[2], 8);
        if (!have_ref) {
            ref_hash = h;
            ref_sum = ssum;
            ref_abs = sabs;
            have_ref = true;
        } else if (h != ref_hash || fabs(ssum - ref_sum) > 1e-6 * ref_abs + 1e-30) {
            mismatch = true;
        }
        if (tmin < best) {
            best = tmin;
            best_opt = o;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == UGS_OK && skipped == cands.size()) rc = UGS_ERR_CAPACITY;
    ctx->opt = (rc == UGS_OK) ? best_opt : base;
    ctx->have_problem = false;
    ctx->sorted = false;
    if (rc == UGS_OK) rc = zero_grads(ctx, g, dg, s);
    if (rc != UGS_OK) return rc;
    if (chosen) *chosen = best_opt;
    if (ms) *ms = best;
    return mismatch ? UGS_ERR_STATE : UGS_OK;
}

int ugs_time_stage(ugs_ctx *ctx, int stage, void *ev_start, void *ev_stop)
{
    if (!ctx || stage < 0 || stage > 7) return UGS_ERR_INVALID_ARG;
    if (stage && (!ev_start || !ev_stop)) return UGS_ERR_INVALID_ARG;
    ctx->timed_stage = stage;
    ctx->ev_start = (hipEvent_t)ev_start;
    ctx->ev_stop = (hipEvent_t)ev_stop;
    return UGS_OK;
}

int ugs_debug_buffer(ugs_ctx *ctx, void *ws, int which, void *stream, void **dev_ptr, int64_t *count)
{
    if (!ctx || !ws || !dev_ptr || !count) return UGS_ERR_INVALID_ARG;
    if (!ctx->have_problem || ws != ctx->ws) return UGS_ERR_STATE;
    const WsLayout &L = ctx->L;
    char *b = ctx->ws;
    switch (which) {
    case 0: *dev_ptr = b + L.rec; *count = L.VN; return UGS_OK;
    case 1: *dev_ptr = b + L.rect; *count = L.VN; return UGS_OK;
    case 2: *dev_ptr = b + L.touched; *count = L.VN; return UGS_OK;
    case 3:
    case 4: {
        if (!ctx->sorted) return UGS_ERR_STATE;
        DevCounters c;
        int rc = read_counters(ctx, ws, (hipStream_t)stream, &c);
        if (rc) return rc;
        *count = (int64_t)c.P_eff;
        *dev_ptr = b + (which == 3 ? (ctx->final_buf ? L.keys1 : L.keys0) : (ctx->final_buf ? L.vals1 : L.vals0));
        return UGS_OK;
    }
    case 5: *dev_ptr = b + L.ranges; *count = L.total_tiles; return UGS_OK;
    case 6: *dev_ptr = b + L.grec; *count = L.VN; return UGS_OK;
    case 7: *dev_ptr = b + L.gd; *count = L.total_pix; return UGS_OK;
    case 8: *dev_ptr = b + L.tclk; *count = L.total_tiles; return UGS_OK;
    case 9: *dev_ptr = b + L.tclk + (size_t)L.total_tiles * 16; *count = L.total_tiles; return UGS_OK;
    case 10: *dev_ptr = b + L.amask; *count = (int64_t)kMaskPlanes * L.amask_words; return UGS_OK;
    default: return UGS_ERR_INVALID_ARG;
    }
}

const char *ugs_status_string(int st)
{
    switch (st) {
    case UGS_OK: return "ok";
    case UGS_ERR_INVALID_ARG: return "invalid argument";
    case UGS_ERR_UNSUPPORTED: return "unsupported size or option";
    case UGS_ERR_CAPACITY: return "pair capacity exceeded";
    case UGS_ERR_HIP: return "HIP runtime error";
    case UGS_ERR_NOT_CAPTURED: return "no captured step";
    case UGS_ERR_STATE: return "call out of order or inconsistent results";
    default: return "unknown status";
    }
}

const char *ugs_last_hip_error(const ugs_ctx *ctx) { return ctx ? ctx->err : ""; }

int ugs_enable_counters(ugs_ctx *ctx, int on)
{
    if (!ctx) return UGS_ERR_INVALID_ARG;
    ctx->counters = on != 0;
    return UGS_OK;
}

int ugs_read_counters(ugs_ctx *ctx, void *ws, void *stream, int64_t *evaluated, int64_t *contributing)
{
    if (!ctx || !ws) return UGS_ERR_INVALID_ARG;
    if (!ctx->have_problem || ws != ctx->ws) return UGS_ERR_STATE;
    DevCounters c;
    int rc = read_counters(ctx, ws, (hipStream_t)stream, &c);
    if (rc) return rc;
    if (evaluated) *evaluated = (int64_t)c.n_eval;
    if (contributing) *contributing = (int64_t)c.n_contrib;
    return UGS_OK;
}

}  // extern "C"
