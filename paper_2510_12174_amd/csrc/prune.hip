// Differentiable pruning (section 3.3, "Pruning"): every K_p iterations the
// Gaussians whose gradient factor strays from 1 by more than T_k are dropped
// and the gradient factor of the survivors is reset to 0.9.  On the device this
// is a stream compaction of the structure-of-arrays parameter set (and of any
// per-Gaussian state laid out like it, such as optimiser moments): keep flags,
// an exclusive scan, and one scatter that copies every field of a kept
// Gaussian to its compacted position.  The keep test is the projection's skip
// test, |sigmoid(mask_logit) - 1| <= T_k evaluated in FP64, so a pruned set
// renders exactly like the full set with the skip enabled.
#include <mutex>

#include "ugs_internal.h"

namespace ugs {
namespace {

constexpr int kPruneThreads = 256;

__global__ void __launch_bounds__(kPruneThreads) prune_flags(const float *__restrict__ mask_logit, int64_t N,
                                                             double T_k, uint32_t *__restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * kPruneThreads + threadIdx.x;
    if (i >= N) return;
    const double k = 1.0 / (1.0 + exp(-(double)mask_logit[i]));
    flags[i] = fabs(k - 1.0) > T_k ? 0u : 1u;
}

// One structure-of-arrays row per grid row: src points at the input row
// (length N), dst at the output field, whose row `rl` starts at rl * M with M
// the kept count (known on the device only).
constexpr int kMaxRows = 64;
struct RowTable {
    const float *src[kMaxRows];
    float *dst[kMaxRows];
    int rl[kMaxRows];
    int reset[kMaxRows];  // write reset_logit instead of copying (mask logits)
};

// One thread per (Gaussian, row): every element is one coalesced load and one
// coalesced store, so the copy runs at memory speed instead of walking a
// Gaussian's rows one after the other.
__global__ void __launch_bounds__(kPruneThreads) prune_rows(RowTable t, int64_t N, const uint32_t *__restrict__ flags,
                                                            const uint32_t *__restrict__ pos,
                                                            const uint32_t *__restrict__ total, float reset_logit)
{
    const int64_t i = (int64_t)blockIdx.x * kPruneThreads + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= N || !flags[i]) return;
    const int64_t j = pos[i], M = *total;
    t.dst[r][t.rl[r] * M + j] = t.reset[r] ? reset_logit : t.src[r][i];
}

// Row-major [N][C] arrays (semantic logits): one thread per element.
__global__ void __launch_bounds__(kPruneThreads) prune_rowmajor(const float *__restrict__ src, float *__restrict__ dst,
                                                                int64_t N, int C, const uint32_t *__restrict__ flags,
                                                                const uint32_t *__restrict__ pos)
{
    const int64_t e = (int64_t)blockIdx.x * kPruneThreads + threadIdx.x;
    if (e >= N * C) return;
    const int64_t i = e / C;
    if (!flags[i]) return;
    dst[(int64_t)pos[i] * C + (e - i * C)] = src[e];
}

// Fills the row table of one parameter set; returns the row count.
int row_table(const ugs_gaussians &in, const ugs_gaussian_grads &out, int nsh, int reset, RowTable &t)
{
    int n = 0;
    auto add = [&](const float *src, float *dst, int rows, int rs) {
        if (!src || !dst) return;
        for (int r = 0; r < rows; ++r) {
            t.src[n] = src + (int64_t)r * in.N;
            t.dst[n] = dst;
            t.rl[n] = r;
            t.reset[n] = rs;
            ++n;
        }
    };
    add(in.mean, out.mean, 3, 0);
    add(in.quat, out.quat, 4, 0);
    add(in.log_scale, out.log_scale, 3, 0);
    add(in.opacity_logit, out.opacity_logit, 1, 0);
    if (reset && out.mask_logit) add(out.mask_logit, out.mask_logit, 1, 1);  // src unused
    else add(in.mask_logit, out.mask_logit, 1, 0);
    add(in.sh, out.sh, nsh, 0);
    return n;
}

int compact_set(const ugs_gaussians &in, const ugs_gaussian_grads &out, int nsh, int reset, const uint32_t *flags,
                const uint32_t *pos, const uint32_t *total, float reset_logit, hipStream_t s)
{
    RowTable t;
    const int n = row_table(in, out, nsh, reset, t);
    const unsigned bx = (unsigned)((in.N + kPruneThreads - 1) / kPruneThreads);
    if (n > 0)
        hipLaunchKernelGGL(prune_rows, dim3(bx, (unsigned)n), dim3(kPruneThreads), 0, s, t, in.N, flags, pos, total,
                           reset_logit);
    if (in.sem && out.sem && in.C_o > 0) {
        const int64_t ne = in.N * in.C_o;
        hipLaunchKernelGGL(prune_rowmajor, dim3((unsigned)((ne + kPruneThreads - 1) / kPruneThreads)),
                           dim3(kPruneThreads), 0, s, in.sem, out.sem, in.N, in.C_o, flags, pos);
    }
    return hipGetLastError() == hipSuccess ? UGS_OK : UGS_ERR_HIP;
}

int64_t scan_parts(int64_t N) { return (N + kScanBlock - 1) / kScanBlock; }

size_t prune_scratch_bytes(int64_t N) { return (size_t)(8 * N + 4 * scan_parts(N) + 256); }

int check_prune_args(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state,
                     const ugs_gaussians *state_in, const ugs_gaussian_grads *state_out, float T_k,
                     const int64_t *n_kept)
{
    if (!g || !out || !n_kept || n_state < 0 || (n_state > 0 && (!state_in || !state_out)))
        return UGS_ERR_INVALID_ARG;
    if (!(T_k >= 0.f) || g->N < 0 || g->N > 0xffffffffll || g->sh_deg < 0 || g->sh_deg > 3 || g->C_o < 0 ||
        g->C_o > UGS_MAX_CHANNELS)
        return UGS_ERR_INVALID_ARG;
    if (!g->mask_logit) return UGS_ERR_INVALID_ARG;
    return UGS_OK;
}

// The compaction itself, given a device scratch of prune_scratch_bytes(g->N)
// bytes (256-byte aligned): keep flags, their exclusive scan and the kept count
// are all written before they are read, so the scratch needs no clearing.
int prune_impl(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state, const ugs_gaussians *state_in,
               const ugs_gaussian_grads *state_out, float T_k, int reset_k, char *p, int64_t *n_kept, hipStream_t s)
{
    const int64_t N = g->N;
    if (N == 0) {
        *n_kept = 0;
        return UGS_OK;
    }
    uint32_t *total = (uint32_t *)p;            // 256 B header
    uint32_t *flags = (uint32_t *)(p + 256);
    uint32_t *pos = flags + N;
    uint32_t *part = pos + N;
    const unsigned blocks = (unsigned)((N + kPruneThreads - 1) / kPruneThreads);
    const int nsh = 3 * (g->sh_deg + 1) * (g->sh_deg + 1);
    hipLaunchKernelGGL(prune_flags, dim3(blocks), dim3(kPruneThreads), 0, s, g->mask_logit, N, (double)T_k, flags);
    if (hipGetLastError() != hipSuccess) return UGS_ERR_HIP;
    if (launch_scan_flags(flags, N, part, pos, total, s) != hipSuccess) return UGS_ERR_HIP;
    // logit(0.9) = ln 9
    const float reset_logit = 2.19722457733621956f;
    int rc = compact_set(*g, *out, nsh, reset_k ? 1 : 0, flags, pos, total, reset_logit, s);
    for (int k = 0; k < n_state && rc == UGS_OK; ++k) {
        ugs_gaussians si = state_in[k];
        si.N = N;
        si.sh_deg = g->sh_deg;
        si.C_o = g->C_o;
        rc = compact_set(si, state_out[k], nsh, 0, flags, pos, total, 0.f, s);
    }
    if (rc != UGS_OK) return rc;
    uint32_t h = 0;
    if (hipMemcpyAsync(&h, total, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return UGS_ERR_HIP;
    *n_kept = (int64_t)h;
    return UGS_OK;
}

// Library-held scratch of ugs_prune_noalloc: one copy per GPU, kept until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name is a host-side stand-in, not a device address): it passes the
// device address that hipGetSymbolAddress returns for the current device,
// looked up once per device on the first call there.
constexpr size_t kNoAllocScratchBytes = (size_t)8 * UGS_PRUNE_NOALLOC_MAX_N +
                                        (size_t)4 * ((UGS_PRUNE_NOALLOC_MAX_N + kScanBlock - 1) / kScanBlock) + 256;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

int noalloc_scratch(char **p)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return UGS_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return UGS_ERR_HIP;
        g_scratch_dev[dev] = ptr;
    }
    *p = (char *)g_scratch_dev[dev];
    return UGS_OK;
}

}  // namespace
}  // namespace ugs

using namespace ugs;

extern "C" {

int ugs_prune_scratch_size(int64_t N, size_t *bytes)
{
    if (N < 0 || !bytes) return UGS_ERR_INVALID_ARG;
    *bytes = prune_scratch_bytes(N);
    return UGS_OK;
}

int ugs_prune(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state, const ugs_gaussians *state_in,
              const ugs_gaussian_grads *state_out, float T_k, int reset_k, void *scratch_mem, size_t scratch_bytes,
              int64_t *n_kept, void *stream)
{
    int rc = check_prune_args(g, out, n_state, state_in, state_out, T_k, n_kept);
    if (rc) return rc;
    if (!scratch_mem || (reinterpret_cast<uintptr_t>(scratch_mem) & 255)) return UGS_ERR_INVALID_ARG;
    if (scratch_bytes < prune_scratch_bytes(g->N)) return UGS_ERR_INVALID_ARG;
    return prune_impl(g, out, n_state, state_in, state_out, T_k, reset_k, (char *)scratch_mem, n_kept,
                      (hipStream_t)stream);
}

int ugs_prune_noalloc(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state,
                      const ugs_gaussians *state_in, const ugs_gaussian_grads *state_out, float T_k, int reset_k,
                      int64_t *n_kept, void *stream)
{
    int rc = check_prune_args(g, out, n_state, state_in, state_out, T_k, n_kept);
    if (rc) return rc;
    if (g->N > UGS_PRUNE_NOALLOC_MAX_N) return UGS_ERR_UNSUPPORTED;
    char *p = nullptr;
    if ((rc = noalloc_scratch(&p))) return rc;
    return prune_impl(g, out, n_state, state_in, state_out, T_k, reset_k, p, n_kept, (hipStream_t)stream);
}

}  // extern "C"
