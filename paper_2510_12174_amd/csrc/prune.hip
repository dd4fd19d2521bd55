// Differentiable pruning (section 3.3, "Pruning"): every K_p iterations the
// Gaussians whose gradient factor strays from 1 by more than T_k are dropped
// and the gradient factor of the survivors is reset to 0.9.  On the device this
// is a stream compaction of the structure-of-arrays parameter set (and of any
// per-Gaussian state laid out like it, such as optimiser moments): keep flags,
// an exclusive scan, and one scatter that copies every field of a kept
// Gaussian to its compacted position.  The keep test is the projection's skip
// test, |sigmoid(mask_logit) - 1| <= T_k evaluated in FP64, so a pruned set
// renders exactly like the full set with the skip enabled.
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

// Copies row r (stride N in, stride M out) of a structure-of-arrays field.
__device__ __forceinline__ void copy_rows(const float *in, float *out, int rows, int64_t N, int64_t M, int64_t i,
                                          int64_t j)
{
    if (!in || !out) return;
    for (int r = 0; r < rows; ++r) out[r * M + j] = in[r * N + i];
}

__global__ void __launch_bounds__(kPruneThreads) prune_scatter(ugs_gaussians in, ugs_gaussian_grads out, int nsh,
                                                               const uint32_t *__restrict__ flags,
                                                               const uint32_t *__restrict__ pos,
                                                               const uint32_t *__restrict__ total, int reset,
                                                               float reset_logit)
{
    const int64_t N = in.N;
    const int64_t i = (int64_t)blockIdx.x * kPruneThreads + threadIdx.x;
    if (i >= N || !flags[i]) return;
    const int64_t j = pos[i], M = *total;
    copy_rows(in.mean, out.mean, 3, N, M, i, j);
    copy_rows(in.quat, out.quat, 4, N, M, i, j);
    copy_rows(in.log_scale, out.log_scale, 3, N, M, i, j);
    copy_rows(in.opacity_logit, out.opacity_logit, 1, N, M, i, j);
    if (out.mask_logit) out.mask_logit[j] = reset ? reset_logit : (in.mask_logit ? in.mask_logit[i] : 0.f);
    copy_rows(in.sh, out.sh, nsh, N, M, i, j);
    if (in.sem && out.sem)
        for (int c = 0; c < in.C_o; ++c) out.sem[j * in.C_o + c] = in.sem[i * in.C_o + c];
}

int64_t scan_parts(int64_t N) { return (N + kScanBlock - 1) / kScanBlock; }

}  // namespace
}  // namespace ugs

using namespace ugs;

extern "C" {

int ugs_prune_scratch_size(int64_t N, size_t *bytes)
{
    if (N < 0 || !bytes) return UGS_ERR_INVALID_ARG;
    *bytes = (size_t)(8 * N + 4 * scan_parts(N) + 256);
    return UGS_OK;
}

int ugs_prune(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state, const ugs_gaussians *state_in,
              const ugs_gaussian_grads *state_out, float T_k, int reset_k, void *scratch, size_t scratch_bytes,
              int64_t *n_kept, void *stream)
{
    if (!g || !out || !n_kept || !scratch || n_state < 0 || (n_state > 0 && (!state_in || !state_out)))
        return UGS_ERR_INVALID_ARG;
    if (!(T_k >= 0.f) || g->N < 0 || g->N > 0xffffffffll || g->sh_deg < 0 || g->sh_deg > 3 || g->C_o < 0 ||
        g->C_o > UGS_MAX_CHANNELS)
        return UGS_ERR_INVALID_ARG;
    if (!g->mask_logit || (reinterpret_cast<uintptr_t>(scratch) & 255)) return UGS_ERR_INVALID_ARG;
    size_t need;
    ugs_prune_scratch_size(g->N, &need);
    if (scratch_bytes < need) return UGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = g->N;
    if (N == 0) {
        *n_kept = 0;
        return UGS_OK;
    }
    char *p = (char *)scratch;
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
    hipLaunchKernelGGL(prune_scatter, dim3(blocks), dim3(kPruneThreads), 0, s, *g, *out, nsh, (const uint32_t *)flags,
                       (const uint32_t *)pos, (const uint32_t *)total, reset_k ? 1 : 0, reset_logit);
    for (int k = 0; k < n_state; ++k) {
        ugs_gaussians si = state_in[k];
        si.N = N;
        si.sh_deg = g->sh_deg;
        si.C_o = g->C_o;
        hipLaunchKernelGGL(prune_scatter, dim3(blocks), dim3(kPruneThreads), 0, s, si, state_out[k], nsh,
                           (const uint32_t *)flags, (const uint32_t *)pos, (const uint32_t *)total, 0, 0.f);
    }
    if (hipGetLastError() != hipSuccess) return UGS_ERR_HIP;
    uint32_t h = 0;
    if (hipMemcpyAsync(&h, total, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return UGS_ERR_HIP;
    *n_kept = (int64_t)h;
    return UGS_OK;
}

}  // extern "C"
