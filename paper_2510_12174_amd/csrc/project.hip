// Stage S1 (projection) and stage S9 (its backward) for gfx950.
//
// One thread per Gaussian; the thread loops over all views so that the
// parameters (up to ~750 B per Gaussian) are read from HBM once per step, not
// once per view.  Parameters are structure-of-arrays, so every load is a fully
// coalesced 4-byte-per-lane stream.
#include "ugs_internal.h"

namespace ugs {
namespace {

constexpr int kProjThreads = 256;

// Real SH basis (degree <= 3, Condon-Shortley phase, the 3DGS ordering that
// UniGS inherits for colour).  Values are the closed-form normalisations
// sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) times the Legendre factors.
struct SHK {
    static constexpr double c0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
    static constexpr double c1 = 0.48860251190291992;   // sqrt(3)/(2 sqrt(pi))
    static constexpr double c2a = 1.0925484305920792;   // sqrt(15)/(2 sqrt(pi))
    static constexpr double c2b = 0.31539156525252005;  // sqrt(5)/(4 sqrt(pi))
    static constexpr double c2c = 0.54627421529603959;  // sqrt(15)/(4 sqrt(pi))
    static constexpr double c3a = 0.59004358992664352;  // sqrt(35/(2 pi))/4
    static constexpr double c3b = 2.8906114426405538;   // sqrt(105/pi)/2
    static constexpr double c3c = 0.45704579946446572;  // sqrt(21/(2 pi))/4
    static constexpr double c3d = 0.37317633259011546;  // sqrt(7/pi)/4
    static constexpr double c3e = 1.4453057213202769;   // sqrt(105/pi)/4
};

template <int DEG, typename F>
__device__ __forceinline__ void sh_basis(F x, F y, F z, F *Y)
{
    Y[0] = F(SHK::c0);
    if constexpr (DEG >= 1) {
        Y[1] = -F(SHK::c1) * y;
        Y[2] = F(SHK::c1) * z;
        Y[3] = -F(SHK::c1) * x;
    }
    if constexpr (DEG >= 2) {
        F xx = x * x, yy = y * y, zz = z * z;
        Y[4] = F(SHK::c2a) * x * y;
        Y[5] = -F(SHK::c2a) * y * z;
        Y[6] = F(SHK::c2b) * (F(2) * zz - xx - yy);
        Y[7] = -F(SHK::c2a) * x * z;
        Y[8] = F(SHK::c2c) * (xx - yy);
    }
    if constexpr (DEG >= 3) {
        F xx = x * x, yy = y * y, zz = z * z;
        Y[9] = -F(SHK::c3a) * y * (F(3) * xx - yy);
        Y[10] = F(SHK::c3b) * x * y * z;
        Y[11] = -F(SHK::c3c) * y * (F(4) * zz - xx - yy);
        Y[12] = F(SHK::c3d) * z * (F(2) * zz - F(3) * xx - F(3) * yy);
        Y[13] = -F(SHK::c3c) * x * (F(4) * zz - xx - yy);
        Y[14] = F(SHK::c3e) * z * (xx - yy);
        Y[15] = -F(SHK::c3a) * x * (xx - F(3) * yy);
    }
}

// d/d(x,y,z) of sum_c Y_c(x,y,z) w_c for a weight vector w (one colour channel's
// coefficients scaled by its upstream gradient).
template <int DEG, typename F>
__device__ __forceinline__ void sh_basis_vjp(F x, F y, F z, const F *w, F &gx, F &gy, F &gz)
{
    gx = gy = gz = F(0);
    if constexpr (DEG >= 1) {
        gy += -F(SHK::c1) * w[1];
        gz += F(SHK::c1) * w[2];
        gx += -F(SHK::c1) * w[3];
    }
    if constexpr (DEG >= 2) {
        gx += F(SHK::c2a) * y * w[4];
        gy += F(SHK::c2a) * x * w[4];
        gy += -F(SHK::c2a) * z * w[5];
        gz += -F(SHK::c2a) * y * w[5];
        gx += -F(2) * F(SHK::c2b) * x * w[6];
        gy += -F(2) * F(SHK::c2b) * y * w[6];
        gz += F(4) * F(SHK::c2b) * z * w[6];
        gx += -F(SHK::c2a) * z * w[7];
        gz += -F(SHK::c2a) * x * w[7];
        gx += F(2) * F(SHK::c2c) * x * w[8];
        gy += -F(2) * F(SHK::c2c) * y * w[8];
    }
    if constexpr (DEG >= 3) {
        F xx = x * x, yy = y * y, zz = z * z;
        gx += -F(6) * F(SHK::c3a) * x * y * w[9];
        gy += -F(3) * F(SHK::c3a) * (xx - yy) * w[9];
        gx += F(SHK::c3b) * y * z * w[10];
        gy += F(SHK::c3b) * x * z * w[10];
        gz += F(SHK::c3b) * x * y * w[10];
        gx += F(2) * F(SHK::c3c) * x * y * w[11];
        gy += -F(SHK::c3c) * (F(4) * zz - xx - F(3) * yy) * w[11];
        gz += -F(8) * F(SHK::c3c) * y * z * w[11];
        gx += -F(6) * F(SHK::c3d) * x * z * w[12];
        gy += -F(6) * F(SHK::c3d) * y * z * w[12];
        gz += F(SHK::c3d) * (F(6) * zz - F(3) * xx - F(3) * yy) * w[12];
        gx += -F(SHK::c3c) * (F(4) * zz - F(3) * xx - yy) * w[13];
        gy += F(2) * F(SHK::c3c) * x * y * w[13];
        gz += -F(8) * F(SHK::c3c) * x * z * w[13];
        gx += F(2) * F(SHK::c3e) * x * z * w[14];
        gy += -F(2) * F(SHK::c3e) * y * z * w[14];
        gz += F(SHK::c3e) * (xx - yy) * w[14];
        gx += -F(3) * F(SHK::c3a) * (xx - yy) * w[15];
        gy += F(6) * F(SHK::c3a) * x * y * w[15];
    }
}

__device__ __forceinline__ float m_exp(float x) { return __expf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
template <typename F> __device__ __forceinline__ F m_min(F a, F b) { return a < b ? a : b; }
template <typename F> __device__ __forceinline__ F m_max(F a, F b) { return a > b ? a : b; }
template <typename F> __device__ __forceinline__ F m_sigmoid(F x) { return F(1) / (F(1) + m_exp(-x)); }

// Rotation matrix (row-major) of the unit quaternion (w, x, y, z).
template <typename F>
__device__ __forceinline__ void rotmat(F w, F x, F y, F z, F *M)
{
    M[0] = F(1) - F(2) * (y * y + z * z);
    M[1] = F(2) * (x * y - w * z);
    M[2] = F(2) * (x * z + w * y);
    M[3] = F(2) * (x * y + w * z);
    M[4] = F(1) - F(2) * (x * x + z * z);
    M[5] = F(2) * (y * z - w * x);
    M[6] = F(2) * (x * z - w * y);
    M[7] = F(2) * (y * z + w * x);
    M[8] = F(1) - F(2) * (x * x + y * y);
}

// Gaussian-level quantities shared by every view.
template <typename F>
struct GaussState {
    F mu[3], s[3], is2[3], qn, qh[4], Rg[9], Sig[6];  // Sig: 00 01 02 11 12 22
    F o, k;
};

template <typename F>
__device__ __forceinline__ void load_gauss(const ugs_gaussians &g, int64_t i, GaussState<F> &G)
{
    const int64_t N = g.N;
    for (int a = 0; a < 3; ++a) {
        G.mu[a] = F(g.mean[a * N + i]);
        G.s[a] = m_exp(F(g.log_scale[a * N + i]));
        G.is2[a] = F(1) / (G.s[a] * G.s[a]);
    }
    F q0 = F(g.quat[i]), q1 = F(g.quat[N + i]), q2 = F(g.quat[2 * N + i]), q3 = F(g.quat[3 * N + i]);
    G.qn = m_sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    F iq = F(1) / G.qn;
    G.qh[0] = q0 * iq; G.qh[1] = q1 * iq; G.qh[2] = q2 * iq; G.qh[3] = q3 * iq;
    rotmat(G.qh[0], G.qh[1], G.qh[2], G.qh[3], G.Rg);
    F s2[3] = {G.s[0] * G.s[0], G.s[1] * G.s[1], G.s[2] * G.s[2]};
    const F *M = G.Rg;
    auto sig = [&](int a, int b) { return M[3 * a] * s2[0] * M[3 * b] + M[3 * a + 1] * s2[1] * M[3 * b + 1] + M[3 * a + 2] * s2[2] * M[3 * b + 2]; };
    G.Sig[0] = sig(0, 0); G.Sig[1] = sig(0, 1); G.Sig[2] = sig(0, 2);
    G.Sig[3] = sig(1, 1); G.Sig[4] = sig(1, 2); G.Sig[5] = sig(2, 2);
    G.o = m_sigmoid(F(g.opacity_logit[i]));
    G.k = m_sigmoid(F(g.mask_logit[i]));
}

// View-dependent projection state.
template <typename F>
struct ViewState {
    F mc[3], z, tx, ty;
    bool clx, cly;
    F T0[3], T1[3];      // rows of J R
    F cov00, cov01, cov11;
    F ca, cb, cc;         // conic
    F m2x, m2y;
    F dir[3], dist;
    F M[9];               // R Rg
    F p0[3], wv[3], A, iA, Qp0x, Qp0y, Q00, Q01, Q11;
};

template <typename F>
__device__ __forceinline__ void project_view(const GaussState<F> &G, const DevCam &cam, ViewState<F> &S)
{
    F R[9];
    for (int k = 0; k < 9; ++k) R[k] = F(cam.R[k]);
    const F fx = F(cam.fx), fy = F(cam.fy), limx = F(cam.limx), limy = F(cam.limy);
    for (int a = 0; a < 3; ++a) S.mc[a] = R[3 * a] * G.mu[0] + R[3 * a + 1] * G.mu[1] + R[3 * a + 2] * G.mu[2] + F(cam.t[a]);
    F z = S.mc[2];
    S.z = z;
    F iz = F(1) / z;
    F rx = S.mc[0] * iz, ry = S.mc[1] * iz;
    S.clx = rx < -limx || rx > limx;
    S.cly = ry < -limy || ry > limy;
    S.tx = m_min(limx, m_max(-limx, rx)) * z;
    S.ty = m_min(limy, m_max(-limy, ry)) * z;
    F J00 = fx * iz, J02 = -fx * S.tx * iz * iz;
    F J11 = fy * iz, J12 = -fy * S.ty * iz * iz;
    for (int b = 0; b < 3; ++b) {
        S.T0[b] = J00 * R[b] + J02 * R[6 + b];
        S.T1[b] = J11 * R[3 + b] + J12 * R[6 + b];
    }
    const F *Sg = G.Sig;
    auto quad = [&](const F *u, const F *v) {
        F su0 = Sg[0] * u[0] + Sg[1] * u[1] + Sg[2] * u[2];
        F su1 = Sg[1] * u[0] + Sg[3] * u[1] + Sg[4] * u[2];
        F su2 = Sg[2] * u[0] + Sg[4] * u[1] + Sg[5] * u[2];
        return v[0] * su0 + v[1] * su1 + v[2] * su2;
    };
    S.cov00 = quad(S.T0, S.T0) + F(kLowPass);
    S.cov01 = quad(S.T0, S.T1);
    S.cov11 = quad(S.T1, S.T1) + F(kLowPass);
    F idet = F(1) / (S.cov00 * S.cov11 - S.cov01 * S.cov01);
    S.ca = S.cov11 * idet;
    S.cb = -S.cov01 * idet;
    S.cc = S.cov00 * idet;
    S.m2x = fx * S.mc[0] * iz + F(cam.cx);
    S.m2y = fy * S.mc[1] * iz + F(cam.cy);
    F v0 = G.mu[0] - F(cam.C[0]), v1 = G.mu[1] - F(cam.C[1]), v2 = G.mu[2] - F(cam.C[2]);
    S.dist = m_sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    F id = F(1) / S.dist;
    S.dir[0] = v0 * id; S.dir[1] = v1 * id; S.dir[2] = v2 * id;
    // camera-frame axes of the ellipsoid and the depth quadric
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) S.M[3 * a + k] = R[3 * a] * G.Rg[k] + R[3 * a + 1] * G.Rg[3 + k] + R[3 * a + 2] * G.Rg[6 + k];
    S.p0[0] = S.mc[0] * iz; S.p0[1] = S.mc[1] * iz; S.p0[2] = F(1);
    S.A = F(0);
    for (int k = 0; k < 3; ++k) {
        S.wv[k] = S.M[k] * S.p0[0] + S.M[3 + k] * S.p0[1] + S.M[6 + k];
        S.A += S.wv[k] * S.wv[k] * G.is2[k];
    }
    S.iA = F(1) / S.A;
    S.Qp0x = S.Qp0y = S.Q00 = S.Q01 = S.Q11 = F(0);
    for (int k = 0; k < 3; ++k) {
        F e = S.wv[k] * G.is2[k];
        S.Qp0x += S.M[k] * e;
        S.Qp0y += S.M[3 + k] * e;
        S.Q00 += S.M[k] * S.M[k] * G.is2[k];
        S.Q01 += S.M[k] * S.M[3 + k] * G.is2[k];
        S.Q11 += S.M[3 + k] * S.M[3 + k] * G.is2[k];
    }
}

template <int DEG>
__global__ void __launch_bounds__(kProjThreads) project_fwd_kernel(ugs_gaussians g, const DevCam *__restrict__ cams,
                                                                   int V, int tile_w, int tile_h, float prune_Tk,
                                                                   float4 *__restrict__ rec, uint2 *__restrict__ rect,
                                                                   uint32_t *__restrict__ touched,
                                                                   float4 *__restrict__ grec, int zero_grad,
                                                                   float *__restrict__ hrec,
                                                                   uint32_t *__restrict__ zbits)
{
    const int64_t N = g.N;
    const int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
    if (i >= N) return;
    constexpr int NC = (DEG + 1) * (DEG + 1);
    // FP64 here: the 2D covariance of a thin splat is nearly singular, so its
    // inverse and the depth coefficients need the extra precision; the record
    // is rounded to FP32 once.
    using D = double;
    GaussState<D> G;
    load_gauss(g, i, G);
    const bool alive = G.o >= D(kAlphaMin) && !(prune_Tk > 0.f && fabs(G.k - D(1)) > D(prune_Tk));
    float sh[NC][3];
    if (alive)
        for (int c = 0; c < NC; ++c)
            for (int ch = 0; ch < 3; ++ch) sh[c][ch] = g.sh[((int64_t)c * 3 + ch) * N + i];
    const D r2 = alive ? D(2) * log(D(255) * G.o) : D(0);
    for (int v = 0; v < V; ++v) {
        const DevCam &cam = cams[v];
        const int64_t idx = (int64_t)v * N + i;
        uint32_t nt = 0;
        uint2 rc = make_uint2(0, 0);
        const D zc = D(cam.R[6]) * G.mu[0] + D(cam.R[7]) * G.mu[1] + D(cam.R[8]) * G.mu[2] + D(cam.t[2]);
        if (alive && zc > D(cam.z_near)) {
            ViewState<D> S;
            project_view(G, cam, S);
            const D rx = sqrt(S.cov00 * r2) * D(1.0001) + D(1e-3);
            const D ry = sqrt(S.cov11 * r2) * D(1.0001) + D(1e-3);
            const D u0 = fmax(ceil(S.m2x - rx), D(0)), u1 = fmin(floor(S.m2x + rx), D(cam.W - 1));
            const D v0 = fmax(ceil(S.m2y - ry), D(0)), v1 = fmin(floor(S.m2y + ry), D(cam.H - 1));
            if (u0 <= u1 && v0 <= v1 && isfinite(S.m2x) && isfinite(S.m2y)) {
                const int tx0 = (int)u0 / tile_w, tx1 = (int)u1 / tile_w + 1;
                const int ty0 = (int)v0 / tile_h, ty1 = (int)v1 / tile_h + 1;
                const int area = (tx1 - tx0) * (ty1 - ty0);
                rc = make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16));
                D Y[NC];
                sh_basis<DEG>(S.dir[0], S.dir[1], S.dir[2], Y);
                float col[3];
                for (int ch = 0; ch < 3; ++ch) {
                    D acc = D(0.5);
                    for (int c = 0; c < NC; ++c) acc += Y[c] * D(sh[c][ch]);
                    col[ch] = (float)fmax(acc, D(0));
                }
                // Cholesky factor of the conic (inverse 2D covariance): the
                // exponent becomes a sum of two squares per fragment
                const D det = S.cov00 * S.cov11 - S.cov01 * S.cov01;
                const D l11 = sqrt(S.cov11 / det), l21 = -S.cov01 / (det * l11), l22 = D(1) / sqrt(S.cov11);
                const D iA = S.iA, fx = D(cam.fx), fy = D(cam.fy);
                float4 *r = rec + idx * 4;
                const float4 q0 = make_float4((float)S.m2x, (float)S.m2y, (float)l11, (float)l21);
                const float4 q1 = make_float4((float)l22, (float)G.o, (float)G.k, (float)S.z);
                r[0] = q0;
                r[1] = q1;
                zbits[idx] = __float_as_uint(q1.w);  // depth key bits for the binning's compaction
                r[2] = make_float4((float)(S.Qp0x * iA / fx), (float)(S.Qp0y * iA / fy), (float)(S.Q00 * iA / (fx * fx)),
                                   (float)(S.Q01 * iA / (fx * fy)));
                r[3] = make_float4((float)(S.Q11 * iA / (fy * fy)), col[0], col[1], col[2]);
                // hit constant of depth_mode 2: the Mahalanobis distance of the
                // camera centre, z0^2 p0^T Q p0
                if (hrec) hrec[idx] = (float)(S.z * S.z * S.A);
                // every tile of the rectangle, for now: the binning pass culls
                // the tiles that the alpha ellipse misses
                nt = (uint32_t)area;
                if (zero_grad) {
                    float4 zf = make_float4(0.f, 0.f, 0.f, 0.f);
                    float4 *gr = grec + idx * 4;
                    gr[0] = zf; gr[1] = zf; gr[2] = zf; gr[3] = zf;
                }
            }
        }
        touched[idx] = nt;
        rect[idx] = rc;
    }
}

// Backward of the per-view records into the Gaussian parameters, in two
// passes.  The first runs the whole chain rule once per visible (view,
// Gaussian) record -- one thread per record of the (Gaussian, view)-ordered
// visible list, so no lane idles on views where its Gaussian is not visible and
// neighbouring lanes read the same or neighbouring parameters -- and writes the
// record's contributions to the parameter gradients back into its gradient
// record: mean 0-2, quaternion 3-6, log-scale 7-9, opacity logit 10, mask logit
// 11 and the clamped colour gradient 12-14 (the SH coefficients' share is
// Y(dir) times it).  The chain is linear in the record gradients, so applying
// it per view and summing equals summing first.  The second pass sums the
// contributions of each Gaussian's visible views and forms the SH gradients.
template <int DEG>
__global__ void __launch_bounds__(kProjThreads) project_bwd_rec_kernel(ugs_gaussians g, const DevCam *__restrict__ cams,
                                                                       const uint32_t *__restrict__ didx,
                                                                       const DevCounters *__restrict__ cnt,
                                                                       const uint32_t *__restrict__ touched,
                                                                       float4 *__restrict__ grec)
{
    const int64_t N = g.N;
    constexpr int NC = (DEG + 1) * (DEG + 1);
    using D = double;  // the chain rule runs in FP64: its terms scale like 1/s^2 and cancel
    // the list holds exactly the records still touched after the binning walk,
    // which sets a record's count to its kept tiles (0 when the ellipse cull
    // drops them all): R_gauss <= R, and no entry needs its count re-checked
    const uint32_t Rn = cnt->R_gauss;
    (void)touched;
    for (uint64_t rr = (uint64_t)blockIdx.x * kProjThreads + threadIdx.x; rr < Rn;
         rr += (uint64_t)gridDim.x * kProjThreads) {
        const uint32_t idx = didx[rr];
        const int v = (int)(idx / (uint64_t)N);
        const int64_t i = (int64_t)idx - (int64_t)v * N;
        GaussState<D> G;
        load_gauss(g, i, G);
        D dmu[3] = {D(0), D(0), D(0)}, dRg[9], ds[3] = {D(0), D(0), D(0)}, dSig[6], dis2[3] = {D(0), D(0), D(0)};
        for (int k = 0; k < 9; ++k) dRg[k] = D(0);
        for (int k = 0; k < 6; ++k) dSig[k] = D(0);
        D dop = D(0), dk = D(0);
        float sh[NC][3], dcs[3] = {0.f, 0.f, 0.f};
        for (int c = 0; c < NC; ++c)
            for (int ch = 0; ch < 3; ++ch) sh[c][ch] = g.sh[((int64_t)c * 3 + ch) * N + i];
        const DevCam &cam = cams[v];
        const float4 *gin = grec + (int64_t)idx * 4;
        float4 g0 = gin[0], g1 = gin[1], g2 = gin[2], g3 = gin[3];
        ViewState<D> S;
        project_view(G, cam, S);
        D R[9];
        for (int k = 0; k < 9; ++k) R[k] = D(cam.R[k]);
        const D fx = D(cam.fx), fy = D(cam.fy), z = S.z, iz = D(1) / z;
        dop += g1.y;
        dk += g1.z;
        D dmc[3] = {D(0), D(0), D(0)};

        // colour (SH) and the view direction
        {
            D Y[NC];
            sh_basis<DEG>(S.dir[0], S.dir[1], S.dir[2], Y);
            D dcol[3] = {g3.y, g3.z, g3.w};
            D ddx = D(0), ddy = D(0), ddz = D(0);
            for (int ch = 0; ch < 3; ++ch) {
                D raw = D(0.5);
                for (int c = 0; c < NC; ++c) raw += Y[c] * sh[c][ch];
                D dc = raw > D(0) ? dcol[ch] : D(0);
                dcs[ch] = (float)dc;
                if (dc == D(0)) continue;
                D w[NC];
                for (int c = 0; c < NC; ++c) {
                    w[c] = dc * sh[c][ch];
                }
                D gx, gy, gz;
                sh_basis_vjp<DEG>(S.dir[0], S.dir[1], S.dir[2], w, gx, gy, gz);
                ddx += gx; ddy += gy; ddz += gz;
            }
            D pr = S.dir[0] * ddx + S.dir[1] * ddy + S.dir[2] * ddz;
            D id = D(1) / S.dist;
            dmu[0] += (ddx - S.dir[0] * pr) * id;
            dmu[1] += (ddy - S.dir[1] * pr) * id;
            dmu[2] += (ddz - S.dir[2] * pr) * id;
        }
        // 2D mean
        dmc[0] += g0.x * fx * iz;
        dmc[1] += g0.y * fy * iz;
        dmc[2] -= (g0.x * fx * S.mc[0] + g0.y * fy * S.mc[1]) * iz * iz;
        // Cholesky factor of the conic -> 2D covariance (entries s00, s01, s11):
        //   l11 = sqrt(s11 / det), l21 = -s01 / (det l11), l22 = 1 / sqrt(s11),
        //   det = s00 s11 - s01^2.
        {
            const D s00 = S.cov00, s01 = S.cov01, s11 = S.cov11;
            const D det = s00 * s11 - s01 * s01;
            const D l11 = sqrt(s11 / det), l21 = -s01 / (det * l11), l22 = D(1) / sqrt(s11);
            const D dl11 = g0.z, dl21 = g0.w, dl22 = g1.x;
            // partials of det and of l11
            const D ddet[3] = {s11, D(-2) * s01, s00};
            const D dl11_[3] = {D(-0.5) * l11 * s11 / det, l11 * s01 / det, D(0.5) * l11 * (D(1) / s11 - s00 / det)};
            // l21 = -s01 / u with u = det * l11
            const D u = det * l11;
            D dP[3];  // gradient wrt the parameters (s00, s01, s11)
            for (int q = 0; q < 3; ++q) {
                const D du = ddet[q] * l11 + det * dl11_[q];
                const D dl21_q = -(q == 1 ? D(1) : D(0)) / u + s01 * du / (u * u);
                const D dl22_q = q == 2 ? D(-0.5) * l22 / s11 : D(0);
                dP[q] = dl11 * dl11_[q] + dl21 * dl21_q + dl22 * dl22_q;
            }
            // full-entry symmetric gradient of the 2D covariance matrix
            const D dS00 = dP[0], dS01 = D(0.5) * dP[1], dS11 = dP[2];
            // cov = T Sig T^T: dSig += T^T dS T, dT = 2 dS T Sig
            const D *t0 = S.T0, *t1 = S.T1;
            for (int p = 0, n = 0; p < 3; ++p)
                for (int q = p; q < 3; ++q, ++n) {
                    D val = t0[p] * dS00 * t0[q] + t0[p] * dS01 * t1[q] + t1[p] * dS01 * t0[q] + t1[p] * dS11 * t1[q];
                    dSig[n] += val;
                }
            const D *Sg = G.Sig;
            D TS0[3], TS1[3];
            TS0[0] = t0[0] * Sg[0] + t0[1] * Sg[1] + t0[2] * Sg[2];
            TS0[1] = t0[0] * Sg[1] + t0[1] * Sg[3] + t0[2] * Sg[4];
            TS0[2] = t0[0] * Sg[2] + t0[1] * Sg[4] + t0[2] * Sg[5];
            TS1[0] = t1[0] * Sg[0] + t1[1] * Sg[1] + t1[2] * Sg[2];
            TS1[1] = t1[0] * Sg[1] + t1[1] * Sg[3] + t1[2] * Sg[4];
            TS1[2] = t1[0] * Sg[2] + t1[1] * Sg[4] + t1[2] * Sg[5];
            D dT0[3], dT1[3];
            for (int q = 0; q < 3; ++q) {
                dT0[q] = D(2) * (dS00 * TS0[q] + dS01 * TS1[q]);
                dT1[q] = D(2) * (dS01 * TS0[q] + dS11 * TS1[q]);
            }
            // T0 = J00 R0 + J02 R2, T1 = J11 R1 + J12 R2
            D dJ00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
            D dJ02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
            D dJ11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
            D dJ12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
            D iz2 = iz * iz, iz3 = iz2 * iz;
            dmc[2] += -dJ00 * fx * iz2 - dJ11 * fy * iz2 + D(2) * dJ02 * fx * S.tx * iz3 + D(2) * dJ12 * fy * S.ty * iz3;
            D dtx = -dJ02 * fx * iz2, dty = -dJ12 * fy * iz2;
            if (!S.clx) dmc[0] += dtx; else dmc[2] += dtx * S.tx * iz;
            if (!S.cly) dmc[1] += dty; else dmc[2] += dty * S.ty * iz;
        }
        // depth coefficients: beta = (Qp0)_xy / (A f), gam = Q_xy / (A f f), z0 = mc.z
        {
            D iA = S.iA;
            D bx = S.Qp0x * iA / fx, by = S.Qp0y * iA / fy;
            D gA = S.Q00 * iA / (fx * fx), gB = S.Q01 * iA / (fx * fy), gC = S.Q11 * iA / (fy * fy);
            D dbx = g2.x, dby = g2.y, dgA = g2.z, dgB = g2.w, dgC = g3.x;
            D dA = -iA * (dbx * bx + dby * by + dgA * gA + dgB * gB + dgC * gC);
            D dQpx = dbx * iA / fx, dQpy = dby * iA / fy;
            D dQ00 = dgA * iA / (fx * fx), dQ01 = dgB * iA / (fx * fy), dQ11 = dgC * iA / (fy * fy);
            D dM[9];
            for (int k = 0; k < 9; ++k) dM[k] = D(0);
            D dwv[3];
            const D *M = S.M;
            for (int k = 0; k < 3; ++k) {
                D e = G.is2[k], w = S.wv[k];
                // A = sum_k wv_k^2 is2_k
                dwv[k] = D(2) * dA * w * e;
                dis2[k] += dA * w * w;
                // Qp0_a = sum_k M_ak wv_k is2_k  (a = 0, 1)
                D t = dQpx * M[k] + dQpy * M[3 + k];
                dM[k] += dQpx * w * e;
                dM[3 + k] += dQpy * w * e;
                dwv[k] += t * e;
                dis2[k] += t * w;
                // Q00, Q01, Q11
                dM[k] += D(2) * dQ00 * M[k] * e + dQ01 * M[3 + k] * e;
                dM[3 + k] += D(2) * dQ11 * M[3 + k] * e + dQ01 * M[k] * e;
                dis2[k] += dQ00 * M[k] * M[k] + dQ01 * M[k] * M[3 + k] + dQ11 * M[3 + k] * M[3 + k];
            }
            // wv_k = sum_a M_ak p0_a
            D dp0[2] = {D(0), D(0)};
            for (int k = 0; k < 3; ++k) {
                dM[k] += dwv[k] * S.p0[0];
                dM[3 + k] += dwv[k] * S.p0[1];
                dM[6 + k] += dwv[k];
                dp0[0] += dwv[k] * M[k];
                dp0[1] += dwv[k] * M[3 + k];
            }
            dmc[0] += dp0[0] * iz;
            dmc[1] += dp0[1] * iz;
            dmc[2] += g1.w - (dp0[0] * S.mc[0] + dp0[1] * S.mc[1]) * iz * iz;
            // M = R Rg  ->  dRg = R^T dM
            for (int b = 0; b < 3; ++b)
                for (int k = 0; k < 3; ++k) dRg[3 * b + k] += R[b] * dM[k] + R[3 + b] * dM[3 + k] + R[6 + b] * dM[6 + k];
        }
        // mc = R mu + t
        for (int e = 0; e < 3; ++e) dmu[e] += R[e] * dmc[0] + R[3 + e] * dmc[1] + R[6 + e] * dmc[2];
        {
        // Sig = Rg S^2 Rg^T: with Mg = Rg S, dMg = 2 dSig Mg (full symmetric dSig)
        {
            D dS3[9] = {dSig[0], dSig[1], dSig[2], dSig[1], dSig[3], dSig[4], dSig[2], dSig[4], dSig[5]};
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    D acc = D(0);
                    for (int k = 0; k < 3; ++k) acc += dS3[3 * r + k] * G.Rg[3 * k + q];
                    D dMg = D(2) * acc * G.s[q];
                    dRg[3 * r + q] += dMg * G.s[q];
                    ds[q] += G.Rg[3 * r + q] * dMg;
                }
        }
        for (int k = 0; k < 3; ++k) ds[k] += dis2[k] * (-D(2)) * G.is2[k] / G.s[k];
        // rotation matrix -> unit quaternion -> quaternion
        D w = G.qh[0], x = G.qh[1], y = G.qh[2], z = G.qh[3];
        const D *d = dRg;
        D gw = D(2) * (-z * d[1] + y * d[2] + z * d[3] - x * d[5] - y * d[6] + x * d[7]);
        D gx = D(2) * (y * d[1] + z * d[2] + y * d[3] - D(2) * x * d[4] - w * d[5] + z * d[6] + w * d[7] - D(2) * x * d[8]);
        D gy = D(2) * (-D(2) * y * d[0] + x * d[1] + w * d[2] + x * d[3] + z * d[5] - w * d[6] + z * d[7] - D(2) * y * d[8]);
        D gz = D(2) * (-D(2) * z * d[0] - w * d[1] + x * d[2] + w * d[3] - D(2) * z * d[4] + y * d[5] + x * d[6] + y * d[7]);
        D pq = gw * w + gx * x + gy * y + gz * z;
        D iq = D(1) / G.qn;
        float4 *gr = grec + (int64_t)idx * 4;
        gr[0] = make_float4((float)dmu[0], (float)dmu[1], (float)dmu[2], (float)((gw - w * pq) * iq));
        gr[1] = make_float4((float)((gx - x * pq) * iq), (float)((gy - y * pq) * iq), (float)((gz - z * pq) * iq),
                            (float)(ds[0] * G.s[0]));
        gr[2] = make_float4((float)(ds[1] * G.s[1]), (float)(ds[2] * G.s[2]), (float)(dop * G.o * (D(1) - G.o)),
                            (float)(dk * G.k * (D(1) - G.k)));
        gr[3] = make_float4(dcs[0], dcs[1], dcs[2], 0.f);
        }
    }
}

// Second pass: per Gaussian, the sum over its visible views of the record
// contributions, and the SH gradients Y(dir_v) times the clamped colour
// gradient of each view (Y in FP64, as in the projection).
template <int DEG>
__global__ void __launch_bounds__(kProjThreads) project_bwd_sum_kernel(ugs_gaussians g, const DevCam *__restrict__ cams,
                                                                       int V, const uint32_t *__restrict__ touched,
                                                                       const float4 *__restrict__ grec,
                                                                       ugs_gaussian_grads dg)
{
    const int64_t N = g.N;
    const int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
    if (i >= N) return;
    constexpr int NC = (DEG + 1) * (DEG + 1);
    using D = double;
    D acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = D(0);
    float dsh[NC][3];
    for (int c = 0; c < NC; ++c)
        for (int ch = 0; ch < 3; ++ch) dsh[c][ch] = 0.f;
    // The views that see this Gaussian (V <= 64): their flags are loaded
    // without a branch between them, instead of a flag, a branch and a record
    // per view in one dependent chain.
    uint64_t vis = 0;
#pragma unroll 8
    for (int v = 0; v < V; ++v) vis |= (uint64_t)(touched[(int64_t)v * N + i] != 0u) << v;
    if (!vis) return;
    const D mu[3] = {D(g.mean[i]), D(g.mean[N + i]), D(g.mean[2 * N + i])};
    while (vis) {
        const int v = __builtin_ctzll(vis);
        vis &= vis - 1ull;
        const float4 *gr = grec + ((int64_t)v * N + i) * 4;
        const float4 a = gr[0], b = gr[1], c2 = gr[2], d3 = gr[3];
        const float f[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c2.x, c2.y, c2.z, c2.w};
        for (int k = 0; k < 12; ++k) acc[k] += D(f[k]);
        const DevCam &cam = cams[v];
        const D v0 = mu[0] - D(cam.C[0]), v1 = mu[1] - D(cam.C[1]), v2 = mu[2] - D(cam.C[2]);
        const D id = D(1) / m_sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        D Y[NC];
        sh_basis<DEG>(v0 * id, v1 * id, v2 * id, Y);
        const D dc[3] = {D(d3.x), D(d3.y), D(d3.z)};
        for (int ch = 0; ch < 3; ++ch) {
            if (dc[ch] == D(0)) continue;
            for (int c = 0; c < NC; ++c) dsh[c][ch] += dc[ch] * Y[c];
        }
    }
    for (int e = 0; e < 3; ++e) dg.mean[e * N + i] += acc[e];
    for (int e = 0; e < 4; ++e) dg.quat[e * N + i] += acc[3 + e];
    for (int e = 0; e < 3; ++e) dg.log_scale[e * N + i] += acc[7 + e];
    dg.opacity_logit[i] += acc[10];
    dg.mask_logit[i] += acc[11];
    for (int c = 0; c < NC; ++c)
        for (int ch = 0; ch < 3; ++ch) dg.sh[((int64_t)c * 3 + ch) * N + i] += dsh[c][ch];
}

}  // namespace

hipError_t launch_project_fwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws, bool zero_grad,
                              hipStream_t s)
{
    if (g.N == 0) return hipSuccess;
    dim3 grid((unsigned)((g.N + kProjThreads - 1) / kProjThreads));
    auto cams = (const DevCam *)(ws + L.cams);
    auto rec = (float4 *)(ws + L.rec);
    auto rect = (uint2 *)(ws + L.rect);
    auto touched = (uint32_t *)(ws + L.touched);
    auto grec = (float4 *)(ws + L.grec);
    auto hrec = pb.depth_mode == 2 ? (float *)(ws + L.hrec) : nullptr;
    auto zbits = (uint32_t *)(ws + L.dkey1);  // free until the binning's depth sort
    switch (g.sh_deg) {
    case 0: hipLaunchKernelGGL(project_fwd_kernel<0>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, pb.tile_w, pb.tile_h, pb.prune_Tk, rec, rect, touched, grec, (int)zero_grad, hrec, zbits); break;
    case 1: hipLaunchKernelGGL(project_fwd_kernel<1>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, pb.tile_w, pb.tile_h, pb.prune_Tk, rec, rect, touched, grec, (int)zero_grad, hrec, zbits); break;
    case 2: hipLaunchKernelGGL(project_fwd_kernel<2>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, pb.tile_w, pb.tile_h, pb.prune_Tk, rec, rect, touched, grec, (int)zero_grad, hrec, zbits); break;
    default: hipLaunchKernelGGL(project_fwd_kernel<3>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, pb.tile_w, pb.tile_h, pb.prune_Tk, rec, rect, touched, grec, (int)zero_grad, hrec, zbits); break;
    }
    return hipGetLastError();
}

hipError_t launch_project_bwd(const ugs_gaussians &g, const Problem &pb, const WsLayout &L, char *ws,
                              const ugs_gaussian_grads &dg, hipStream_t s)
{
    if (g.N == 0) return hipSuccess;
    auto cams = (const DevCam *)(ws + L.cams);
    auto touched = (const uint32_t *)(ws + L.touched);
    auto grec = (float4 *)(ws + L.grec);
    auto cnt = (const DevCounters *)(ws + L.counters);
    // visible records in (Gaussian, view) order: a wavefront's records belong
    // to a few consecutive Gaussians, so the parameter loads coalesce (in
    // index order, a view's visible Gaussians are sparse and every parameter
    // row read pulled in several cache lines per wavefront)
    hipError_t e = launch_gauss_major_list(L, ws, pb.V, s);
    if (e != hipSuccess) return e;
    auto didx = (const uint32_t *)(ws + L.vlist);
    const int64_t VN = L.VN;
    const unsigned rec_blocks = (unsigned)std::min<int64_t>(std::max<int64_t>((VN + kProjThreads - 1) / kProjThreads, 1), 8192);
    dim3 grid((unsigned)((g.N + kProjThreads - 1) / kProjThreads));
    switch (g.sh_deg) {
    case 0:
        hipLaunchKernelGGL(project_bwd_rec_kernel<0>, dim3(rec_blocks), dim3(kProjThreads), 0, s, g, cams, didx, cnt, touched, grec);
        hipLaunchKernelGGL(project_bwd_sum_kernel<0>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, touched, (const float4 *)grec, dg);
        break;
    case 1:
        hipLaunchKernelGGL(project_bwd_rec_kernel<1>, dim3(rec_blocks), dim3(kProjThreads), 0, s, g, cams, didx, cnt, touched, grec);
        hipLaunchKernelGGL(project_bwd_sum_kernel<1>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, touched, (const float4 *)grec, dg);
        break;
    case 2:
        hipLaunchKernelGGL(project_bwd_rec_kernel<2>, dim3(rec_blocks), dim3(kProjThreads), 0, s, g, cams, didx, cnt, touched, grec);
        hipLaunchKernelGGL(project_bwd_sum_kernel<2>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, touched, (const float4 *)grec, dg);
        break;
    default:
        hipLaunchKernelGGL(project_bwd_rec_kernel<3>, dim3(rec_blocks), dim3(kProjThreads), 0, s, g, cams, didx, cnt, touched, grec);
        hipLaunchKernelGGL(project_bwd_sum_kernel<3>, grid, dim3(kProjThreads), 0, s, g, cams, pb.V, touched, (const float4 *)grec, dg);
        break;
    }
    return hipGetLastError();
}

}  // namespace ugs
