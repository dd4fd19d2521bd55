/*
 * oracle.c -- plain FP64 CPU reference of the UniGS multimodal Gaussian
 * rasterizer, forward and backward.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the benchmark's
 * CPU baseline can compare the HIP implementation against an independent,
 * obviously correct definition.  It shares no code, header, table or constant
 * with the GPU sources.
 *
 * Everything is double precision, compiled without fast-math.  The forward
 * follows the paper's definitions literally (UniGS, arXiv 2510.12174):
 *   - ray per pixel, Eq. (computeRay), section 3.2, with r(t) = C + t d;
 *   - transform into the ellipsoid's local scaled frame and the unit-sphere
 *     quadratic, section 3.2 and supplementary S1.1 (coefficients a, b, c);
 *   - midpoint depth t_mid = -b / 2a and the camera-frame z of C + t_mid d,
 *     Eq. (midpoint), taken for every fragment, hit or miss (depth_mode 0);
 *     depth_mode 1 takes the centre's camera depth, depth_mode 2 the midpoint
 *     where the quadratic has a real root and the centre depth elsewhere;
 *   - alpha-blended depth, gradient-factor and semantic maps, Eq.
 *     (depth_render), Eq. (t_render), Eq. (semantic_render), Alg. forward_render,
 *     front to back in the order of the per-Gaussian sort key of the tile-based
 *     rasterizer (section 3.4): the camera depth of the centre, computed in FP64
 *     from the FP32 inputs and rounded to FP32 (the depth key of 3DGS's
 *     (tile, depth) sort), ties going to the lower Gaussian index;
 *   - normals from depth, Alg. normal_estimation with the back-projection and
 *     view-facing flip of supplementary S1.3.
 * The splatting part the paper inherits from 3DGS (EWA projection with a
 * 0.3 px low-pass, FOV-clamped Jacobian, alpha cut-off 1/255, clamp 0.99,
 * termination below T = 1e-4, SH colour + 0.5 clamped at 0) uses those
 * published constants.
 *
 * The backward is hand-written reverse mode:
 *   - normals -> depth: Alg. normal_gradient (supplementary S1.4) with the
 *     exact cross-product adjoints;
 *   - compositing: Alg. backward_render (supplementary S1.6), including the
 *     alpha path of every channel;
 *   - depth -> (mu, s, R): supplementary S1.2, Eqs. (d->tmid), (tmid->abc),
 *     (abc->vs), (tmid->vs), (vs->s), (vs->mu), (vs->r);
 *   - R -> q through q/|q| (tangent projection on S^3);
 *   - EWA and SH adjoints for colour, conic and 2D mean.
 * Discrete decisions (fragment sets, termination, culling, flips, clamps) are
 * held fixed; the derivative through an active clamp is zero.
 *
 * A decision-margin report (smallest relative distance of any discrete test
 * from its threshold) accompanies every forward quantity so that tests can
 * exclude pixels whose outcome a rounding difference could flip.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_STOP 1e-4
#define LOWPASS 0.3
#define FOV_CLAMP 1.3
#define MAX_FRAG 8192

typedef struct {
    int W, H;
    double fx, fy, cx, cy;
    double R[9]; /* world -> camera, row-major */
    double t[3];
    double z_near;
} orc_cam;

typedef struct {
    int64_t N;
    int sh_deg, C_o;
    const double *mean;          /* [3][N] */
    const double *quat;          /* [4][N] (w,x,y,z) */
    const double *log_scale;     /* [3][N] */
    const double *opacity_logit; /* [N] */
    const double *mask_logit;    /* [N] */
    const double *sh;            /* [(deg+1)^2][3][N] */
    const double *sem;           /* [N][C_o] */
} orc_gs;

typedef struct {
    int step1, step2;
    double lambda;
    int orient_sign;
    double prune_Tk; /* <= 0 disables the pruning skip */
    double eps_n;
    int depth_mode;  /* 0: ray-ellipsoid midpoint depth (section 3.2); 1: the
                        Gaussian centre's camera depth (the "Center Point" row of
                        the supplementary's module ablation table); 2: the
                        midpoint where the ray meets the ellipsoid (two real
                        roots or one, discriminant >= 0) and the centre depth
                        where it has no valid solution */
} orc_opt;

/* Per-Gaussian projected state for one view. */
typedef struct {
    int visible;
    int ambiguous; /* a cull test lies within 1e-5 (relative) of its threshold */
    double s[3], qn, qh[4], Rg[9], Sig[9];
    double o, k;
    double mc[3];
    double xcl, ycl;
    int clx, cly;
    double Tm[6]; /* J R, 2x3 */
    double cov[3], conic[3];
    double m2[2];
    double dir[3], dist;
    double Y[16], dY[16][3];
    double raw[3], rgb[3];
    double z;
    float zkey;     /* the sort key: the camera depth rounded to FP32 */
    double zmargin; /* margin of that rounding (common 1e-5 scale) */
    double rx, ry; /* pixel half-widths of the alpha >= 1/255 region */
} proj_t;

typedef struct {
    int64_t id;
    double alpha, T, w, G, d;
    int clamped;
} frag_t;

typedef struct {
    const orc_gs *g;
    const orc_cam *cam;
    const orc_opt *opt;
    double C[3];
    proj_t *P;
    int64_t *order;
    int64_t n_vis;
    int path; /* 0: every visible Gaussian per pixel; 1: row lists filtered by the alpha box */
    int64_t *row_start, *row_items;
} ctx_t;

static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

/* ---------------------------------------------------------------- SH basis */
/* Real spherical harmonics up to degree 3 with the Condon-Shortley phase, in the
 * ordering used by 3DGS (the colour model the paper inherits).  Normalisation
 * constants are written from their closed forms.  dY holds the gradient of each
 * polynomial with respect to the (unit) direction components. */
void orc_sh_basis(int deg, const double *d, double *Y, double *dY)
{
    const double pi = 3.14159265358979323846;
    const double sp = sqrt(pi);
    const double k0 = 1.0 / (2.0 * sp);
    const double k1 = sqrt(3.0) / (2.0 * sp);
    const double k2a = sqrt(15.0) / (2.0 * sp);
    const double k2b = sqrt(5.0) / (4.0 * sp);
    const double k2c = sqrt(15.0) / (4.0 * sp);
    const double k3a = sqrt(35.0 / (2.0 * pi)) / 4.0;
    const double k3b = sqrt(105.0 / pi) / 2.0;
    const double k3c = sqrt(21.0 / (2.0 * pi)) / 4.0;
    const double k3d = sqrt(7.0 / pi) / 4.0;
    const double k3e = sqrt(105.0 / pi) / 4.0;
    double x = d[0], y = d[1], z = d[2];
    double xx = x * x, yy = y * y, zz = z * z;
    for (int i = 0; i < 16 * 3; ++i) dY[i] = 0.0;
    for (int i = 0; i < 16; ++i) Y[i] = 0.0;
#define DY(i, a, b, c) (dY[3 * (i)] = (a), dY[3 * (i) + 1] = (b), dY[3 * (i) + 2] = (c))
    Y[0] = k0;
    if (deg < 1) return;
    Y[1] = -k1 * y; DY(1, 0, -k1, 0);
    Y[2] = k1 * z;  DY(2, 0, 0, k1);
    Y[3] = -k1 * x; DY(3, -k1, 0, 0);
    if (deg < 2) return;
    Y[4] = k2a * x * y;            DY(4, k2a * y, k2a * x, 0);
    Y[5] = -k2a * y * z;           DY(5, 0, -k2a * z, -k2a * y);
    Y[6] = k2b * (2 * zz - xx - yy); DY(6, -2 * k2b * x, -2 * k2b * y, 4 * k2b * z);
    Y[7] = -k2a * x * z;           DY(7, -k2a * z, 0, -k2a * x);
    Y[8] = k2c * (xx - yy);        DY(8, 2 * k2c * x, -2 * k2c * y, 0);
    if (deg < 3) return;
    Y[9] = -k3a * y * (3 * xx - yy);          DY(9, -6 * k3a * x * y, -k3a * (3 * xx - 3 * yy), 0);
    Y[10] = k3b * x * y * z;                  DY(10, k3b * y * z, k3b * x * z, k3b * x * y);
    Y[11] = -k3c * y * (4 * zz - xx - yy);    DY(11, 2 * k3c * x * y, -k3c * (4 * zz - xx - 3 * yy), -8 * k3c * y * z);
    Y[12] = k3d * z * (2 * zz - 3 * xx - 3 * yy); DY(12, -6 * k3d * x * z, -6 * k3d * y * z, k3d * (6 * zz - 3 * xx - 3 * yy));
    Y[13] = -k3c * x * (4 * zz - xx - yy);    DY(13, -k3c * (4 * zz - 3 * xx - yy), 2 * k3c * x * y, -8 * k3c * x * z);
    Y[14] = k3e * z * (xx - yy);              DY(14, 2 * k3e * x * z, -2 * k3e * y * z, k3e * (xx - yy));
    Y[15] = -k3a * x * (xx - 3 * yy);         DY(15, -k3a * (3 * xx - 3 * yy), 6 * k3a * x * y, 0);
#undef DY
}

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_rot(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Vector-Jacobian product of quat_rot: dR (row-major) -> dq. */
static void quat_rot_vjp(const double *q, const double *dR, double *dq)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2 * x * dR[8]);
    dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2 * y * dR[8]);
    dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
}

static void cam_centre(const orc_cam *c, double *C)
{
    for (int i = 0; i < 3; ++i)
        C[i] = -(c->R[0 + i] * c->t[0] + c->R[3 + i] * c->t[1] + c->R[6 + i] * c->t[2]);
}

static double relmargin(double x, double thr) { return fabs(x - thr) / fabs(thr); }

/* ---------------------------------------------------------------- projection */
static void project_one(const orc_gs *g, const orc_cam *cam, const orc_opt *opt,
                        const double *C, int64_t i, proj_t *P)
{
    const int64_t N = g->N;
    const double *R = cam->R;
    double mu[3] = {g->mean[i], g->mean[N + i], g->mean[2 * N + i]};
    for (int k = 0; k < 3; ++k) P->s[k] = exp(g->log_scale[k * N + i]);
    double q[4], qn = 0;
    for (int k = 0; k < 4; ++k) { q[k] = g->quat[k * N + i]; qn += q[k] * q[k]; }
    qn = sqrt(qn);
    P->qn = qn;
    for (int k = 0; k < 4; ++k) P->qh[k] = q[k] / qn;
    quat_rot(P->qh, P->Rg);
    /* Sigma = Rg diag(s^2) Rg^T */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += P->Rg[3 * a + k] * P->s[k] * P->s[k] * P->Rg[3 * b + k];
            P->Sig[3 * a + b] = acc;
        }
    P->o = sigm(g->opacity_logit[i]);
    P->k = sigm(g->mask_logit[i]);
    for (int a = 0; a < 3; ++a) P->mc[a] = R[3 * a] * mu[0] + R[3 * a + 1] * mu[1] + R[3 * a + 2] * mu[2] + cam->t[a];
    P->z = P->mc[2];
    P->zkey = (float)P->z;
    {
        /* The FP32 key is the rounding of mu_c.z = R_3 . mu + t_z.  With FP32
         * inputs the three products are exact in FP64, so the only rounding is
         * in the additions: when the left-to-right sum is exact (every TwoSum
         * residual zero) the key is the rounding of the exact depth and nothing
         * is ambiguous; otherwise the key is ambiguous only if z lies within the
         * summation error bound (4 eps sum |terms|) of a midpoint between two
         * FP32 values.  The distance is mapped onto the common 1e-5 margin scale. */
        double terms[4] = {R[6] * mu[0], R[7] * mu[1], R[8] * mu[2], cam->t[2]};
        double s = terms[0], resid = 0.0, mag = fabs(terms[0]);
        for (int k = 1; k < 4; ++k) {
            double t = s + terms[k], bb = t - s;
            resid += fabs((s - (t - bb)) + (terms[k] - bb));
            s = t;
            mag += fabs(terms[k]);
        }
        double up = (double)nextafterf(P->zkey, INFINITY), dn = (double)nextafterf(P->zkey, -INFINITY);
        double dm = fmin(fabs(P->z - 0.5 * ((double)P->zkey + up)), fabs(P->z - 0.5 * ((double)P->zkey + dn)));
        double bound = 4.0 * 1.1102230246251565e-16 * mag;
        P->zmargin = resid == 0.0 ? INFINITY : 1e-5 * dm / bound;
    }
    int vis = P->mc[2] > cam->z_near;
    int amb = relmargin(P->mc[2], cam->z_near) < 1e-5;
    if (opt->prune_Tk > 0) {
        double dev = fabs(P->k - 1.0);
        if (dev > opt->prune_Tk) vis = 0;
        if (relmargin(dev, opt->prune_Tk) < 1e-5) amb = 1;
    }
    if (P->o < ALPHA_MIN) vis = 0;
    if (relmargin(P->o, ALPHA_MIN) < 1e-5) amb = 1;
    P->visible = vis;
    P->ambiguous = amb;
    if (!(P->mc[2] > 0)) { P->visible = 0; return; }

    /* EWA: Sigma2D = J R Sigma R^T J^T + 0.3 I, J at the FOV-clamped point */
    double z = P->mc[2];
    double limx = FOV_CLAMP * cam->W / (2.0 * cam->fx), limy = FOV_CLAMP * cam->H / (2.0 * cam->fy);
    double tx = P->mc[0] / z, ty = P->mc[1] / z;
    P->clx = (tx < -limx || tx > limx);
    P->cly = (ty < -limy || ty > limy);
    tx = tx < -limx ? -limx : (tx > limx ? limx : tx);
    ty = ty < -limy ? -limy : (ty > limy ? limy : ty);
    P->xcl = tx * z;
    P->ycl = ty * z;
    double J[6] = {cam->fx / z, 0, -cam->fx * P->xcl / (z * z), 0, cam->fy / z, -cam->fy * P->ycl / (z * z)};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            P->Tm[3 * a + b] = J[3 * a] * R[b] + J[3 * a + 1] * R[3 + b] + J[3 * a + 2] * R[6 + b];
    double S2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += P->Tm[3 * a + k] * P->Sig[3 * k + l] * P->Tm[3 * b + l];
            S2[2 * a + b] = acc;
        }
    P->cov[0] = S2[0] + LOWPASS;
    P->cov[1] = 0.5 * (S2[1] + S2[2]);
    P->cov[2] = S2[3] + LOWPASS;
    double det = P->cov[0] * P->cov[2] - P->cov[1] * P->cov[1];
    P->conic[0] = P->cov[2] / det;
    P->conic[1] = -P->cov[1] / det;
    P->conic[2] = P->cov[0] / det;
    P->m2[0] = cam->fx * P->mc[0] / z + cam->cx;
    P->m2[1] = cam->fy * P->mc[1] / z + cam->cy;

    /* colour from SH at the view direction */
    double v[3] = {mu[0] - C[0], mu[1] - C[1], mu[2] - C[2]};
    P->dist = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) P->dir[k] = v[k] / P->dist;
    orc_sh_basis(g->sh_deg, P->dir, P->Y, &P->dY[0][0]);
    int nc = (g->sh_deg + 1) * (g->sh_deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0;
        for (int c = 0; c < nc; ++c) acc += P->Y[c] * g->sh[((int64_t)c * 3 + ch) * N + i];
        P->raw[ch] = acc + 0.5;
        P->rgb[ch] = P->raw[ch] > 0 ? P->raw[ch] : 0.0;
    }
    double r2 = P->o >= ALPHA_MIN ? 2.0 * log(255.0 * P->o) : 0.0;
    P->rx = sqrt(P->cov[0] * r2);
    P->ry = sqrt(P->cov[2] * r2);
}

/* ---------------------------------------------------------------- context */
static const proj_t *g_sort_P;
static int cmp_zid(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    float zi = g_sort_P[i].zkey, zj = g_sort_P[j].zkey;
    if (zi < zj) return -1;
    if (zi > zj) return 1;
    return (i > j) - (i < j);
}

static int ctx_init(ctx_t *c, const orc_gs *g, const orc_cam *cam, const orc_opt *opt, int path)
{
    memset(c, 0, sizeof(*c));
    c->g = g; c->cam = cam; c->opt = opt; c->path = path;
    cam_centre(cam, c->C);
    c->P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(g->N > 0 ? g->N : 1));
    c->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->N > 0 ? g->N : 1));
    if (!c->P || !c->order) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->N; ++i) project_one(g, cam, opt, c->C, i, &c->P[i]);
    int64_t n = 0;
    for (int64_t i = 0; i < g->N; ++i)
        if (c->P[i].visible) c->order[n++] = i;
    c->n_vis = n;
    g_sort_P = c->P;
    qsort(c->order, (size_t)n, sizeof(int64_t), cmp_zid);
    if (path == 1) {
        /* row lists: every visible Gaussian whose alpha box (padded by one pixel)
         * covers row v, kept in (depth, id) order */
        int H = cam->H;
        c->row_start = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
        if (!c->row_start) return -1;
        for (int64_t j = 0; j < n; ++j) {
            const proj_t *P = &c->P[c->order[j]];
            double lo = ceil(P->m2[1] - P->ry - 1.0), hi = floor(P->m2[1] + P->ry + 1.0);
            if (lo < 0) lo = 0;
            if (hi > H - 1) hi = H - 1;
            for (int v = (int)lo; v <= (int)hi; ++v) c->row_start[v + 1]++;
        }
        for (int v = 0; v < H; ++v) c->row_start[v + 1] += c->row_start[v];
        c->row_items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(c->row_start[H] > 0 ? c->row_start[H] : 1));
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
        if (!c->row_items || !fill) return -1;
        for (int v = 0; v < H; ++v) fill[v] = c->row_start[v];
        for (int64_t j = 0; j < n; ++j) {
            int64_t id = c->order[j];
            const proj_t *P = &c->P[id];
            double lo = ceil(P->m2[1] - P->ry - 1.0), hi = floor(P->m2[1] + P->ry + 1.0);
            if (lo < 0) lo = 0;
            if (hi > H - 1) hi = H - 1;
            for (int v = (int)lo; v <= (int)hi; ++v) c->row_items[fill[v]++] = id;
        }
        free(fill);
    }
    return 0;
}

static void ctx_free(ctx_t *c)
{
    free(c->P); free(c->order); free(c->row_start); free(c->row_items);
}

/* ---------------------------------------------------------------- depth */
/* Ray-ellipsoid midpoint depth of Gaussian P at pixel (u,v): Eq. (computeRay),
 * the local scaled frame of section 3.2, a = ds.ds, b = 2 vs.ds,
 * t_mid = -b/(2a), d = z-component in the camera frame of C + t_mid dray. */
typedef struct {
    double dr[3], v[3], vl[3], dl[3], vs[3], ds[3], a, b, c, disc, hmargin, tm, d, dd_dt;
} depth_t;

static void depth_literal(const ctx_t *c, const proj_t *P, const double *mu, double u, double v, depth_t *D)
{
    const orc_cam *cam = c->cam;
    const double *R = cam->R;
    double p[3] = {(u - cam->cx) / cam->fx, (v - cam->cy) / cam->fy, 1.0};
    double n = 0;
    for (int k = 0; k < 3; ++k) {
        D->dr[k] = R[k] * p[0] + R[3 + k] * p[1] + R[6 + k] * p[2];
        n += D->dr[k] * D->dr[k];
    }
    n = sqrt(n);
    for (int k = 0; k < 3; ++k) D->dr[k] /= n;
    for (int k = 0; k < 3; ++k) D->v[k] = c->C[k] - mu[k];
    for (int k = 0; k < 3; ++k) {
        D->vl[k] = P->Rg[k] * D->v[0] + P->Rg[3 + k] * D->v[1] + P->Rg[6 + k] * D->v[2];
        D->dl[k] = P->Rg[k] * D->dr[0] + P->Rg[3 + k] * D->dr[1] + P->Rg[6 + k] * D->dr[2];
        D->vs[k] = D->vl[k] / P->s[k];
        D->ds[k] = D->dl[k] / P->s[k];
    }
    D->a = D->ds[0] * D->ds[0] + D->ds[1] * D->ds[1] + D->ds[2] * D->ds[2];
    D->b = 2.0 * (D->vs[0] * D->ds[0] + D->vs[1] * D->ds[1] + D->vs[2] * D->ds[2]);
    double vv = D->vs[0] * D->vs[0] + D->vs[1] * D->vs[1] + D->vs[2] * D->vs[2];
    D->c = vv - 1.0;
    D->disc = D->b * D->b - 4.0 * D->a * D->c; /* >= 0: the ray meets the ellipsoid */
    D->tm = -D->b / (2.0 * D->a);
    double X[3];
    for (int k = 0; k < 3; ++k) X[k] = c->C[k] + D->tm * D->dr[k];
    D->d = R[6] * X[0] + R[7] * X[1] + R[8] * X[2] + cam->t[2];
    D->dd_dt = R[6] * D->dr[0] + R[7] * D->dr[1] + R[8] * D->dr[2];
    /* Decision margin of the hit test.  disc >= 0 exactly when the smallest
     * squared Mahalanobis distance along the ray, m = |vs|^2 - (vs.ds)^2 / a, is
     * at most 1; the margin is m's relative distance from 1, divided by the
     * cancellation factor of m when it is formed from the pixel's offset delta
     * from the centre's ray p0 (m is proportional to |p0|^2 |delta|^2 -
     * (p0.delta)^2 in the scaled frame). */
    double m = vv - (D->b * D->b) / (4.0 * D->a);
    double p0s[3], dls[3], pp = 0, dd2 = 0, pd = 0;
    for (int k = 0; k < 3; ++k) {
        p0s[k] = -D->vs[k] / P->z;              /* mu_c / z0 in the scaled frame */
        dls[k] = D->ds[k] / D->dd_dt - p0s[k];  /* ray point at camera depth 1, minus p0 */
        pp += p0s[k] * p0s[k];
        dd2 += dls[k] * dls[k];
        pd += p0s[k] * dls[k];
    }
    double lag = pp * dd2 - pd * pd, kappa = lag > 0 ? (pp * dd2 + pd * pd) / lag : 1.0;
    D->hmargin = fabs(m - 1.0) / ((1.0 + m) * kappa);
}

static void gauss_mean(const orc_gs *g, int64_t i, double *mu)
{
    mu[0] = g->mean[i]; mu[1] = g->mean[g->N + i]; mu[2] = g->mean[2 * g->N + i];
}

/* ---------------------------------------------------------------- per pixel */
typedef struct {
    double margin;      /* forward decisions */
    double grad_margin; /* alpha clamp */
    double T;
    int n, n_clamped;
    int64_t term_id; /* the fragment whose alpha would take T below 1e-4, -1 if none */
} pixinfo_t;

/* Fragments of pixel (u,v) in (depth, id) order that pass alpha >= 1/255, up
 * to (excluding) the first one that would take T below 1e-4. */
static int pixel_frags(const ctx_t *c, int u, int v, frag_t *F, pixinfo_t *info)
{
    double T = 1.0, margin = INFINITY, gmargin = INFINITY;
    int n = 0, ncl = 0;
    int64_t term = -1;
    int64_t jb, je;
    const int64_t *items;
    if (c->path == 1) { items = c->row_items; jb = c->row_start[v]; je = c->row_start[v + 1]; }
    else { items = c->order; jb = 0; je = c->n_vis; }
    for (int64_t j = jb; j < je; ++j) {
        int64_t id = items[j];
        const proj_t *P = &c->P[id];
        if (c->path == 1 && (u < P->m2[0] - P->rx - 1.0 || u > P->m2[0] + P->rx + 1.0)) continue;
        double dx = u - P->m2[0], dy = v - P->m2[1];
        double power = -0.5 * (P->conic[0] * dx * dx + P->conic[2] * dy * dy) - P->conic[1] * dx * dy;
        double G = exp(power);
        double oG = P->o * G;
        double alpha = oG < ALPHA_MAX ? oG : ALPHA_MAX;
        double m1 = relmargin(alpha, ALPHA_MIN);
        if (m1 < margin) margin = m1;
        if (alpha < ALPHA_MIN) continue;
        /* the order of the fragments is exact given the FP32 keys */
        if (P->zmargin < margin) margin = P->zmargin;
        double tT = T * (1.0 - alpha);
        double m2 = relmargin(tT, T_STOP);
        if (m2 < margin) margin = m2;
        if (tT < T_STOP) {
            term = id;
            break;
        }
        double mc = relmargin(oG, ALPHA_MAX);
        if (mc < gmargin) gmargin = mc;
        if (n >= MAX_FRAG) return -1;
        F[n].id = id;
        F[n].alpha = alpha;
        F[n].T = T;
        F[n].w = alpha * T;
        F[n].G = G;
        F[n].clamped = oG >= ALPHA_MAX;
        ncl += F[n].clamped;
        if (c->opt->depth_mode == 1) {
            F[n].d = P->z;
        } else {
            double mu[3];
            gauss_mean(c->g, id, mu);
            depth_t D;
            depth_literal(c, P, mu, u, v, &D);
            F[n].d = D.d;
            if (c->opt->depth_mode == 2) {
                if (D.hmargin < margin) margin = D.hmargin;
                if (D.disc < 0.0) F[n].d = P->z; /* no valid solution: centre depth */
            }
        }
        T = tT;
        ++n;
    }
    info->margin = margin;
    info->grad_margin = gmargin;
    info->T = T;
    info->n = n;
    info->n_clamped = ncl;
    info->term_id = term;
    return n;
}

typedef struct {
    double *rgb, *depth, *kmap, *sem, *T_final, *margin, *grad_margin;
    int32_t *last_id, *n_frag, *n_clamped;
} orc_fwd_out;

/* ---------------------------------------------------------------- API */
int orc_project(const orc_gs *g, const orc_cam *cam, const orc_opt *opt,
                int32_t *visible, int32_t *ambiguous, double *m2d, double *conic, double *cov,
                double *opac, double *kf, double *rgb, double *raw, double *z, double *radius)
{
    double C[3];
    cam_centre(cam, C);
    const int64_t N = g->N;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        proj_t P;
        memset(&P, 0, sizeof(P));
        project_one(g, cam, opt, C, i, &P);
        visible[i] = P.visible;
        ambiguous[i] = P.ambiguous;
        for (int k = 0; k < 2; ++k) m2d[2 * i + k] = P.m2[k];
        for (int k = 0; k < 3; ++k) {
            conic[3 * i + k] = P.conic[k];
            cov[3 * i + k] = P.cov[k];
            rgb[3 * i + k] = P.rgb[k];
            raw[3 * i + k] = P.raw[k];
        }
        opac[i] = P.o;
        kf[i] = P.k;
        z[i] = P.z;
        radius[2 * i] = P.rx;
        radius[2 * i + 1] = P.ry;
    }
    return 0;
}

/* Forward render.  pixmask (H*W bytes) selects the pixels to compute (NULL: all);
 * path 0 tests every visible Gaussian at every pixel, path 1 uses row lists. */
int orc_render(const orc_gs *g, const orc_cam *cam, const orc_opt *opt, int path,
               const uint8_t *pixmask, double *rgb, double *depth, double *kmap, double *sem,
               double *T_final, int32_t *last_id, int32_t *n_frag, int32_t *n_clamped,
               double *margin, double *grad_margin, int32_t *term_id)
{
    ctx_t c;
    if (ctx_init(&c, g, cam, opt, path)) { ctx_free(&c); return -1; }
    const int W = cam->W, H = cam->H, Co = g->C_o;
    const int64_t HW = (int64_t)W * H;
    int err = 0;
#pragma omp parallel
    {
        frag_t *F = (frag_t *)malloc(sizeof(frag_t) * MAX_FRAG);
#pragma omp for schedule(dynamic, 1)
        for (int v = 0; v < H; ++v) {
            for (int u = 0; u < W; ++u) {
                int64_t pix = (int64_t)v * W + u;
                if (pixmask && !pixmask[pix]) continue;
                pixinfo_t info;
                int n = pixel_frags(&c, u, v, F, &info);
                if (n < 0) { err = -2; continue; }
                double acc[3] = {0, 0, 0}, D = 0, K = 0;
                for (int ch = 0; ch < Co; ++ch) sem[ch * HW + pix] = 0.0;
                for (int f = 0; f < n; ++f) {
                    const proj_t *P = &c.P[F[f].id];
                    double w = F[f].w;
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += w * P->rgb[ch];
                    D += w * F[f].d;
                    K += w * P->k;
                    const double *o = g->sem + F[f].id * Co;
                    for (int ch = 0; ch < Co; ++ch) sem[ch * HW + pix] += w * o[ch];
                }
                for (int ch = 0; ch < 3; ++ch) rgb[ch * HW + pix] = acc[ch];
                depth[pix] = D;
                kmap[pix] = K;
                T_final[pix] = info.T;
                last_id[pix] = n > 0 ? (int32_t)F[n - 1].id : -1;
                n_frag[pix] = n;
                n_clamped[pix] = info.n_clamped;
                margin[pix] = info.margin;
                grad_margin[pix] = info.grad_margin;
                if (term_id) term_id[pix] = (int32_t)info.term_id;
            }
        }
        free(F);
    }
    ctx_free(&c);
    return err;
}

/* ---------------------------------------------------------------- normals */
#define NS_BORDER 0
#define NS_ZERO 1
#define NS_VALID 2

typedef struct {
    int state, flip, sgn;
    double vx[2][3], vy[2][3], n0[3], nn;
    double N[3];
    double margin;
} nrm_t;

static void backproject(const orc_cam *cam, const double *C, double D, int u, int v, double *P)
{
    double pc[3] = {(u - cam->cx) / cam->fx * D, (v - cam->cy) / cam->fy * D, D};
    for (int k = 0; k < 3; ++k) P[k] = cam->R[k] * pc[0] + cam->R[3 + k] * pc[1] + cam->R[6 + k] * pc[2] + C[k];
}

static void cross3(const double *a, const double *b, double *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Alg. normal_estimation at pixel (u,v) of a depth image. */
static void normal_at(const double *Dimg, const orc_cam *cam, const orc_opt *opt, const double *C,
                      int u, int v, nrm_t *R)
{
    const int W = cam->W, H = cam->H;
    int gs[2] = {opt->step1, opt->step2};
    int gm = gs[0] > gs[1] ? gs[0] : gs[1];
    memset(R, 0, sizeof(*R));
    R->margin = INFINITY;
    R->sgn = 1;
    if (u - gm < 0 || u + gm >= W || v - gm < 0 || v + gm >= H) { R->state = NS_BORDER; return; }
    double n[2][3];
    for (int s = 0; s < 2; ++s) {
        int g = gs[s];
        double Pxp[3], Pxm[3], Pyp[3], Pym[3];
        backproject(cam, C, Dimg[(int64_t)v * W + u + g], u + g, v, Pxp);
        backproject(cam, C, Dimg[(int64_t)v * W + u - g], u - g, v, Pxm);
        backproject(cam, C, Dimg[(int64_t)(v + g) * W + u], u, v + g, Pyp);
        backproject(cam, C, Dimg[(int64_t)(v - g) * W + u], u, v - g, Pym);
        for (int k = 0; k < 3; ++k) { R->vx[s][k] = Pxp[k] - Pxm[k]; R->vy[s][k] = Pyp[k] - Pym[k]; }
        cross3(R->vx[s], R->vy[s], n[s]);
    }
    double d12 = dot3(n[0], n[1]);
    double l1 = sqrt(dot3(n[0], n[0])), l2 = sqrt(dot3(n[1], n[1]));
    if (l1 > 0 && l2 > 0) {
        double m = fabs(d12) / (l1 * l2);
        if (m < R->margin) R->margin = m;
    }
    R->sgn = d12 < 0 ? -1 : 1;
    double nf[3];
    for (int k = 0; k < 3; ++k) nf[k] = opt->lambda * n[0][k] + (1.0 - opt->lambda) * R->sgn * n[1][k];
    R->nn = sqrt(dot3(nf, nf));
    double thr = opt->eps_n * sqrt(dot3(R->vx[0], R->vx[0])) * sqrt(dot3(R->vy[0], R->vy[0]));
    if (R->nn > 0) {
        double m = fabs(R->nn - thr) / R->nn;
        if (m < R->margin) R->margin = m;
    }
    if (!(R->nn > thr)) { R->state = NS_ZERO; return; }
    for (int k = 0; k < 3; ++k) R->n0[k] = nf[k] / R->nn;
    double P0[3];
    backproject(cam, C, Dimg[(int64_t)v * W + u], u, v, P0);
    double dv[3] = {C[0] - P0[0], C[1] - P0[1], C[2] - P0[2]};
    double nd = dot3(R->n0, dv), ldv = sqrt(dot3(dv, dv));
    if (ldv > 0) {
        double m = fabs(nd) / ldv;
        if (m < R->margin) R->margin = m;
    }
    R->flip = (opt->orient_sign * nd) < 0;
    for (int k = 0; k < 3; ++k) R->N[k] = R->flip ? -R->n0[k] : R->n0[k];
    R->state = NS_VALID;
}

int orc_normals(const double *depth, const orc_cam *cam, const orc_opt *opt, const uint8_t *pixmask,
                double *normal, int32_t *state, double *margin)
{
    double C[3];
    cam_centre(cam, C);
    const int W = cam->W, H = cam->H;
    const int64_t HW = (int64_t)W * H;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int64_t pix = (int64_t)v * W + u;
            if (pixmask && !pixmask[pix]) continue;
            nrm_t R;
            normal_at(depth, cam, opt, C, u, v, &R);
            for (int k = 0; k < 3; ++k) normal[k * HW + pix] = R.N[k];
            state[pix] = R.state | (R.flip ? 4 : 0) | (R.sgn < 0 ? 8 : 0);
            margin[pix] = R.margin;
        }
    return 0;
}

/* Alg. normal_gradient: dL/dN -> dL/dD for every pixel.  dnormal is [3][H][W];
 * pixels whose normal is not valid receive and send nothing.  Output is added
 * to gD. */
int orc_normal_backward(const double *depth, const orc_cam *cam, const orc_opt *opt,
                        const double *dnormal, double *gD)
{
    double C[3];
    cam_centre(cam, C);
    const int W = cam->W, H = cam->H;
    const int64_t HW = (int64_t)W * H;
    double *GP = (double *)calloc((size_t)HW * 3, sizeof(double));
    if (!GP) return -1;
    int gs[2] = {opt->step1, opt->step2};
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int64_t pix = (int64_t)v * W + u;
            double gN[3] = {dnormal[pix], dnormal[HW + pix], dnormal[2 * HW + pix]};
            if (gN[0] == 0 && gN[1] == 0 && gN[2] == 0) continue;
            nrm_t R;
            normal_at(depth, cam, opt, C, u, v, &R);
            if (R.state != NS_VALID) continue;
            /* 1. view-facing flip */
            if (R.flip) for (int k = 0; k < 3; ++k) gN[k] = -gN[k];
            /* 2. normalisation: (I - N N^T) / |n_fused| */
            double pr = dot3(R.n0, gN), gn[3];
            for (int k = 0; k < 3; ++k) gn[k] = (gN[k] - R.n0[k] * pr) / R.nn;
            /* 3. fusion */
            double gns[2][3];
            for (int k = 0; k < 3; ++k) {
                gns[0][k] = opt->lambda * gn[k];
                gns[1][k] = (1.0 - opt->lambda) * R.sgn * gn[k];
            }
            /* 4. cross products and finite-difference scatter */
            for (int s = 0; s < 2; ++s) {
                int g = gs[s];
                double gvx[3], gvy[3];
                cross3(R.vy[s], gns[s], gvx);
                cross3(gns[s], R.vx[s], gvy);
                int64_t qxp = (int64_t)v * W + u + g, qxm = (int64_t)v * W + u - g;
                int64_t qyp = (int64_t)(v + g) * W + u, qym = (int64_t)(v - g) * W + u;
                for (int k = 0; k < 3; ++k) {
                    GP[3 * qxp + k] += gvx[k];
                    GP[3 * qxm + k] -= gvx[k];
                    GP[3 * qyp + k] += gvy[k];
                    GP[3 * qym + k] -= gvy[k];
                }
            }
        }
    /* 5. back-projection Jacobian dP/dD = R^T p */
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int64_t pix = (int64_t)v * W + u;
            double p[3] = {(u - cam->cx) / cam->fx, (v - cam->cy) / cam->fy, 1.0}, J[3];
            for (int k = 0; k < 3; ++k) J[k] = cam->R[k] * p[0] + cam->R[3 + k] * p[1] + cam->R[6 + k] * p[2];
            gD[pix] += dot3(&GP[3 * pix], J);
        }
    free(GP);
    return 0;
}

/* ---------------------------------------------------------------- backward */
enum { A_DC = 0, A_DCONIC = 3, A_DM = 6, A_DOP = 8, A_DMU = 9, A_DS = 12, A_DRG = 15, A_N = 24 };

static void atomic_add(double *p, double x)
{
#pragma omp atomic
    *p += x;
}

/* Alg. backward_render for one pixel: reverse traversal restoring T, with the
 * full alpha path; per-Gaussian adjoints go to adj[id*A_N + .], the semantic
 * and gradient-factor gradients straight to dsem / dmask. */
static void pixel_backward(const ctx_t *c, int u, int v, const frag_t *F, int n, const double *gC,
                           double gD, double gK, const double *gO, double *adj, double *dsem, double *dmask)
{
    const orc_gs *g = c->g;
    const int Co = g->C_o;
    double A = 0.0;
    for (int f = n - 1; f >= 0; --f) {
        int64_t id = F[f].id;
        const proj_t *P = &c->P[id];
        const double *o = g->sem + id * Co;
        double s = gC[0] * P->rgb[0] + gC[1] * P->rgb[1] + gC[2] * P->rgb[2] + gD * F[f].d + gK * P->k;
        for (int ch = 0; ch < Co; ++ch) s += gO[ch] * o[ch];
        double w = F[f].w, al = F[f].alpha;
        double dalpha = F[f].T * s - A / (1.0 - al);
        A += w * s;
        double *a = adj + id * A_N;
        for (int ch = 0; ch < 3; ++ch) atomic_add(&a[A_DC + ch], w * gC[ch]);
        atomic_add(&dmask[id], w * gK * P->k * (1.0 - P->k));
        for (int ch = 0; ch < Co; ++ch) atomic_add(&dsem[id * Co + ch], w * gO[ch]);
        /* depth: supplementary S1.2 chain */
        double dd = w * gD;
        depth_t D;
        int centre = c->opt->depth_mode == 1;
        if (dd != 0.0 && !centre) {
            double mu[3];
            gauss_mean(g, id, mu);
            depth_literal(c, P, mu, u, v, &D);
            centre = c->opt->depth_mode == 2 && D.disc < 0.0;
        }
        if (dd != 0.0 && centre) {
            /* d = mu_c.z = R[2,:] mu + t_z */
            for (int r = 0; r < 3; ++r) atomic_add(&a[A_DMU + r], dd * c->cam->R[6 + r]);
        } else if (dd != 0.0) {
            double dtm = dd * D.dd_dt;                 /* Eq. (d->tmid) */
            double gvs[3], gds[3], gvl[3], gdl[3];
            for (int k = 0; k < 3; ++k) {              /* Eq. (tmid->vs) */
                gvs[k] = dtm * (-D.ds[k] / D.a);
                gds[k] = dtm * (D.b / (D.a * D.a) * D.ds[k] - D.vs[k] / D.a);
            }
            for (int k = 0; k < 3; ++k) {              /* Eq. (vs->s) */
                gvl[k] = gvs[k] / P->s[k];
                gdl[k] = gds[k] / P->s[k];
                atomic_add(&a[A_DS + k], -(gvs[k] * D.vl[k] + gds[k] * D.dl[k]) / (P->s[k] * P->s[k]));
            }
            for (int r = 0; r < 3; ++r) {              /* Eq. (vs->mu), Eq. (vs->r) */
                atomic_add(&a[A_DMU + r], -(P->Rg[3 * r] * gvl[0] + P->Rg[3 * r + 1] * gvl[1] + P->Rg[3 * r + 2] * gvl[2]));
                for (int k = 0; k < 3; ++k)
                    atomic_add(&a[A_DRG + 3 * r + k], D.v[r] * gvl[k] + D.dr[r] * gdl[k]);
            }
        }
        /* alpha = min(0.99, o G), G = exp(power) */
        if (!F[f].clamped) {
            double G = F[f].G;
            atomic_add(&a[A_DOP], dalpha * G);
            double dpow = dalpha * P->o * G;
            double dx = u - P->m2[0], dy = v - P->m2[1];
            atomic_add(&a[A_DCONIC + 0], -0.5 * dx * dx * dpow);
            atomic_add(&a[A_DCONIC + 1], -dx * dy * dpow);
            atomic_add(&a[A_DCONIC + 2], -0.5 * dy * dy * dpow);
            double ddx = -(P->conic[0] * dx + P->conic[1] * dy) * dpow;
            double ddy = -(P->conic[1] * dx + P->conic[2] * dy) * dpow;
            atomic_add(&a[A_DM + 0], -ddx);
            atomic_add(&a[A_DM + 1], -ddy);
        }
    }
}

/* Chain one Gaussian's per-view adjoints into parameter gradients (added). */
static void chain_one(const ctx_t *c, int64_t i, const double *a, double *dmean, double *dquat,
                      double *dls, double *dop, double *dsh)
{
    const orc_gs *g = c->g;
    const orc_cam *cam = c->cam;
    const double *R = cam->R;
    const int64_t N = g->N;
    const proj_t *P = &c->P[i];
    double dmu[3] = {a[A_DMU], a[A_DMU + 1], a[A_DMU + 2]};
    double ds[3] = {a[A_DS], a[A_DS + 1], a[A_DS + 2]};
    double dRg[9];
    for (int k = 0; k < 9; ++k) dRg[k] = a[A_DRG + k];
    dop[i] += a[A_DOP] * P->o * (1.0 - P->o);

    /* colour */
    int nc = (g->sh_deg + 1) * (g->sh_deg + 1);
    double ddir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
        double dc = P->raw[ch] > 0 ? a[A_DC + ch] : 0.0;
        if (dc == 0.0) continue;
        for (int k = 0; k < nc; ++k) {
            dsh[((int64_t)k * 3 + ch) * N + i] += dc * P->Y[k];
            double shv = g->sh[((int64_t)k * 3 + ch) * N + i];
            for (int e = 0; e < 3; ++e) ddir[e] += dc * shv * P->dY[k][e];
        }
    }
    double pr = dot3(P->dir, ddir);
    for (int e = 0; e < 3; ++e) dmu[e] += (ddir[e] - P->dir[e] * pr) / P->dist;

    /* 2D mean */
    double z = P->mc[2], dmc[3] = {0, 0, 0};
    dmc[0] += a[A_DM] * cam->fx / z;
    dmc[1] += a[A_DM + 1] * cam->fy / z;
    dmc[2] -= a[A_DM] * cam->fx * P->mc[0] / (z * z) + a[A_DM + 1] * cam->fy * P->mc[1] / (z * z);

    /* conic -> Sigma2D (full-entry symmetric convention) */
    double Cm[4] = {P->conic[0], P->conic[1], P->conic[1], P->conic[2]};
    double dCm[4] = {a[A_DCONIC], 0.5 * a[A_DCONIC + 1], 0.5 * a[A_DCONIC + 1], a[A_DCONIC + 2]};
    double tmp[4], dS2[4];
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) tmp[2 * r + q] = dCm[2 * r] * Cm[q] + dCm[2 * r + 1] * Cm[2 + q];
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) dS2[2 * r + q] = -(Cm[2 * r] * tmp[q] + Cm[2 * r + 1] * tmp[2 + q]);
    /* Sigma2D = T Sigma T^T: dSigma = T^T dS2 T, dT = 2 dS2 T Sigma */
    double dSig[9], dT[6], TS[6];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += P->Tm[3 * k + r] * dS2[2 * k + l] * P->Tm[3 * l + q];
            dSig[3 * r + q] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 3; ++q) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += P->Tm[3 * r + k] * P->Sig[3 * k + q];
            TS[3 * r + q] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 3; ++q) dT[3 * r + q] = 2.0 * (dS2[2 * r] * TS[q] + dS2[2 * r + 1] * TS[3 + q]);
    /* T = J R: dJ = dT R^T */
    double dJ[6];
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 3; ++q) dJ[3 * r + q] = dT[3 * r] * R[3 * q] + dT[3 * r + 1] * R[3 * q + 1] + dT[3 * r + 2] * R[3 * q + 2];
    double fx = cam->fx, fy = cam->fy;
    dmc[2] += dJ[0] * (-fx / (z * z)) + dJ[4] * (-fy / (z * z)) + dJ[2] * (2 * fx * P->xcl / (z * z * z)) +
              dJ[5] * (2 * fy * P->ycl / (z * z * z));
    double dxc = dJ[2] * (-fx / (z * z)), dyc = dJ[5] * (-fy / (z * z));
    if (!P->clx) dmc[0] += dxc; else dmc[2] += dxc * P->xcl / z;
    if (!P->cly) dmc[1] += dyc; else dmc[2] += dyc * P->ycl / z;
    for (int e = 0; e < 3; ++e) dmu[e] += R[e] * dmc[0] + R[3 + e] * dmc[1] + R[6 + e] * dmc[2];

    /* Sigma = M M^T, M = Rg diag(s) */
    double M[9], dM[9];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) M[3 * r + q] = P->Rg[3 * r + q] * P->s[q];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += (dSig[3 * r + k] + dSig[3 * k + r]) * M[3 * k + q];
            dM[3 * r + q] = acc;
        }
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) dRg[3 * r + q] += dM[3 * r + q] * P->s[q];
    for (int q = 0; q < 3; ++q) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += P->Rg[3 * k + q] * dM[3 * k + q];
        ds[q] += acc;
    }
    for (int e = 0; e < 3; ++e) {
        dmean[e * N + i] += dmu[e];
        dls[e * N + i] += ds[e] * P->s[e];
    }
    double dqh[4];
    quat_rot_vjp(P->qh, dRg, dqh);
    double pq = dqh[0] * P->qh[0] + dqh[1] * P->qh[1] + dqh[2] * P->qh[2] + dqh[3] * P->qh[3];
    for (int k = 0; k < 4; ++k) dquat[k * N + i] += (dqh[k] - P->qh[k] * pq) / P->qn;
}

/* Backward of L = <W, outputs> for one view.  Upstream maps are planar [C][H][W];
 * depth is the forward depth image (needed by the normal branch).  pixmask selects
 * the pixels whose compositing adjoint is evaluated (NULL: all); the normal branch
 * always runs on the whole image.  Gradients are ADDED to the outputs.  gD_out
 * (nullable) receives dL/dD + normal-branch gradient per pixel. */
int orc_backward(const orc_gs *g, const orc_cam *cam, const orc_opt *opt, int path, const uint8_t *pixmask,
                 const double *depth, const double *drgb, const double *ddepth, const double *dkmap,
                 const double *dnormal, const double *dsem_img, double *dmean, double *dquat, double *dls,
                 double *dop, double *dmask, double *dsh, double *dsem, double *gD_out)
{
    const int W = cam->W, H = cam->H, Co = g->C_o;
    const int64_t HW = (int64_t)W * H;
    double *gD = (double *)malloc(sizeof(double) * (size_t)HW);
    if (!gD) return -1;
    for (int64_t p = 0; p < HW; ++p) gD[p] = ddepth[p];
    if (dnormal && orc_normal_backward(depth, cam, opt, dnormal, gD)) { free(gD); return -1; }
    if (gD_out) memcpy(gD_out, gD, sizeof(double) * (size_t)HW);
    ctx_t c;
    if (ctx_init(&c, g, cam, opt, path)) { ctx_free(&c); free(gD); return -1; }
    double *adj = (double *)calloc((size_t)(g->N > 0 ? g->N : 1) * A_N, sizeof(double));
    if (!adj) { ctx_free(&c); free(gD); return -1; }
    int err = 0;
#pragma omp parallel
    {
        frag_t *F = (frag_t *)malloc(sizeof(frag_t) * MAX_FRAG);
        double *gO = (double *)malloc(sizeof(double) * (size_t)(Co > 0 ? Co : 1));
#pragma omp for schedule(dynamic, 1)
        for (int v = 0; v < H; ++v)
            for (int u = 0; u < W; ++u) {
                int64_t pix = (int64_t)v * W + u;
                if (pixmask && !pixmask[pix]) continue;
                double gC[3] = {drgb[pix], drgb[HW + pix], drgb[2 * HW + pix]};
                int any = gC[0] != 0 || gC[1] != 0 || gC[2] != 0 || gD[pix] != 0 || dkmap[pix] != 0;
                for (int ch = 0; ch < Co; ++ch) {
                    gO[ch] = dsem_img[ch * HW + pix];
                    any |= gO[ch] != 0;
                }
                if (!any) continue;
                pixinfo_t info;
                int n = pixel_frags(&c, u, v, F, &info);
                if (n < 0) { err = -2; continue; }
                pixel_backward(&c, u, v, F, n, gC, gD[pix], dkmap[pix], gO, adj, dsem, dmask);
            }
        free(F);
        free(gO);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->N; ++i) {
        if (!c.P[i].visible) continue;
        chain_one(&c, i, adj + i * A_N, dmean, dquat, dls, dop, dsh);
    }
    free(adj);
    ctx_free(&c);
    free(gD);
    return err;
}

/* Depth of one fragment by the literal ray-ellipsoid construction (for pins). */
int orc_fragment_depth(const orc_gs *g, const orc_cam *cam, const orc_opt *opt, int64_t i, double u, double v,
                       double *out /* d, t_mid, a, b */)
{
    ctx_t c;
    memset(&c, 0, sizeof(c));
    c.g = g; c.cam = cam; c.opt = opt;
    cam_centre(cam, c.C);
    proj_t P;
    memset(&P, 0, sizeof(P));
    project_one(g, cam, opt, c.C, i, &P);
    double mu[3];
    gauss_mean(g, i, mu);
    depth_t D;
    depth_literal(&c, &P, mu, u, v, &D);
    out[0] = D.d;
    out[1] = D.tm;
    out[2] = D.a;
    out[3] = D.b;
    out[4] = dot3(D.vs, D.vs) - 1.0;
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the OpenMP thread count of later calls (timing at one thread). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
