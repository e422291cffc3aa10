/*
 * FP64 CPU oracle of the sort-free, order-independent-transparency (OIT)
 * Gaussian-splat renderer and of its gradient.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU renderer, and the GPU renderer never calls it.
 *
 * Everything is evaluated in double precision, single-threaded, splat by splat, in
 * the order the definitions are stated:
 *   - the 3D Gaussian and its covariance Sigma = R S S^T R^T
 *       (Sec. 3.1, Eq. "3d_gaussian");
 *   - the EWA screen-space covariance Sigma' = J W Sigma W^T J^T
 *       (Sec. 3.1, Eq. "3dgs_proj"), plus the 0.3 px^2 low-pass of 3DGS;
 *   - the colour c = Y(dir, h) from degree-3 spherical harmonics
 *       (Sec. 3.1, Eq. "3dgs_color");
 *   - the opacity falloff alpha = o exp(-1/2 d^T Sigma'^-1 d)
 *       (Sec. 3.1, Eq. "3dgs_alpha");
 *   - the weight w = max(0, 1 - d/sigma) v(r) (Sec. 1, Eq. "sf_weight");
 *   - the weighted OIT composite C = T c0 + (1-T) P/Q, T = prod(1 - alpha)
 *       (Sec. 3.2, Eq. "oit_rendering"; App. B, Eq. "oit_rendering_md");
 *   - its partials dC/dc, dC/dalpha, dC/dw (App. B, Eq. "oit_rendering_detail")
 *     and the chain rule from there to every splat parameter and to sigma.
 *
 * Readings where the paper is silent or garbled (each is one named constant or one
 * commented line below): opacity is a sigmoid of a logit; the colour and the view
 * weight are evaluated at the unit direction from the camera centre to the mean,
 * plus 0.5 and clamped at 0; d is the camera-space depth of the mean; the 3DGS
 * defaults apply (alpha capped at 0.99, a pair contributes iff alpha >= 1/255,
 * 0.3 px^2 dilation, 1.3x guard band on the Jacobian, near plane 0.2); F = 0 and
 * no gradient flows through F when Q = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ALPHA_MIN (1.0 / 255.0)
#define ORC_ALPHA_MAX 0.99
#define ORC_DILATION 0.3
#define ORC_GUARD 1.3
#define ORC_COLOR_OFFSET 0.5

typedef struct {
    int width, height;
    double fx, fy, cx, cy;
    double R[9]; /* world -> camera rotation, row-major */
    double t[3];
    double near_z;
} orc_camera;

typedef struct {
    long n;
    const double *mean;          /* [3][n] */
    const double *log_scale;     /* [3][n] */
    const double *quat;          /* [4][n]  (w, x, y, z) */
    const double *opacity_logit; /* [n] */
    const double *sh;            /* [16][3][n] */
    const double *vsh;           /* [16][n] */
} orc_splats;

typedef struct {
    double *mean, *log_scale, *quat, *opacity_logit, *sh, *vsh; /* same layout, added to */
} orc_grads;

typedef struct { int x0, y0, x1, y1; } orc_window; /* half-open pixel rectangle */

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics of degree <= 3 at a unit direction (x, y, z).     */
/* Normalisation constants from their closed form sqrt((2l+1)/4pi (l-m)!/(l+m)!) */
/* with the usual sqrt(2) for m != 0; signs as in the 3DGS colour model.      */
/* ------------------------------------------------------------------------- */
static void sh_basis(const double dir[3], double Y[16], double dY[16][3])
{
    const double pi = 3.14159265358979323846;
    const double k0 = 0.5 * sqrt(1.0 / pi);
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = 0.5 * sqrt(15.0 / pi);
    const double k2b = 0.25 * sqrt(5.0 / pi);
    const double k2c = 0.25 * sqrt(15.0 / pi);
    const double k3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double k3b = 0.5 * sqrt(105.0 / pi);
    const double k3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double k3d = 0.25 * sqrt(7.0 / pi);
    const double k3e = 0.25 * sqrt(105.0 / pi);
    const double x = dir[0], y = dir[1], z = dir[2];
    const double xx = x * x, yy = y * y, zz = z * z;

    Y[0] = k0;
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    Y[4] = k2a * x * y;
    Y[5] = -k2a * y * z;
    Y[6] = k2b * (2.0 * zz - xx - yy);
    Y[7] = -k2a * x * z;
    Y[8] = k2c * (xx - yy);
    Y[9] = -k3a * y * (3.0 * xx - yy);
    Y[10] = k3b * x * y * z;
    Y[11] = -k3c * y * (4.0 * zz - xx - yy);
    Y[12] = k3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -k3c * x * (4.0 * zz - xx - yy);
    Y[14] = k3e * z * (xx - yy);
    Y[15] = -k3a * x * (xx - 3.0 * yy);

    if (!dY) return;
    memset(dY, 0, sizeof(double) * 48);
    dY[1][1] = -k1;
    dY[2][2] = k1;
    dY[3][0] = -k1;
    dY[4][0] = k2a * y;            dY[4][1] = k2a * x;
    dY[5][1] = -k2a * z;           dY[5][2] = -k2a * y;
    dY[6][0] = -2.0 * k2b * x;     dY[6][1] = -2.0 * k2b * y;   dY[6][2] = 4.0 * k2b * z;
    dY[7][0] = -k2a * z;           dY[7][2] = -k2a * x;
    dY[8][0] = 2.0 * k2c * x;      dY[8][1] = -2.0 * k2c * y;
    dY[9][0] = -k3a * 6.0 * x * y; dY[9][1] = -k3a * (3.0 * xx - 3.0 * yy);
    dY[10][0] = k3b * y * z;       dY[10][1] = k3b * x * z;     dY[10][2] = k3b * x * y;
    dY[11][0] = -k3c * (-2.0 * x * y);
    dY[11][1] = -k3c * (4.0 * zz - xx - 3.0 * yy);
    dY[11][2] = -k3c * (8.0 * y * z);
    dY[12][0] = k3d * (-6.0 * x * z);
    dY[12][1] = k3d * (-6.0 * y * z);
    dY[12][2] = k3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    dY[13][0] = -k3c * (4.0 * zz - 3.0 * xx - yy);
    dY[13][1] = -k3c * (-2.0 * x * y);
    dY[13][2] = -k3c * (8.0 * x * z);
    dY[14][0] = k3e * 2.0 * x * z; dY[14][1] = -k3e * 2.0 * y * z; dY[14][2] = k3e * (xx - yy);
    dY[15][0] = -k3a * (3.0 * xx - 3.0 * yy);
    dY[15][1] = -k3a * (-6.0 * x * y);
}

/* Exported for the basis tests (orthonormality on the sphere, derivative by FD). */
void orc_sh_basis(const double dir[3], double Y[16], double dY[48])
{
    double d[16][3];
    sh_basis(dir, Y, d);
    if (dY) memcpy(dY, d, sizeof(d));
}

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

void orc_quat_to_rot(const double q[4], double R[9]) { quat_to_rot(q, R); }

/* ------------------------------------------------------------------------- */
/* Per-splat projection                                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int valid;
    double mu[3];        /* world mean */
    double tc[3];        /* camera-space mean, W mu + t */
    double scale[3];
    double qn[4], qlen;  /* unit quaternion and the raw length */
    double Rq[9];
    double Sigma[9];     /* 3D covariance */
    int clamp_x, clamp_y;
    double lim_x, lim_y; /* guard-band limits on tx/tz, ty/tz */
    double J[6];         /* 2x3 */
    double T[6];         /* J W, 2x3 */
    double cov[4];       /* 2x2 screen covariance incl. dilation */
    double conic[4];     /* its inverse */
    double mx, my;
    double opacity;
    double cc[3];        /* camera centre */
    double dir[3], dist; /* unit direction from the camera centre to the mean */
    double Y[16], dY[16][3];
    double raw_c[3], color[3];
    double raw_v, v;
    double d, w;
    int w_on;            /* d < sigma */
    double tau;          /* 2 ln(255 o): alpha >= 1/255  <=>  m <= tau */
    int x0, x1, y0, y1;  /* conservative pixel bbox (half-open), clipped to the image */
} orc_proj;

static double get(const double *a, long n, int c, long i) { return a[(long)c * n + i]; }

static void project_splat(const orc_splats *s, long i, double sigma, const orc_camera *cam, orc_proj *p)
{
    long n = s->n;
    memset(p, 0, sizeof(*p));
    for (int k = 0; k < 3; ++k) p->mu[k] = get(s->mean, n, k, i);
    const double *W = cam->R;
    for (int r = 0; r < 3; ++r)
        p->tc[r] = W[3 * r] * p->mu[0] + W[3 * r + 1] * p->mu[1] + W[3 * r + 2] * p->mu[2] + cam->t[r];
    p->d = p->tc[2];
    if (!(p->d > cam->near_z)) { p->valid = 0; return; }

    /* 3D covariance Sigma = Rq S S^T Rq^T */
    for (int k = 0; k < 3; ++k) p->scale[k] = exp(get(s->log_scale, n, k, i));
    double q[4], ql = 0.0;
    for (int k = 0; k < 4; ++k) { q[k] = get(s->quat, n, k, i); ql += q[k] * q[k]; }
    ql = sqrt(ql);
    p->qlen = ql;
    for (int k = 0; k < 4; ++k) p->qn[k] = q[k] / ql;
    quat_to_rot(p->qn, p->Rq);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                acc += p->Rq[3 * a + k] * p->scale[k] * p->scale[k] * p->Rq[3 * b + k];
            p->Sigma[3 * a + b] = acc;
        }

    /* EWA: Jacobian of the perspective map at the (guard-band clamped) mean */
    const double tz = p->tc[2];
    p->lim_x = ORC_GUARD * (0.5 * cam->width / cam->fx);
    p->lim_y = ORC_GUARD * (0.5 * cam->height / cam->fy);
    double rx = p->tc[0] / tz, ry = p->tc[1] / tz;
    if (rx > p->lim_x) { rx = p->lim_x; p->clamp_x = 1; }
    if (rx < -p->lim_x) { rx = -p->lim_x; p->clamp_x = -1; }
    if (ry > p->lim_y) { ry = p->lim_y; p->clamp_y = 1; }
    if (ry < -p->lim_y) { ry = -p->lim_y; p->clamp_y = -1; }
    const double txp = rx * tz, typ = ry * tz;
    p->J[0] = cam->fx / tz; p->J[1] = 0.0;             p->J[2] = -cam->fx * txp / (tz * tz);
    p->J[3] = 0.0;          p->J[4] = cam->fy / tz;    p->J[5] = -cam->fy * typ / (tz * tz);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += p->J[3 * a + k] * W[3 * k + b];
            p->T[3 * a + b] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l)
                    acc += p->T[3 * a + k] * p->Sigma[3 * k + l] * p->T[3 * b + l];
            p->cov[2 * a + b] = acc;
        }
    p->cov[0] += ORC_DILATION;
    p->cov[3] += ORC_DILATION;
    const double det = p->cov[0] * p->cov[3] - p->cov[1] * p->cov[2];
    if (!(det > 0.0)) { p->valid = 0; return; }
    p->conic[0] = p->cov[3] / det;
    p->conic[1] = -p->cov[1] / det;
    p->conic[2] = -p->cov[2] / det;
    p->conic[3] = p->cov[0] / det;
    p->mx = cam->fx * p->tc[0] / tz + cam->cx;
    p->my = cam->fy * p->tc[1] / tz + cam->cy;

    /* appearance */
    p->opacity = 1.0 / (1.0 + exp(-s->opacity_logit[i]));
    for (int r = 0; r < 3; ++r)
        p->cc[r] = -(W[r] * cam->t[0] + W[3 + r] * cam->t[1] + W[6 + r] * cam->t[2]);
    double u[3], ul = 0.0;
    for (int k = 0; k < 3; ++k) { u[k] = p->mu[k] - p->cc[k]; ul += u[k] * u[k]; }
    ul = sqrt(ul);
    p->dist = ul;
    for (int k = 0; k < 3; ++k) p->dir[k] = u[k] / ul;
    sh_basis(p->dir, p->Y, p->dY);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < 16; ++k) acc += p->Y[k] * s->sh[((long)k * 3 + ch) * n + i];
        p->raw_c[ch] = acc + ORC_COLOR_OFFSET;
        p->color[ch] = p->raw_c[ch] > 0.0 ? p->raw_c[ch] : 0.0;
    }
    {
        double acc = 0.0;
        for (int k = 0; k < 16; ++k) acc += p->Y[k] * s->vsh[(long)k * n + i];
        p->raw_v = acc + ORC_COLOR_OFFSET;
        p->v = p->raw_v > 0.0 ? p->raw_v : 0.0;
    }
    /* w(d, r) = max(0, 1 - d/sigma) v(r) */
    p->w_on = p->d < sigma;
    p->w = p->w_on ? (1.0 - p->d / sigma) * p->v : 0.0;

    /* footprint: alpha >= 1/255  <=>  m <= 2 ln(255 o) */
    p->tau = 2.0 * log(p->opacity / ORC_ALPHA_MIN);
    p->valid = 1;
    if (p->tau < 0.0) { p->x0 = p->x1 = p->y0 = p->y1 = 0; return; }
    const double hx = sqrt(p->tau * p->cov[0]), hy = sqrt(p->tau * p->cov[3]);
    /* pixel centres i + 0.5 within [mx - hx, mx + hx], widened by one pixel */
    double fx0 = floor(p->mx - hx - 0.5) - 1.0, fx1 = ceil(p->mx + hx - 0.5) + 2.0;
    double fy0 = floor(p->my - hy - 0.5) - 1.0, fy1 = ceil(p->my + hy - 0.5) + 2.0;
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > cam->width) fx1 = cam->width;
    if (fy1 > cam->height) fy1 = cam->height;
    p->x0 = (int)fx0; p->x1 = (int)fx1; p->y0 = (int)fy0; p->y1 = (int)fy1;
    if (p->x1 < p->x0) p->x1 = p->x0;
    if (p->y1 < p->y0) p->y1 = p->y0;
}

/* Stage output, ORC_PROJ_FIELDS doubles per splat:
 * valid, mx, my, conic_xx, conic_xy, conic_yy, opacity, c_r, c_g, c_b, v, d, w, tau,
 * cov_xx, cov_xy, cov_yy, x0, x1, y0, y1 (footprint box) */
#define ORC_PROJ_FIELDS 21
int orc_project(const orc_splats *s, double sigma, const orc_camera *cam, double *out)
{
    orc_proj p;
    for (long i = 0; i < s->n; ++i) {
        project_splat(s, i, sigma, cam, &p);
        double *o = out + ORC_PROJ_FIELDS * i;
        o[0] = p.valid; o[1] = p.mx; o[2] = p.my;
        o[3] = p.conic[0]; o[4] = p.conic[1]; o[5] = p.conic[3];
        o[6] = p.opacity; o[7] = p.color[0]; o[8] = p.color[1]; o[9] = p.color[2];
        o[10] = p.v; o[11] = p.d; o[12] = p.w; o[13] = p.tau;
        o[14] = p.cov[0]; o[15] = p.cov[1]; o[16] = p.cov[3];
        o[17] = p.x0; o[18] = p.x1; o[19] = p.y0; o[20] = p.y1;
    }
    return 0;
}

/* Opacity of splat p at pixel (px, py) (pixel-centre coordinates).
 * Returns 1 iff the pair contributes (alpha >= 1/255). */
static int pair_alpha(const orc_proj *p, double px, double py, double *alpha, double *G,
                      double *dx, double *dy, int *capped, double *raw)
{
    *dx = px - p->mx;
    *dy = py - p->my;
    const double m = p->conic[0] * *dx * *dx + (p->conic[1] + p->conic[2]) * *dx * *dy +
                     p->conic[3] * *dy * *dy;
    *G = exp(-0.5 * m);
    const double a = p->opacity * *G;
    *raw = a;
    *capped = a > ORC_ALPHA_MAX;
    *alpha = *capped ? ORC_ALPHA_MAX : a;
    return a >= ORC_ALPHA_MIN;
}

static uint64_t mix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

/* Discrete state of a splat that a finite-difference stencil must not change. */
static uint64_t splat_signature(const orc_proj *p, long i)
{
    uint64_t b = (uint64_t)(p->valid & 1) | ((uint64_t)(p->clamp_x + 1) << 1) |
                 ((uint64_t)(p->clamp_y + 1) << 3) | ((uint64_t)(p->raw_c[0] > 0) << 5) |
                 ((uint64_t)(p->raw_c[1] > 0) << 6) | ((uint64_t)(p->raw_c[2] > 0) << 7) |
                 ((uint64_t)(p->raw_v > 0) << 8) | ((uint64_t)p->w_on << 9);
    return mix64(((uint64_t)i << 12) ^ b ^ 0x5bd1e995ULL);
}

/* Per-pixel accumulators of one render. */
typedef struct {
    double P[3], Q, T;
    double P0[3], P1[3], Q0, Q1, logT; /* sigma-free parts (for pre-rendered buffers) */
} orc_acc;

static void acc_init(orc_acc *a)
{
    memset(a, 0, sizeof(*a));
    a->T = 1.0;
}

static void acc_add(orc_acc *a, const orc_proj *p, double alpha)
{
    for (int ch = 0; ch < 3; ++ch) a->P[ch] += p->color[ch] * alpha * p->w;
    a->Q += alpha * p->w;
    a->T *= (1.0 - alpha);
    if (p->w_on) {
        for (int ch = 0; ch < 3; ++ch) {
            a->P0[ch] += p->color[ch] * alpha * p->v;
            a->P1[ch] += p->color[ch] * alpha * p->v * p->d;
        }
        a->Q0 += alpha * p->v;
        a->Q1 += alpha * p->v * p->d;
    }
    a->logT += log(1.0 - alpha);
}

/* C = T c0 + (1 - T) F,  F = P / Q  (F = 0 when Q = 0). */
static void acc_finish(const orc_acc *a, const double bg[3], double C[3], double F[3])
{
    for (int ch = 0; ch < 3; ++ch) {
        F[ch] = a->Q > 0.0 ? a->P[ch] / a->Q : 0.0;
        C[ch] = a->T * bg[ch] + (1.0 - a->T) * F[ch];
    }
}

static int window_ok(const orc_window *win, const orc_camera *cam, orc_window *out)
{
    if (win) *out = *win;
    else { out->x0 = 0; out->y0 = 0; out->x1 = cam->width; out->y1 = cam->height; }
    if (out->x0 < 0) out->x0 = 0;
    if (out->y0 < 0) out->y0 = 0;
    if (out->x1 > cam->width) out->x1 = cam->width;
    if (out->y1 > cam->height) out->y1 = cam->height;
    return out->x1 > out->x0 && out->y1 > out->y0;
}

/*
 * Render one view.  Splat-major: every splat (in index order) visits the pixels of
 * its conservative footprint box (or every pixel of the window when `brute`), so
 * each pixel sums its contributions in splat-index order in both modes.
 *   include   [n] bytes or NULL: render only splats with include[i] != 0
 *   image     [3][H][W]   C inside the window (untouched outside)
 *   pixstate  [5][H][W]   T, Q, F_r, F_g, F_b   (may be NULL)
 *   pre       [9][H][W]   P0 (3), P1 (3), Q0, Q1, logT (may be NULL)
 *   near_mask [H][W]      set to 1 where some pair has |255 alpha_raw - 1| < near_margin
 */
int orc_render(const orc_splats *s, double sigma, const double bg[3], const orc_camera *cam,
               const unsigned char *include, int brute, const orc_window *win,
               double *image, double *pixstate, double *pre, unsigned char *near_mask,
               double near_margin, long long *n_pairs, unsigned long long *signature)
{
    orc_window wd;
    const long W = cam->width, H = cam->height, HW = W * H;
    if (!window_ok(win, cam, &wd)) return 0;
    const long ww = wd.x1 - wd.x0, wh = wd.y1 - wd.y0;
    orc_acc *acc = (orc_acc *)malloc(sizeof(orc_acc) * ww * wh);
    if (!acc) return -1;
    for (long k = 0; k < ww * wh; ++k) acc_init(&acc[k]);
    long long pairs = 0;
    uint64_t sig = 0;
    orc_proj p;
    for (long i = 0; i < s->n; ++i) {
        if (include && !include[i]) continue;
        project_splat(s, i, sigma, cam, &p);
        sig ^= splat_signature(&p, i);
        if (!p.valid) continue;
        int x0 = brute ? wd.x0 : (p.x0 > wd.x0 ? p.x0 : wd.x0);
        int x1 = brute ? wd.x1 : (p.x1 < wd.x1 ? p.x1 : wd.x1);
        int y0 = brute ? wd.y0 : (p.y0 > wd.y0 ? p.y0 : wd.y0);
        int y1 = brute ? wd.y1 : (p.y1 < wd.y1 ? p.y1 : wd.y1);
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) {
                double alpha, G, dx, dy, raw;
                int capped;
                int on = pair_alpha(&p, x + 0.5, y + 0.5, &alpha, &G, &dx, &dy, &capped, &raw);
                if (near_mask && fabs(raw / ORC_ALPHA_MIN - 1.0) < near_margin)
                    near_mask[(long)y * W + x] = 1;
                if (!on) continue;
                acc_add(&acc[(long)(y - wd.y0) * ww + (x - wd.x0)], &p, alpha);
                ++pairs;
                sig ^= mix64(((uint64_t)i << 32) ^ ((uint64_t)y << 16) ^ (uint64_t)x ^
                             ((uint64_t)capped << 63));
            }
    }
    for (int y = wd.y0; y < wd.y1; ++y)
        for (int x = wd.x0; x < wd.x1; ++x) {
            const orc_acc *a = &acc[(long)(y - wd.y0) * ww + (x - wd.x0)];
            const long px = (long)y * W + x;
            double C[3], F[3];
            acc_finish(a, bg, C, F);
            if (image)
                for (int ch = 0; ch < 3; ++ch) image[ch * HW + px] = C[ch];
            if (pixstate) {
                pixstate[0 * HW + px] = a->T;
                pixstate[1 * HW + px] = a->Q;
                for (int ch = 0; ch < 3; ++ch) pixstate[(2 + ch) * HW + px] = F[ch];
            }
            if (pre) {
                for (int ch = 0; ch < 3; ++ch) {
                    pre[ch * HW + px] = a->P0[ch];
                    pre[(3 + ch) * HW + px] = a->P1[ch];
                }
                pre[6 * HW + px] = a->Q0;
                pre[7 * HW + px] = a->Q1;
                pre[8 * HW + px] = a->logT;
            }
        }
    free(acc);
    if (n_pairs) *n_pairs = pairs;
    if (signature) *signature = sig;
    return 0;
}

/*
 * Render a list of pixels, pixel-major: each pixel loops over all splats in index
 * order (no footprint boxes).  out_C [npix][3], out_state [npix][5] (T, Q, F).
 */
int orc_render_pixels(const orc_splats *s, double sigma, const double bg[3],
                      const orc_camera *cam, long npix, const int *pxs, const int *pys,
                      double *out_C, double *out_state, long long *n_pairs)
{
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (s->n > 0 ? s->n : 1));
    if (!pr) return -1;
    for (long i = 0; i < s->n; ++i) project_splat(s, i, sigma, cam, &pr[i]);
    long long pairs = 0;
    for (long k = 0; k < npix; ++k) {
        orc_acc a;
        acc_init(&a);
        for (long i = 0; i < s->n; ++i) {
            if (!pr[i].valid) continue;
            double alpha, G, dx, dy, raw;
            int capped;
            if (!pair_alpha(&pr[i], pxs[k] + 0.5, pys[k] + 0.5, &alpha, &G, &dx, &dy, &capped, &raw))
                continue;
            acc_add(&a, &pr[i], alpha);
            ++pairs;
        }
        double C[3], F[3];
        acc_finish(&a, bg, C, F);
        for (int ch = 0; ch < 3; ++ch) out_C[3 * k + ch] = C[ch];
        if (out_state) {
            out_state[5 * k + 0] = a.T;
            out_state[5 * k + 1] = a.Q;
            for (int ch = 0; ch < 3; ++ch) out_state[5 * k + 2 + ch] = F[ch];
        }
    }
    free(pr);
    if (n_pairs) *n_pairs = pairs;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Backward                                                                     */
/* ------------------------------------------------------------------------- */

/* Screen-space gradient of one splat, summed over pixels. */
typedef struct {
    double mx, my;     /* dL/dmu' */
    double conic[4];   /* dL/d(conic entries), full 2x2 */
    double opacity;    /* dL/do */
    double color[3];   /* dL/dc */
    double w;          /* dL/dw */
} orc_sgrad;

/* Per-pixel state the backward needs: the totals of the forward pass. */
typedef struct { double T, Q, F[3]; } orc_pix;

/* Gradient contribution of one contributing pair (Eq. "oit_rendering_detail"). */
static void pair_backward(const orc_proj *p, const orc_pix *px, const double g[3], const double bg[3],
                          double alpha, double G, double dx, double dy, int capped, orc_sgrad *sg)
{
    const double T = px->T, Q = px->Q;
    double dL_dalpha = 0.0, dL_dw = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double F = px->F[ch];
        /* dC/dc_i = (1 - T) alpha_i w_i / Q */
        const double dC_dc = Q > 0.0 ? (1.0 - T) * alpha * p->w / Q : 0.0;
        /* dC/dalpha_i = T/(1 - alpha_i) (F - c0) + (1 - T) (w_i / Q) (c_i - F) */
        const double dC_dalpha = T / (1.0 - alpha) * (F - bg[ch]) +
                                 (Q > 0.0 ? (1.0 - T) * (p->w / Q) * (p->color[ch] - F) : 0.0);
        /* dC/dw_i = (1 - T) (alpha_i / Q) (c_i - F) */
        const double dC_dw = Q > 0.0 ? (1.0 - T) * (alpha / Q) * (p->color[ch] - F) : 0.0;
        sg->color[ch] += g[ch] * dC_dc;
        dL_dalpha += g[ch] * dC_dalpha;
        dL_dw += g[ch] * dC_dw;
    }
    sg->w += dL_dw;
    if (capped) return; /* alpha = 0.99 is constant there */
    /* alpha = o exp(-m/2),  m = d^T conic d,  d = x - mu' */
    sg->opacity += dL_dalpha * G;
    const double dL_dm = dL_dalpha * (-0.5 * alpha);
    sg->conic[0] += dL_dm * dx * dx;
    sg->conic[1] += dL_dm * dx * dy;
    sg->conic[2] += dL_dm * dy * dx;
    sg->conic[3] += dL_dm * dy * dy;
    sg->mx += dL_dm * (-(2.0 * p->conic[0] * dx + (p->conic[1] + p->conic[2]) * dy));
    sg->my += dL_dm * (-((p->conic[1] + p->conic[2]) * dx + 2.0 * p->conic[3] * dy));
}

/* Chain rule from the screen-space gradient of splat i to its parameters. */
static void splat_backward(const orc_splats *s, long i, double sigma, const orc_camera *cam,
                           const orc_proj *p, const orc_sgrad *sg, orc_grads *gr, double *g_sigma)
{
    const long n = s->n;
    const double *W = cam->R;
    double g_tc[3] = {0, 0, 0}, g_mu[3] = {0, 0, 0}, g_dir[3] = {0, 0, 0};

    /* opacity: o = sigmoid(logit) */
    gr->opacity_logit[i] += sg->opacity * p->opacity * (1.0 - p->opacity);

    /* weight: w = (1 - d/sigma) v for d < sigma, else 0 */
    double g_v = 0.0;
    if (p->w_on) {
        g_v = sg->w * (1.0 - p->d / sigma);
        g_tc[2] += sg->w * (-p->v / sigma);
        *g_sigma += sg->w * p->v * p->d / (sigma * sigma);
    }
    /* v = max(0, Y . vsh + 0.5) */
    if (p->raw_v > 0.0) {
        for (int k = 0; k < 16; ++k) {
            gr->vsh[(long)k * n + i] += g_v * p->Y[k];
            for (int a = 0; a < 3; ++a) g_dir[a] += g_v * s->vsh[(long)k * n + i] * p->dY[k][a];
        }
    }
    /* colour: c = max(0, Y . h + 0.5) per channel */
    for (int ch = 0; ch < 3; ++ch) {
        if (!(p->raw_c[ch] > 0.0)) continue;
        const double gc = sg->color[ch];
        for (int k = 0; k < 16; ++k) {
            gr->sh[((long)k * 3 + ch) * n + i] += gc * p->Y[k];
            for (int a = 0; a < 3; ++a) g_dir[a] += gc * s->sh[((long)k * 3 + ch) * n + i] * p->dY[k][a];
        }
    }
    /* dir = (mu - cc) / |mu - cc| */
    {
        double dd = g_dir[0] * p->dir[0] + g_dir[1] * p->dir[1] + g_dir[2] * p->dir[2];
        for (int a = 0; a < 3; ++a) g_mu[a] += (g_dir[a] - p->dir[a] * dd) / p->dist;
    }

    /* conic = cov^-1  =>  dL/dcov = -conic^T G conic^T */
    double g_cov[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l)
                    acc += p->conic[2 * k + a] * sg->conic[2 * k + l] * p->conic[2 * b + l];
            g_cov[2 * a + b] = -acc;
        }
    /* cov = T Sigma T^T + 0.3 I:
     *   dL/dT[a][b] = sum_jl G[a][j] T[j][l] Sigma[b][l] + sum_ik G[i][a] T[i][k] Sigma[k][b]
     *   dL/dSigma   = T^T G T */
    double g_T[6], g_Sigma[9];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int j = 0; j < 2; ++j)
                for (int l = 0; l < 3; ++l)
                    acc += g_cov[2 * a + j] * p->T[3 * j + l] * p->Sigma[3 * b + l] +
                           g_cov[2 * j + a] * p->T[3 * j + l] * p->Sigma[3 * l + b];
            g_T[3 * a + b] = acc;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l)
                    acc += p->T[3 * k + a] * g_cov[2 * k + l] * p->T[3 * l + b];
            g_Sigma[3 * a + b] = acc;
        }
    /* T = J W  =>  dL/dJ = dL/dT W^T */
    double g_J[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += g_T[3 * a + k] * W[3 * b + k];
            g_J[3 * a + b] = acc;
        }
    /* J entries as functions of the camera-space mean */
    {
        const double tz = p->tc[2], tz2 = tz * tz, tz3 = tz2 * tz;
        g_tc[2] += g_J[0] * (-cam->fx / tz2) + g_J[4] * (-cam->fy / tz2);
        if (p->clamp_x == 0) {
            g_tc[0] += g_J[2] * (-cam->fx / tz2);
            g_tc[2] += g_J[2] * (2.0 * cam->fx * p->tc[0] / tz3);
        } else { /* J02 = -fx lim / tz */
            g_tc[2] += g_J[2] * (cam->fx * (p->clamp_x * p->lim_x) / tz2);
        }
        if (p->clamp_y == 0) {
            g_tc[1] += g_J[5] * (-cam->fy / tz2);
            g_tc[2] += g_J[5] * (2.0 * cam->fy * p->tc[1] / tz3);
        } else {
            g_tc[2] += g_J[5] * (cam->fy * (p->clamp_y * p->lim_y) / tz2);
        }
        /* mu' = (fx tx/tz + cx, fy ty/tz + cy) */
        g_tc[0] += sg->mx * cam->fx / tz;
        g_tc[1] += sg->my * cam->fy / tz;
        g_tc[2] += -sg->mx * cam->fx * p->tc[0] / tz2 - sg->my * cam->fy * p->tc[1] / tz2;
    }
    /* tc = W mu + t */
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) g_mu[a] += W[3 * r + a] * g_tc[r];
    for (int a = 0; a < 3; ++a) gr->mean[(long)a * n + i] += g_mu[a];

    /* Sigma = M M^T with M = Rq diag(scale)  =>  dL/dM = (G + G^T) M */
    double M[9], g_M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = p->Rq[3 * a + b] * p->scale[b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += (g_Sigma[3 * a + k] + g_Sigma[3 * k + a]) * M[3 * k + b];
            g_M[3 * a + b] = acc;
        }
    double g_Rq[9];
    for (int b = 0; b < 3; ++b) {
        double gs = 0.0;
        for (int a = 0; a < 3; ++a) {
            gs += g_M[3 * a + b] * p->Rq[3 * a + b];
            g_Rq[3 * a + b] = g_M[3 * a + b] * p->scale[b];
        }
        gr->log_scale[(long)b * n + i] += gs * p->scale[b]; /* scale = exp(log_scale) */
    }
    /* Rq(q_hat): derivative of each entry by (w, x, y, z) */
    {
        const double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
        const double dR[9][4] = {
            {0.0, 0.0, -4.0 * y, -4.0 * z},
            {-2.0 * z, 2.0 * y, 2.0 * x, -2.0 * w},
            {2.0 * y, 2.0 * z, 2.0 * w, 2.0 * x},
            {2.0 * z, 2.0 * y, 2.0 * x, 2.0 * w},
            {0.0, -4.0 * x, 0.0, -4.0 * z},
            {-2.0 * x, -2.0 * w, 2.0 * z, 2.0 * y},
            {-2.0 * y, 2.0 * z, -2.0 * w, 2.0 * x},
            {2.0 * x, 2.0 * w, 2.0 * z, 2.0 * y},
            {0.0, -4.0 * x, -4.0 * y, 0.0},
        };
        double g_qn[4] = {0, 0, 0, 0};
        for (int e = 0; e < 9; ++e)
            for (int k = 0; k < 4; ++k) g_qn[k] += g_Rq[e] * dR[e][k];
        /* q_hat = q / |q| */
        double dd = 0.0;
        for (int k = 0; k < 4; ++k) dd += g_qn[k] * p->qn[k];
        for (int k = 0; k < 4; ++k) gr->quat[(long)k * n + i] += (g_qn[k] - p->qn[k] * dd) / p->qlen;
    }
}

/*
 * Gradient of L = sum_pixels sum_ch dLdC[ch][pixel] * C[ch][pixel] over the window,
 * for every splat parameter (added into `gr`) and for sigma (added into *g_sigma).
 * The forward totals T, Q, F are recomputed here over the full splat set.
 * screen [n][10] (optional): dL/dmu'x, dL/dmu'y, dL/dconic_xx, dL/dconic_xy (as the
 * one off-diagonal scalar), dL/dconic_yy, dL/do, dL/dc (3), dL/dw.
 */
int orc_backward(const orc_splats *s, double sigma, const double bg[3], const orc_camera *cam,
                 const orc_window *win, const double *dLdC, orc_grads *gr, double *g_sigma,
                 double *screen)
{
    orc_window wd;
    const long W = cam->width, H = cam->height, HW = W * H;
    if (!window_ok(win, cam, &wd)) return 0;
    double *state = (double *)calloc((size_t)5 * HW, sizeof(double));
    if (!state) return -1;
    orc_render(s, sigma, bg, cam, NULL, 0, &wd, NULL, state, NULL, NULL, 0.0, NULL, NULL);
    orc_proj p;
    double gsig = 0.0;
    for (long i = 0; i < s->n; ++i) {
        project_splat(s, i, sigma, cam, &p);
        orc_sgrad sg;
        memset(&sg, 0, sizeof(sg));
        if (p.valid) {
            int x0 = p.x0 > wd.x0 ? p.x0 : wd.x0, x1 = p.x1 < wd.x1 ? p.x1 : wd.x1;
            int y0 = p.y0 > wd.y0 ? p.y0 : wd.y0, y1 = p.y1 < wd.y1 ? p.y1 : wd.y1;
            for (int y = y0; y < y1; ++y)
                for (int x = x0; x < x1; ++x) {
                    double alpha, G, dx, dy, raw;
                    int capped;
                    if (!pair_alpha(&p, x + 0.5, y + 0.5, &alpha, &G, &dx, &dy, &capped, &raw)) continue;
                    const long px = (long)y * W + x;
                    orc_pix st;
                    st.T = state[px];
                    st.Q = state[HW + px];
                    for (int ch = 0; ch < 3; ++ch) st.F[ch] = state[(2 + ch) * HW + px];
                    double g[3] = {dLdC[px], dLdC[HW + px], dLdC[2 * HW + px]};
                    pair_backward(&p, &st, g, bg, alpha, G, dx, dy, capped, &sg);
                }
            splat_backward(s, i, sigma, cam, &p, &sg, gr, &gsig);
        }
        if (screen) {
            double *o = screen + 10 * i;
            o[0] = sg.mx; o[1] = sg.my; o[2] = sg.conic[0]; o[3] = sg.conic[1] + sg.conic[2];
            o[4] = sg.conic[3]; o[5] = sg.opacity;
            o[6] = sg.color[0]; o[7] = sg.color[1]; o[8] = sg.color[2]; o[9] = sg.w;
        }
    }
    *g_sigma += gsig;
    free(state);
    return 0;
}

/*
 * Same gradient with dLdC given only at a list of pixels (zero elsewhere):
 * pixel-major over all splats.  dLdC [npix][3]; screen [n][10] optional, as in
 * orc_backward.
 */
int orc_backward_pixels(const orc_splats *s, double sigma, const double bg[3], const orc_camera *cam,
                        long npix, const int *pxs, const int *pys, const double *dLdC,
                        orc_grads *gr, double *g_sigma, double *screen)
{
    const long n = s->n;
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (n > 0 ? n : 1));
    orc_sgrad *sg = (orc_sgrad *)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_sgrad));
    if (!pr || !sg) { free(pr); free(sg); return -1; }
    for (long i = 0; i < n; ++i) project_splat(s, i, sigma, cam, &pr[i]);
    for (long k = 0; k < npix; ++k) {
        const double px = pxs[k] + 0.5, py = pys[k] + 0.5;
        orc_acc a;
        acc_init(&a);
        for (long i = 0; i < n; ++i) {
            if (!pr[i].valid) continue;
            double alpha, G, dx, dy, raw;
            int capped;
            if (pair_alpha(&pr[i], px, py, &alpha, &G, &dx, &dy, &capped, &raw)) acc_add(&a, &pr[i], alpha);
        }
        double C[3];
        orc_pix st;
        acc_finish(&a, bg, C, st.F);
        st.T = a.T;
        st.Q = a.Q;
        const double *g = dLdC + 3 * k;
        for (long i = 0; i < n; ++i) {
            if (!pr[i].valid) continue;
            double alpha, G, dx, dy, raw;
            int capped;
            if (pair_alpha(&pr[i], px, py, &alpha, &G, &dx, &dy, &capped, &raw))
                pair_backward(&pr[i], &st, g, bg, alpha, G, dx, dy, capped, &sg[i]);
        }
    }
    double gsig = 0.0;
    for (long i = 0; i < n; ++i) {
        if (pr[i].valid) splat_backward(s, i, sigma, cam, &pr[i], &sg[i], gr, &gsig);
        if (screen) {
            double *o = screen + 10 * i;
            o[0] = sg[i].mx; o[1] = sg[i].my; o[2] = sg[i].conic[0]; o[3] = sg[i].conic[1] + sg[i].conic[2];
            o[4] = sg[i].conic[3]; o[5] = sg[i].opacity;
            o[6] = sg[i].color[0]; o[7] = sg[i].color[1]; o[8] = sg[i].color[2]; o[9] = sg[i].w;
        }
    }
    *g_sigma += gsig;
    free(pr);
    free(sg);
    return 0;
}
