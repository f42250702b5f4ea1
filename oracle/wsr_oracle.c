/*
 * Reference checker for sort-free Gaussian splatting via Weighted Sum Rendering.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation of
 * what the GPU path computes, written from the paper's definitions so that the
 * GPU kernels can be checked against it.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; no product code does.  It
 * shares no code, headers or tables with the GPU library.
 *
 * What it computes, per camera view (everything in double precision):
 *   - 3D Gaussian model (Sec. 3, Eq. 3): centre p, max opacity t (or the
 *     view-dependent opacity u of Sec. 4.3, Eq. 11), rotation q, scale s, SH H.
 *   - SH colour (Sec. 3, Eq. 4) evaluated at the unit view direction from the
 *     camera centre to the Gaussian (the printed argument is a norm, which
 *     cannot feed SH; the direction reading is recorded with the others).
 *   - EWA projection (Sec. 3, Eq. 5): Sigma2D = J W Sigma3D W^T J^T, plus a
 *     small dilation on the diagonal.
 *   - Depth weights (Sec. 4.2, Eqs. 8, 9, 10): DIR w = 1, EXP w = exp(-sigma
 *     d^beta), LC w = max(0, 1 - d/sigma) v_i.
 *   - Weighted sum rendering (Sec. 4.2, Eq. 7):
 *         C = (c_B w_B + sum_i c_i alpha_i w(d_i)) / (w_B + sum_i alpha_i w(d_i))
 *     summed over every visible Gaussian for every pixel (no tiling, no sort).
 *   - The analytic gradient of a loss L(C) with respect to every input, by the
 *     chain rule through each of the steps above.
 *
 * Readings of points the paper leaves open (support cutoff q <= tau, pixel
 * centres at +0.5, clamp of the projective Jacobian, near plane, +0.5 SH
 * offset, den == 0 convention) are listed in the project design notes; each
 * is also stated where it is used below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAX_K 16

/* ------------------------------------------------------------------------- */
/* Inputs                                                                    */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n;
    int32_t sh_degree;       /* 0..3 */
    int32_t opacity_mode;    /* 0: t = sigmoid(logit) (Sec. 3); 1: u = SH (Eq. 11) */
    const double *means;     /* [3][n] */
    const double *log_scales;/* [3][n] */
    const double *quats;     /* [4][n], (w, x, y, z) */
    const double *sh;        /* [K][n][4], RGBA */
    const double *opacity_logit; /* [n] */
    const double *lc_v;      /* [n] */
} ora_scene;

typedef struct {
    double viewmat[12];      /* row-major [R | T], world -> camera */
    double fx, fy, cx, cy;
    int32_t width, height;
    int32_t pad_[2];
} ora_camera;

typedef struct {
    int32_t weight_kind;     /* 0 DIR (Eq. 8), 1 EXP (Eq. 9), 2 LC (Eq. 10) */
    int32_t pad_;
    double sigma, beta;
    double w_bg, bg[3];
    double tau, dilation, near_z, opacity_offset;
    double alpha_cut;        /* opacity early-out (App. D): 0 = off */
    int32_t oit;             /* 1: weighted-blended OIT (Eq. 2) instead of Eq. 7 */
    int32_t pad2_;
} ora_params;

/* Per-Gaussian projected quantities exported for stage-wise checks.  Layout of
 * one row of ora_project's output (ORA_PROJ_STRIDE doubles):
 *  0 visible, 1-2 mu, 3-5 cov2d (a, b, c), 6-8 conic (A, B, C),
 *  9-11 rgb (clamped), 12 u, 13 w, 14 depth, 15-17 t (camera space),
 *  18-20 view direction, 21-23 rgb before the clamp, 24 support cutoff      */
#define ORA_PROJ_STRIDE 25

typedef struct {
    int visible;
    double t[3];
    double mu[2];
    double cov[3];
    double conic[3];
    double dir[3];
    double dist;
    double raw[3];
    double rgb[3];
    double u, w, depth;
    double cut;       /* pairs with q <= cut contribute (tau, or less with the early-out) */
    double u_mag;     /* magnitude of the terms of u: |offset| + sum_k |H_k Y_k| (SH opacity), or u */
    double Y[ORA_MAX_K];
} proj_t;

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics, orthonormal on the unit sphere, degrees 0..3.    */
/* Index k = l*l + l + m.  Written from the Cartesian form of the real SH:    */
/* m > 0 uses cos(m phi), m < 0 uses sin(|m| phi), times the associated       */
/* Legendre factor; on the unit sphere these are the polynomials below.       */
/* ------------------------------------------------------------------------- */

static void sh_basis(const double d[3], int degree, double *Y)
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = 3.14159265358979323846;
    Y[0] = 0.5 * sqrt(1.0 / pi);
    if (degree < 1) return;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = k1 * y;
    Y[2] = k1 * z;
    Y[3] = k1 * x;
    if (degree < 2) return;
    Y[4] = 0.5 * sqrt(15.0 / pi) * x * y;
    Y[5] = 0.5 * sqrt(15.0 / pi) * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    Y[7] = 0.5 * sqrt(15.0 / pi) * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    if (degree < 3) return;
    Y[9] = 0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = 0.25 * sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0);
    Y[13] = 0.25 * sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    Y[15] = 0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
}

/* Partial derivatives dY[k][j] = dY_k / d d_j of the polynomials above (the
 * polynomials are differentiated as functions of three free variables; the
 * radial component is removed later by the normalisation's Jacobian). */
static void sh_basis_grad(const double d[3], int degree, double dY[][3])
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < ORA_MAX_K; ++k) dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
    if (degree < 1) return;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    dY[1][1] = k1;
    dY[2][2] = k1;
    dY[3][0] = k1;
    if (degree < 2) return;
    const double a = 0.5 * sqrt(15.0 / pi);
    dY[4][0] = a * y; dY[4][1] = a * x;
    dY[5][1] = a * z; dY[5][2] = a * y;
    dY[6][2] = 0.25 * sqrt(5.0 / pi) * 6.0 * z;
    dY[7][0] = a * z; dY[7][2] = a * x;
    const double b = 0.25 * sqrt(15.0 / pi);
    dY[8][0] = b * 2.0 * x; dY[8][1] = -b * 2.0 * y;
    if (degree < 3) return;
    const double c9 = 0.25 * sqrt(35.0 / (2.0 * pi));
    dY[9][0] = c9 * 6.0 * x * y;
    dY[9][1] = c9 * (3.0 * x * x - 3.0 * y * y);
    const double c10 = 0.5 * sqrt(105.0 / pi);
    dY[10][0] = c10 * y * z; dY[10][1] = c10 * x * z; dY[10][2] = c10 * x * y;
    const double c11 = 0.25 * sqrt(21.0 / (2.0 * pi));
    dY[11][1] = c11 * (5.0 * z * z - 1.0);
    dY[11][2] = c11 * y * 10.0 * z;
    const double c12 = 0.25 * sqrt(7.0 / pi);
    dY[12][2] = c12 * (15.0 * z * z - 3.0);
    dY[13][0] = c11 * (5.0 * z * z - 1.0);
    dY[13][2] = c11 * x * 10.0 * z;
    const double c14 = 0.25 * sqrt(105.0 / pi);
    dY[14][0] = c14 * 2.0 * x * z;
    dY[14][1] = -c14 * 2.0 * y * z;
    dY[14][2] = c14 * (x * x - y * y);
    dY[15][0] = c9 * (3.0 * x * x - 3.0 * y * y);
    dY[15][1] = -c9 * 6.0 * x * y;
}

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* ------------------------------------------------------------------------- */
/* Forward: one Gaussian in one view                                          */
/* ------------------------------------------------------------------------- */

static void project_one(const ora_scene *S, const ora_camera *cam, const ora_params *P,
                        int64_t i, proj_t *o)
{
    const int64_t n = S->n;
    memset(o, 0, sizeof(*o));
    const double *V = cam->viewmat;
    const double p[3] = {S->means[i], S->means[n + i], S->means[2 * n + i]};
    /* view transform (the matrix W of Eq. 5 is its rotation part) */
    for (int r = 0; r < 3; ++r)
        o->t[r] = V[4 * r] * p[0] + V[4 * r + 1] * p[1] + V[4 * r + 2] * p[2] + V[4 * r + 3];
    const double tx = o->t[0], ty = o->t[1], tz = o->t[2];
    o->depth = tz;
    if (!(tz > P->near_z)) return;  /* frustum cull at the near plane */

    /* Sigma3D = R(q) diag(s^2) R(q)^T */
    double q[4] = {S->quats[i], S->quats[n + i], S->quats[2 * n + i], S->quats[3 * n + i]};
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0.0)) return;
    for (int k = 0; k < 4; ++k) q[k] /= qn;
    double Rq[9];
    quat_to_rot(q, Rq);
    const double s[3] = {exp(S->log_scales[i]), exp(S->log_scales[n + i]),
                         exp(S->log_scales[2 * n + i])};
    double Sig3[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int l = 0; l < 3; ++l) acc += Rq[3 * a + l] * s[l] * s[l] * Rq[3 * b + l];
            Sig3[3 * a + b] = acc;
        }

    /* Jacobian of the pinhole projection, lateral ratio clamped to 1.3x the
     * half field of view */
    const double limx = 1.3 * 0.5 * cam->width / cam->fx;
    const double limy = 1.3 * 0.5 * cam->height / cam->fy;
    const double rx = clampd(tx / tz, -limx, limx);
    const double ry = clampd(ty / tz, -limy, limy);
    const double J[6] = {cam->fx / tz, 0.0, -cam->fx * rx / tz,
                         0.0, cam->fy / tz, -cam->fy * ry / tz};
    double Tm[6]; /* J W */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            Tm[3 * r + c] = J[3 * r] * V[c] + J[3 * r + 1] * V[4 + c] + J[3 * r + 2] * V[8 + c];
    double cov[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc += Tm[3 * r + a] * Sig3[3 * a + b] * Tm[3 * c + b];
            cov[2 * r + c] = acc;
        }
    o->cov[0] = cov[0] + P->dilation;
    o->cov[1] = cov[1];
    o->cov[2] = cov[3] + P->dilation;
    const double det = o->cov[0] * o->cov[2] - o->cov[1] * o->cov[1];
    if (!(det > 0.0)) return;
    o->conic[0] = o->cov[2] / det;
    o->conic[1] = -o->cov[1] / det;
    o->conic[2] = o->cov[0] / det;
    o->mu[0] = cam->fx * tx / tz + cam->cx;
    o->mu[1] = cam->fy * ty / tz + cam->cy;

    /* view direction from the camera centre f = -R^T T to the Gaussian */
    double f[3];
    for (int c = 0; c < 3; ++c)
        f[c] = -(V[c] * V[3] + V[4 + c] * V[7] + V[8 + c] * V[11]);
    double dv[3] = {p[0] - f[0], p[1] - f[1], p[2] - f[2]};
    o->dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int c = 0; c < 3; ++c) o->dir[c] = dv[c] / o->dist;

    const int K = (S->sh_degree + 1) * (S->sh_degree + 1);
    sh_basis(o->dir, S->sh_degree, o->Y);
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += S->sh[(k * n + i) * 4 + c] * o->Y[k];
        if (c < 3) {
            o->raw[c] = acc + 0.5;
            o->rgb[c] = o->raw[c] > 0.0 ? o->raw[c] : 0.0;
        } else if (S->opacity_mode == 1) {
            o->u = acc + P->opacity_offset; /* view-dependent opacity, not clamped */
            o->u_mag = fabs(P->opacity_offset);
            for (int k = 0; k < K; ++k) o->u_mag += fabs(S->sh[(k * n + i) * 4 + c] * o->Y[k]);
        }
    }
    if (S->opacity_mode == 0) o->u = o->u_mag = 1.0 / (1.0 + exp(-S->opacity_logit[i]));

    if (P->weight_kind == 0) {
        o->w = 1.0;
    } else if (P->weight_kind == 1) {
        o->w = exp(-P->sigma * pow(tz, P->beta));
    } else {
        const double lin = 1.0 - tz / P->sigma;
        o->w = (lin > 0.0 ? lin : 0.0) * S->lc_v[i];
    }
    /* Opacity early-out, the heuristic App. D proposes as future work (off
     * with alpha_cut = 0): a pair contributes only while its opacity
     * u exp(-q/2) is at least alpha_cut, i.e. q <= 2 ln(u / alpha_cut); a
     * Gaussian with u <= alpha_cut never does. */
    o->cut = P->tau;
    if (P->alpha_cut > 0.0) {
        if (!(o->u > P->alpha_cut)) return;
        const double c = 2.0 * log(o->u / P->alpha_cut);
        if (c < o->cut) o->cut = c;
    }
    o->visible = 1;
}

void ora_project(const ora_scene *S, const ora_camera *cam, const ora_params *P, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i) {
        proj_t g;
        project_one(S, cam, P, i, &g);
        double *r = out + i * ORA_PROJ_STRIDE;
        memset(r, 0, sizeof(double) * ORA_PROJ_STRIDE);
        r[0] = g.visible;
        r[14] = g.depth;
        for (int c = 0; c < 3; ++c) r[15 + c] = g.t[c];
        if (!g.visible) continue;
        r[1] = g.mu[0]; r[2] = g.mu[1];
        for (int c = 0; c < 3; ++c) {
            r[3 + c] = g.cov[c];
            r[6 + c] = g.conic[c];
            r[9 + c] = g.rgb[c];
            r[18 + c] = g.dir[c];
            r[21 + c] = g.raw[c];
        }
        r[12] = g.u; r[13] = g.w;
        r[24] = g.cut;
    }
}

/* The SH basis and the quaternion rotation on their own, so that the tests can
 * pin them against independent library routines. */
void ora_sh_basis(const double *dirs, int64_t m, int32_t degree, double *out)
{
    for (int64_t j = 0; j < m; ++j) {
        double Y[ORA_MAX_K] = {0};
        sh_basis(dirs + 3 * j, degree, Y);
        memcpy(out + j * ORA_MAX_K, Y, sizeof(Y));
    }
}

void ora_quat_to_rot(const double *quats, int64_t m, double *out)
{
    for (int64_t j = 0; j < m; ++j) {
        double q[4];
        const double *s = quats + 4 * j;
        const double nq = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
        for (int k = 0; k < 4; ++k) q[k] = s[k] / nq;
        quat_to_rot(q, out + 9 * j);
    }
}

/* ------------------------------------------------------------------------- */
/* Pixel window helpers                                                      */
/* ------------------------------------------------------------------------- */

/* Pixel-centre range [lo, hi] (inclusive) whose centres px + 0.5 lie within
 * the exact bounding box of the ellipse q <= tau, widened by a hair so that
 * rounding never drops a pixel the strict all-pairs loop would accept. */
static void support_box(const proj_t *g, double tau, int64_t out[4])
{
    const double rx = sqrt(tau * g->cov[0]) * (1.0 + 1e-9) + 1e-9;
    const double ry = sqrt(tau * g->cov[2]) * (1.0 + 1e-9) + 1e-9;
    out[0] = (int64_t)ceil(g->mu[0] - rx - 0.5);
    out[1] = (int64_t)floor(g->mu[0] + rx - 0.5);
    out[2] = (int64_t)ceil(g->mu[1] - ry - 0.5);
    out[3] = (int64_t)floor(g->mu[1] + ry - 0.5);
}

static double pair_q(const proj_t *g, int64_t px, int64_t py)
{
    const double dx = (double)px + 0.5 - g->mu[0];
    const double dy = (double)py + 0.5 - g->mu[1];
    return g->conic[0] * dx * dx + 2.0 * g->conic[1] * dx * dy + g->conic[2] * dy * dy;
}

typedef struct {
    proj_t *g;        /* projected Gaussians of the ones that are visible */
    int64_t *idx;     /* their indices in the scene */
    int64_t *box;     /* [m][4] support boxes */
    int64_t m;
} vis_t;

/* Project every Gaussian and keep the visible ones whose support box meets
 * the pixel window [x0, x1) x [y0, y1).  Skipping the others changes nothing:
 * outside its box a Gaussian has q > tau at every pixel centre. */
static void collect_visible(const ora_scene *S, const ora_camera *cam, const ora_params *P,
                            int64_t x0, int64_t y0, int64_t x1, int64_t y1, vis_t *v)
{
    const int64_t n = S->n;
    proj_t *all = (proj_t *)malloc(sizeof(proj_t) * (n > 0 ? n : 1));
    unsigned char *keep = (unsigned char *)calloc(n > 0 ? n : 1, 1);
    int64_t *boxes = (int64_t *)malloc(sizeof(int64_t) * 4 * (n > 0 ? n : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        project_one(S, cam, P, i, &all[i]);
        if (!all[i].visible) continue;
        support_box(&all[i], all[i].cut, boxes + 4 * i);
        const int64_t *b = boxes + 4 * i;
        keep[i] = (b[1] >= x0 && b[0] < x1 && b[3] >= y0 && b[2] < y1);
    }
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) m += keep[i];
    v->m = m;
    v->g = (proj_t *)malloc(sizeof(proj_t) * (m > 0 ? m : 1));
    v->idx = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    v->box = (int64_t *)malloc(sizeof(int64_t) * 4 * (m > 0 ? m : 1));
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i)
        if (keep[i]) {
            v->g[j] = all[i];
            v->idx[j] = i;
            memcpy(v->box + 4 * j, boxes + 4 * i, 4 * sizeof(int64_t));
            ++j;
        }
    free(all);
    free(keep);
    free(boxes);
}

static void free_visible(vis_t *v)
{
    free(v->g);
    free(v->idx);
    free(v->box);
}

/* ------------------------------------------------------------------------- */
/* Forward render                                                            */
/* ------------------------------------------------------------------------- */

/* Test support, not part of the method: how far q can move when the
 * centre is rounded to float32 relative to a frame origin within pos_h of
 * the pixel centre (a relative error of at most 2^-24 of |d| + pos_h per
 * axis): |dq/dmu_x| (|dx| + pos_h) 2^-24 + |dq/dmu_y| (|dy| + pos_h) 2^-24.
 * Zero when pos_h <= 0. */
static double amb_pos_window(const proj_t *g, double dx, double dy, double pos_h)
{
    if (pos_h <= 0.0) return 0.0;
    const double gx = 2.0 * fabs(g->conic[0] * dx + g->conic[1] * dy);
    const double gy = 2.0 * fabs(g->conic[1] * dx + g->conic[2] * dy);
    return ldexp(gx * (fabs(dx) + pos_h) + gy * (fabs(dy) + pos_h), -24);
}

/*
 * Render the pixel window [x0, x1) x [y0, y1) of one view with Eq. 7.
 *   mode 0 ("strict"): every pixel is tested against every Gaussian in the
 *          window list (the window list only drops Gaussians whose exact
 *          ellipse box misses the window);
 *   mode 1 ("aabb"): every Gaussian only visits the pixels of its own box.
 * Both visit exactly the pairs with q <= cut (cut = tau unless the opacity
 * early-out lowers it, see project_one); they differ in summation order.
 * Outputs, each [h][w] row-major with h = y1-y0, w = x1-x0:
 *   out_C [h][w][3]   colour; den == 0 gives the background colour
 *   out_num [h][w][3] numerator including c_B w_B
 *   out_den [h][w]    denominator including w_B
 *   out_amb [h][w]    sum of |a| over the pairs whose support decision a
 *                     float32 evaluation of q may flip:
 *                     |q - cut| <= eta * M + amb_pos_window(..., pos_h)
 *                     (+ cut_window(g) where the early-out lowers the
 *                     cutoff below tau, see there)
 *                     with M = A dx^2 + 2|B dx dy| + C dy^2, the magnitude of
 *                     the terms q sums (rounding error scales with M, not q,
 *                     because the terms cancel for elongated splats); pos_h
 *                     > 0 adds the effect of a centre rounded in float32
 *                     relative to a point within pos_h of the pixel centre
 *   out_ambc [h][w]   sum over those pairs of |a| * max_c |rgb_c - C_c|
 *   out_absden [h][w] |w_B| + sum of |a| over pairs with q <= tau (with den,
 *                     the conditioning of the normalisation)
 *   out_cnt [h][w]    number of pairs with q <= tau
 * Any output pointer may be NULL.
 */
/* Where the early-out lowers a Gaussian's cutoff below tau, the renderer
 * evaluates u and 2 ln(u / alpha_cut) in double precision, then rounds the
 * cutoff to float32 once and multiplies it by a float32 constant (the scale
 * its q carries too): each rounding moves it by at most 2^-24 of its size,
 * so the cutoff it compares with lies within 2^-23 |cut| of the exact one.
 * The second term bounds the difference of two double-precision
 * evaluations of u (2^-38 of the magnitude of its terms, relative to u,
 * orders of magnitude above double rounding). */
static double cut_window(const proj_t *g)
{
    return 0x1p-23 * fabs(g->cut) + 0x1p-38 * (1.0 + g->u_mag / fabs(g->u));
}

void ora_render(const ora_scene *S, const ora_camera *cam, const ora_params *P,
                int64_t x0, int64_t y0, int64_t x1, int64_t y1, int32_t mode, double eta, double pos_h,
                double *out_C, double *out_num, double *out_den, double *out_amb,
                double *out_ambc, double *out_absden, int64_t *out_cnt)
{
    const int64_t w = x1 - x0, h = y1 - y0;
    if (w <= 0 || h <= 0) return;
    vis_t v;
    collect_visible(S, cam, P, x0, y0, x1, y1, &v);
    double *num = (double *)calloc(w * h * 3, sizeof(double));
    double *den = (double *)calloc(w * h, sizeof(double));
    double *aden = (double *)calloc(w * h, sizeof(double));
    double *cov = (double *)malloc(sizeof(double) * w * h);  /* OIT: prod (1 - alpha) */
    for (int64_t o = 0; o < w * h; ++o) cov[o] = 1.0;
    int64_t *cnt = (int64_t *)calloc(w * h, sizeof(int64_t));
    const double tau = P->tau;

    if (mode == 0) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t yy = 0; yy < h; ++yy)
            for (int64_t xx = 0; xx < w; ++xx) {
                double nr = 0, ng = 0, nb = 0, dd = 0, ad = 0, pc = 1.0;
                int64_t c = 0;
                for (int64_t j = 0; j < v.m; ++j) {
                    const proj_t *g = &v.g[j];
                    const double q = pair_q(g, x0 + xx, y0 + yy);
                    if (q <= g->cut) {
                        const double G = exp(-0.5 * q);
                        const double a = g->u * g->w * G;
                        nr += a * g->rgb[0];
                        ng += a * g->rgb[1];
                        nb += a * g->rgb[2];
                        dd += a;
                        ad += fabs(a);
                        pc *= 1.0 - clampd(g->u * G, 0.0, 1.0);
                        ++c;
                    }
                }
                const int64_t o = yy * w + xx;
                cov[o] = pc;
                num[3 * o] = nr; num[3 * o + 1] = ng; num[3 * o + 2] = nb;
                den[o] = dd;
                aden[o] = ad;
                cnt[o] = c;
            }
    } else {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t yy = 0; yy < h; ++yy) {
            const int64_t py = y0 + yy;
            for (int64_t j = 0; j < v.m; ++j) {
                const int64_t *b = v.box + 4 * j;
                if (py < b[2] || py > b[3]) continue;
                const proj_t *g = &v.g[j];
                const int64_t lo = b[0] > x0 ? b[0] : x0;
                const int64_t hi = b[1] < x1 - 1 ? b[1] : x1 - 1;
                for (int64_t px = lo; px <= hi; ++px) {
                    const double q = pair_q(g, px, py);
                    if (q <= g->cut) {
                        const double G = exp(-0.5 * q);
                        const double a = g->u * g->w * G;
                        const int64_t o = yy * w + (px - x0);
                        cov[o] *= 1.0 - clampd(g->u * G, 0.0, 1.0);
                        num[3 * o] += a * g->rgb[0];
                        num[3 * o + 1] += a * g->rgb[1];
                        num[3 * o + 2] += a * g->rgb[2];
                        den[o] += a;
                        aden[o] += fabs(a);
                        cnt[o] += 1;
                    }
                }
            }
        }
    }

    /* background term and normalisation */
    double *Cimg = (double *)malloc(sizeof(double) * w * h * 3);
    for (int64_t o = 0; o < w * h; ++o) {
        if (P->oit) {
            /* Eq. 2 with c_0 = c_B: coverage-weighted blend of the weighted
             * average over the background (no w_B term).  The average takes
             * Eq. 7's amplitudes u w G with the unclamped opacity of Sec. 4.3
             * (num, den); the coverage takes alpha = u G clamped to [0, 1]
             * (cov), so that it stays a transmittance.  Eq. 2 has one alpha
             * in both places; the two coincide for opacities in [0, 1]. */
            const double D = den[o];
            for (int c = 0; c < 3; ++c) {
                const double avg = (D != 0.0) ? num[3 * o + c] / D : 0.0;
                Cimg[3 * o + c] = cov[o] * P->bg[c] + (1.0 - cov[o]) * avg;
                if (out_num) out_num[3 * o + c] = num[3 * o + c];
                if (out_C) out_C[3 * o + c] = Cimg[3 * o + c];
            }
            if (out_den) out_den[o] = D;
            if (out_absden) out_absden[o] = aden[o];
            if (out_cnt) out_cnt[o] = cnt[o];
            continue;
        }
        const double D = P->w_bg + den[o];
        double N3[3];
        for (int c = 0; c < 3; ++c) N3[c] = P->bg[c] * P->w_bg + num[3 * o + c];
        for (int c = 0; c < 3; ++c) {
            Cimg[3 * o + c] = (D != 0.0) ? N3[c] / D : P->bg[c];
            if (out_num) out_num[3 * o + c] = N3[c];
            if (out_C) out_C[3 * o + c] = Cimg[3 * o + c];
        }
        if (out_den) out_den[o] = D;
        if (out_absden) out_absden[o] = fabs(P->w_bg) + aden[o];
        if (out_cnt) out_cnt[o] = cnt[o];
    }

    if (out_amb || out_ambc) {
        /* pairs whose support decision is within eta*M of the cutoff (plus the
         * float error of a computed early-out cutoff) */
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t yy = 0; yy < h; ++yy)
            for (int64_t xx = 0; xx < w; ++xx) {
                const int64_t o = yy * w + xx;
                double sa = 0.0, sc = 0.0;
                for (int64_t j = 0; j < v.m; ++j) {
                    const proj_t *g = &v.g[j];
                    const double q = pair_q(g, x0 + xx, y0 + yy);
                    const double dx = (double)(x0 + xx) + 0.5 - g->mu[0];
                    const double dy = (double)(y0 + yy) + 0.5 - g->mu[1];
                    const double M = g->conic[0] * dx * dx + 2.0 * fabs(g->conic[1] * dx * dy) +
                                     g->conic[2] * dy * dy;
                    const double win = eta * M + amb_pos_window(g, dx, dy, pos_h) +
                                       (g->cut < tau ? cut_window(g) : 0.0);
                    if (fabs(q - g->cut) <= win) {
                        const double a = fabs(g->u * g->w * exp(-0.5 * q));
                        double md = 0.0;
                        for (int c = 0; c < 3; ++c) {
                            const double d = fabs(g->rgb[c] - Cimg[3 * o + c]);
                            md = d > md ? d : md;
                        }
                        sa += a;
                        sc += a * md;
                    }
                }
                if (out_amb) out_amb[o] = sa;
                if (out_ambc) out_ambc[o] = sc;
            }
    }
    free(Cimg);
    free(num);
    free(den);
    free(aden);
    free(cov);
    free(cnt);
    free_visible(&v);
}

/* ------------------------------------------------------------------------- */
/* Backward                                                                  */
/* ------------------------------------------------------------------------- */

/*
 * Gradient of L with respect to every input, given dL/dC over the pixel window
 * (pixels outside the window contribute nothing).  Output arrays are
 * overwritten:
 *   g_means [3][n], g_log_scales [3][n], g_quats [4][n], g_sh [K][n][4],
 *   g_logit [n], g_lc_v [n],
 *   g_globals [6] = dL/d(sigma, beta, w_bg, bg_r, bg_g, bg_b),
 *   g2d [n][9] = dL/d(mu_x, mu_y, A, B, C, r, g, b, a_scale) where (A, B, C)
 *       are the conic entries (q = A dx^2 + 2 B dx dy + C dy^2) and
 *       a_scale = u * w is the per-Gaussian amplitude; may be NULL.
 */
void ora_render_bwd(const ora_scene *S, const ora_camera *cam, const ora_params *P,
                    int64_t x0, int64_t y0, int64_t x1, int64_t y1, const double *dL_dC,
                    double *g_means, double *g_log_scales, double *g_quats, double *g_sh,
                    double *g_logit, double *g_lc_v, double *g_globals, double *g2d)
{
    const int64_t n = S->n;
    const int K = (S->sh_degree + 1) * (S->sh_degree + 1);
    memset(g_means, 0, sizeof(double) * 3 * n);
    memset(g_log_scales, 0, sizeof(double) * 3 * n);
    memset(g_quats, 0, sizeof(double) * 4 * n);
    memset(g_sh, 0, sizeof(double) * K * n * 4);
    memset(g_logit, 0, sizeof(double) * n);
    memset(g_lc_v, 0, sizeof(double) * n);
    memset(g_globals, 0, sizeof(double) * 6);
    if (g2d) memset(g2d, 0, sizeof(double) * 9 * n);
    const int64_t w = x1 - x0, h = y1 - y0;
    if (w <= 0 || h <= 0 || n == 0) return;

    vis_t v;
    collect_visible(S, cam, P, x0, y0, x1, y1, &v);

    /* pass 1: per-pixel sums, colour, and the two per-pixel factors of the
     * gradient: gbar_c = g_c / den and s = sum_c gbar_c C_c */
    double *gbar = (double *)calloc(w * h * 3, sizeof(double));
    double *sfac = (double *)calloc(w * h, sizeof(double));
    /* OIT (Eq. 2): k = P sum_c g_c (c_B,c - avg_c), so that the coverage term
     * gives dL/dalpha_i = -k / (1 - alpha_i) */
    double *kfac = (double *)calloc(w * h, sizeof(double));
    double bgw[4] = {0, 0, 0, 0}; /* dL/dbg_rgb, dL/dw_bg */
    #pragma omp parallel
    {
        double loc[4] = {0, 0, 0, 0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t yy = 0; yy < h; ++yy)
            for (int64_t xx = 0; xx < w; ++xx) {
                const double wb = P->oit ? 0.0 : P->w_bg;
                double N3[3] = {P->bg[0] * wb, P->bg[1] * wb, P->bg[2] * wb};
                double D = wb, pc = 1.0;
                for (int64_t j = 0; j < v.m; ++j) {
                    const proj_t *g = &v.g[j];
                    const double q = pair_q(g, x0 + xx, y0 + yy);
                    if (q <= g->cut) {
                        const double G = exp(-0.5 * q);
                        const double a = g->u * g->w * G;
                        for (int c = 0; c < 3; ++c) N3[c] += a * g->rgb[c];
                        D += a;
                        pc *= 1.0 - clampd(g->u * G, 0.0, 1.0);
                    }
                }
                const int64_t o = yy * w + xx;
                const double *gc = dL_dC + 3 * o;
                if (P->oit) {
                    /* C = P c_B + (1 - P) N / D: dC/dN = (1 - P) / D,
                     * dC/dD = -(1 - P) N / D^2, dC/dP = c_B - N / D */
                    double avg[3], s = 0.0, kk = 0.0;
                    for (int c = 0; c < 3; ++c) avg[c] = (D != 0.0) ? N3[c] / D : 0.0;
                    for (int c = 0; c < 3; ++c) {
                        gbar[3 * o + c] = (D != 0.0) ? gc[c] * (1.0 - pc) / D : 0.0;
                        s += gbar[3 * o + c] * avg[c];
                        kk += gc[c] * (P->bg[c] - avg[c]);
                        loc[c] += gc[c] * pc;
                    }
                    sfac[o] = s;
                    kfac[o] = pc * kk;
                } else if (D != 0.0) {
                    double s = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        gbar[3 * o + c] = gc[c] / D;
                        s += gbar[3 * o + c] * (N3[c] / D);
                    }
                    sfac[o] = s;
                    /* C = (bg w_bg + N) / (w_bg + D') */
                    for (int c = 0; c < 3; ++c) {
                        loc[c] += gbar[3 * o + c] * P->w_bg;
                        loc[3] += gbar[3 * o + c] * P->bg[c];
                    }
                    loc[3] -= s;
                } else {
                    /* den == 0: C is defined as the background colour */
                    for (int c = 0; c < 3; ++c) loc[c] += gc[c];
                }
            }
        #pragma omp critical
        for (int c = 0; c < 4; ++c) bgw[c] += loc[c];
    }
    g_globals[2] = bgw[3];
    g_globals[3] = bgw[0];
    g_globals[4] = bgw[1];
    g_globals[5] = bgw[2];

    /* pass 2: per Gaussian, sum the per-pair gradients over the pixels of its
     * box, then chain back to the 3D parameters */
    double *gsig = (double *)calloc(v.m > 0 ? v.m : 1, sizeof(double));
    double *gbeta = (double *)calloc(v.m > 0 ? v.m : 1, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < v.m; ++j) {
        const proj_t *g = &v.g[j];
        const int64_t i = v.idx[j];
        const int64_t *b = v.box + 4 * j;
        double dmu[2] = {0, 0}, dcon[3] = {0, 0, 0}, drgb[3] = {0, 0, 0}, das = 0.0, du_cov = 0.0;
        const double as = g->u * g->w;
        const int64_t ylo = b[2] > y0 ? b[2] : y0, yhi = b[3] < y1 - 1 ? b[3] : y1 - 1;
        const int64_t xlo = b[0] > x0 ? b[0] : x0, xhi = b[1] < x1 - 1 ? b[1] : x1 - 1;
        for (int64_t py = ylo; py <= yhi; ++py)
            for (int64_t px = xlo; px <= xhi; ++px) {
                const double q = pair_q(g, px, py);
                if (!(q <= g->cut)) continue;
                const int64_t o = (py - y0) * w + (px - x0);
                const double G = exp(-0.5 * q);
                const double a = as * G;
                const double *gb = gbar + 3 * o;
                const double dLda = gb[0] * g->rgb[0] + gb[1] * g->rgb[1] + gb[2] * g->rgb[2] - sfac[o];
                for (int c = 0; c < 3; ++c) drgb[c] += a * gb[c];
                das += dLda * G;
                double dq = -0.5 * a * dLda;
                if (P->oit) {
                    /* alpha = u G, clamped to [0, 1] (no gradient where clamped) */
                    const double al = g->u * G;
                    if (al > 0.0 && al < 1.0) {
                        const double dLdal = -kfac[o] / (1.0 - al);
                        du_cov += G * dLdal;
                        dq += -0.5 * g->u * G * dLdal;
                    }
                }
                const double dx = (double)px + 0.5 - g->mu[0];
                const double dy = (double)py + 0.5 - g->mu[1];
                dmu[0] += -dq * (2.0 * g->conic[0] * dx + 2.0 * g->conic[1] * dy);
                dmu[1] += -dq * (2.0 * g->conic[1] * dx + 2.0 * g->conic[2] * dy);
                dcon[0] += dq * dx * dx;
                dcon[1] += dq * 2.0 * dx * dy;
                dcon[2] += dq * dy * dy;
            }
        if (g2d) {
            double *r = g2d + 9 * i;
            r[0] = dmu[0]; r[1] = dmu[1];
            r[2] = dcon[0]; r[3] = dcon[1]; r[4] = dcon[2];
            r[5] = drgb[0]; r[6] = drgb[1]; r[7] = drgb[2];
            r[8] = das;
        }

        /* ---- amplitude a_scale = u * w ---- */
        const double du = das * g->w + du_cov;
        const double dw = das * g->u;
        double ddir[3] = {0, 0, 0};
        double dY[ORA_MAX_K][3];
        sh_basis_grad(g->dir, S->sh_degree, dY);
        if (S->opacity_mode == 0) {
            g_logit[i] = du * g->u * (1.0 - g->u);
        } else {
            for (int k = 0; k < K; ++k) {
                g_sh[(k * n + i) * 4 + 3] = du * g->Y[k];
                const double h3 = S->sh[(k * n + i) * 4 + 3];
                for (int c = 0; c < 3; ++c) ddir[c] += du * h3 * dY[k][c];
            }
        }
        /* ---- colour, clamp at zero (derivative 0 where the argument <= 0) ---- */
        for (int c = 0; c < 3; ++c) {
            if (!(g->raw[c] > 0.0)) continue;
            for (int k = 0; k < K; ++k) {
                g_sh[(k * n + i) * 4 + c] = drgb[c] * g->Y[k];
                const double hc = S->sh[(k * n + i) * 4 + c];
                for (int e = 0; e < 3; ++e) ddir[e] += drgb[c] * hc * dY[k][e];
            }
        }
        /* ---- depth weight ---- */
        double dt[3] = {0, 0, 0};
        const double d = g->depth;
        if (P->weight_kind == 1) {
            const double db = pow(d, P->beta);
            gsig[j] = dw * (-db * g->w);
            gbeta[j] = dw * (-P->sigma * db * log(d) * g->w);
            dt[2] += dw * (-P->sigma * P->beta * pow(d, P->beta - 1.0) * g->w);
        } else if (P->weight_kind == 2) {
            const double lin = 1.0 - d / P->sigma;
            if (lin > 0.0) {
                const double v_i = S->lc_v[i];
                g_lc_v[i] = dw * lin;
                gsig[j] = dw * v_i * d / (P->sigma * P->sigma);
                dt[2] += dw * (-v_i / P->sigma);
            }
        }
        /* ---- direction: dir = (p - f) / |p - f| ---- */
        double dp[3];
        const double proj = ddir[0] * g->dir[0] + ddir[1] * g->dir[1] + ddir[2] * g->dir[2];
        for (int c = 0; c < 3; ++c) dp[c] = (ddir[c] - g->dir[c] * proj) / g->dist;

        /* ---- mean: mu = (fx tx/tz + cx, fy ty/tz + cy) ---- */
        const double tx = g->t[0], ty = g->t[1], tz = g->t[2];
        const double fx = cam->fx, fy = cam->fy;
        dt[0] += dmu[0] * fx / tz;
        dt[1] += dmu[1] * fy / tz;
        dt[2] += -(dmu[0] * fx * tx + dmu[1] * fy * ty) / (tz * tz);

        /* ---- conic = inverse of (a b; b c) ---- */
        const double ca = g->cov[0], cb = g->cov[1], cc = g->cov[2];
        const double det = ca * cc - cb * cb, det2 = det * det;
        const double dA = dcon[0], dB = dcon[1], dC = dcon[2];
        const double da = dA * (-cc * cc / det2) + dB * (cb * cc / det2) + dC * (1.0 / det - ca * cc / det2);
        const double dbv = dA * (2.0 * cb * cc / det2) + dB * (-1.0 / det - 2.0 * cb * cb / det2) +
                           dC * (2.0 * ca * cb / det2);
        const double dc = dA * (1.0 / det - ca * cc / det2) + dB * (ca * cb / det2) + dC * (-ca * ca / det2);

        /* recompute the forward pieces needed by the chain */
        const double *V = cam->viewmat;
        double q[4] = {S->quats[i], S->quats[n + i], S->quats[2 * n + i], S->quats[3 * n + i]};
        const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double qh[4];
        for (int k = 0; k < 4; ++k) qh[k] = q[k] / qn;
        double Rq[9];
        quat_to_rot(qh, Rq);
        const double s[3] = {exp(S->log_scales[i]), exp(S->log_scales[n + i]),
                             exp(S->log_scales[2 * n + i])};
        double M[9], Sig3[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int l = 0; l < 3; ++l) acc += M[3 * r + l] * M[3 * c + l];
                Sig3[3 * r + c] = acc;
            }
        const double limx = 1.3 * 0.5 * cam->width / fx;
        const double limy = 1.3 * 0.5 * cam->height / fy;
        const double rxu = tx / tz, ryu = ty / tz;
        const int clx = (rxu < -limx || rxu > limx), cly = (ryu < -limy || ryu > limy);
        const double rx = clampd(rxu, -limx, limx), ry = clampd(ryu, -limy, limy);
        const double J[6] = {fx / tz, 0.0, -fx * rx / tz, 0.0, fy / tz, -fy * ry / tz};
        double Tm[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                Tm[3 * r + c] = J[3 * r] * V[c] + J[3 * r + 1] * V[4 + c] + J[3 * r + 2] * V[8 + c];

        /* a = T0 S T0^T, b = T0 S T1^T, c = T1 S T1^T */
        double ST0[3], ST1[3];
        for (int r = 0; r < 3; ++r) {
            ST0[r] = Sig3[3 * r] * Tm[0] + Sig3[3 * r + 1] * Tm[1] + Sig3[3 * r + 2] * Tm[2];
            ST1[r] = Sig3[3 * r] * Tm[3] + Sig3[3 * r + 1] * Tm[4] + Sig3[3 * r + 2] * Tm[5];
        }
        double dTm[6], dSig3[9];
        for (int c = 0; c < 3; ++c) {
            dTm[c] = 2.0 * da * ST0[c] + dbv * ST1[c];
            dTm[3 + c] = dbv * ST0[c] + 2.0 * dc * ST1[c];
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                dSig3[3 * r + c] = da * Tm[r] * Tm[c] + dbv * Tm[r] * Tm[3 + c] + dc * Tm[3 + r] * Tm[3 + c];
        /* Tm = J W  ->  dJ = dTm W^T */
        double dJ[6];
        for (int r = 0; r < 2; ++r)
            for (int l = 0; l < 3; ++l)
                dJ[3 * r + l] = dTm[3 * r] * V[4 * l] + dTm[3 * r + 1] * V[4 * l + 1] + dTm[3 * r + 2] * V[4 * l + 2];
        dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[4] * (-fy / (tz * tz));
        if (!clx) {
            /* J02 = -fx tx / tz^2 */
            dt[0] += dJ[2] * (-fx / (tz * tz));
            dt[2] += dJ[2] * (2.0 * fx * tx / (tz * tz * tz));
        } else {
            /* J02 = -fx rx / tz with rx held at the clamp */
            dt[2] += dJ[2] * (fx * rx / (tz * tz));
        }
        if (!cly) {
            dt[1] += dJ[5] * (-fy / (tz * tz));
            dt[2] += dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
        } else {
            dt[2] += dJ[5] * (fy * ry / (tz * tz));
        }
        /* t = W p + T  ->  dp += W^T dt */
        for (int c = 0; c < 3; ++c) dp[c] += V[c] * dt[0] + V[4 + c] * dt[1] + V[8 + c] * dt[2];
        for (int c = 0; c < 3; ++c) g_means[c * n + i] = dp[c];

        /* Sigma3 = M M^T  ->  dM = (dS + dS^T) M */
        double dM[9];
        for (int r = 0; r < 3; ++r)
            for (int l = 0; l < 3; ++l) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += (dSig3[3 * r + k] + dSig3[3 * k + r]) * M[3 * k + l];
                dM[3 * r + l] = acc;
            }
        /* M = R diag(s) */
        double dR[9];
        for (int r = 0; r < 3; ++r)
            for (int l = 0; l < 3; ++l) dR[3 * r + l] = dM[3 * r + l] * s[l];
        for (int l = 0; l < 3; ++l) {
            double ds = 0.0;
            for (int r = 0; r < 3; ++r) ds += dM[3 * r + l] * Rq[3 * r + l];
            g_log_scales[l * n + i] = ds * s[l];
        }
        /* rotation entries -> unit quaternion (w, x, y, z) */
        const double qw = qh[0], qx = qh[1], qy = qh[2], qz = qh[3];
        double dqh[4];
        dqh[0] = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
        dqh[1] = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - qw * dR[5] +
                        qz * dR[6] + qw * dR[7] - 2.0 * qx * dR[8]);
        dqh[2] = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] -
                        qw * dR[6] + qz * dR[7] - 2.0 * qy * dR[8]);
        dqh[3] = 2.0 * (-2.0 * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.0 * qz * dR[4] +
                        qy * dR[5] + qx * dR[6] + qy * dR[7]);
        /* normalisation q / |q| */
        const double dot = dqh[0] * qh[0] + dqh[1] * qh[1] + dqh[2] * qh[2] + dqh[3] * qh[3];
        for (int k = 0; k < 4; ++k) g_quats[k * n + i] = (dqh[k] - qh[k] * dot) / qn;
    }
    double ssig = 0.0, sbeta = 0.0;
    for (int64_t j = 0; j < v.m; ++j) {
        ssig += gsig[j];
        sbeta += gbeta[j];
    }
    g_globals[0] = ssig;
    g_globals[1] = sbeta;
    free(gsig);
    free(gbeta);
    free(gbar);
    free(sfac);
    free(kfac);
    free_visible(&v);
}

/* ------------------------------------------------------------------------- */
/* Sorted alpha blending (Eq. 6): the compositing the method removes the      */
/* sort from.  Not part of Eq. 7; a baseline rendered from the same splats.   */
/* ------------------------------------------------------------------------- */

typedef struct {
    double depth;
    int64_t index;     /* scene index: ties in depth keep index order */
    double alpha;
    const proj_t *g;
} layer_t;

static int layer_cmp(const void *a, const void *b)
{
    const layer_t *x = (const layer_t *)a, *y = (const layer_t *)b;
    if (x->depth < y->depth) return -1;
    if (x->depth > y->depth) return 1;
    return (x->index > y->index) - (x->index < y->index);
}

/*
 * Per pixel of the window: the Gaussians with q <= tau, front to back
 * (ascending camera depth t_z, ties by scene index), each with opacity
 * alpha_i = min(alpha_max, u_i exp(-q/2)) where u_i is the Gaussian's
 * opacity (no depth weight: Eq. 6 has none); layers with alpha_i < alpha_min
 * are skipped.  With T_i = prod_{j<i} (1 - alpha_j):
 *     C = sum_i c_i alpha_i T_i + T c_B,   T = the transmittance after the last layer,
 * and composition stops after the layer that takes T below t_min (t_min = 0:
 * never).  Outputs: out_C [h][w][3], out_T [h][w] the final transmittance,
 * out_amb [h][w] the sum of alpha over layers whose support decision is within
 * the window of ora_render of the cutoff.  Any output may be NULL.
 */
void ora_render_sorted(const ora_scene *S, const ora_camera *cam, const ora_params *P,
                       int64_t x0, int64_t y0, int64_t x1, int64_t y1, double alpha_max,
                       double alpha_min, double t_min, double eta, double pos_h,
                       double *out_C, double *out_T, double *out_amb)
{
    const int64_t w = x1 - x0, h = y1 - y0;
    if (w <= 0 || h <= 0) return;
    vis_t v;
    collect_visible(S, cam, P, x0, y0, x1, y1, &v);
    const double tau = P->tau;
    #pragma omp parallel
    {
        layer_t *lay = (layer_t *)malloc(sizeof(layer_t) * (v.m > 0 ? v.m : 1));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t yy = 0; yy < h; ++yy)
            for (int64_t xx = 0; xx < w; ++xx) {
                int64_t k = 0;
                double amb = 0.0;
                for (int64_t j = 0; j < v.m; ++j) {
                    const proj_t *g = &v.g[j];
                    const double q = pair_q(g, x0 + xx, y0 + yy);
                    const double dx = (double)(x0 + xx) + 0.5 - g->mu[0];
                    const double dy = (double)(y0 + yy) + 0.5 - g->mu[1];
                    const double M = g->conic[0] * dx * dx + 2.0 * fabs(g->conic[1] * dx * dy) +
                                     g->conic[2] * dy * dy;
                    double a = g->u * exp(-0.5 * q);
                    if (a > alpha_max) a = alpha_max;
                    if (fabs(q - tau) <= eta * M + amb_pos_window(g, dx, dy, pos_h)) amb += fabs(a);
                    if (q > tau || a < alpha_min) continue;
                    lay[k].depth = g->depth;
                    lay[k].index = v.idx[j];
                    lay[k].alpha = a;
                    lay[k].g = g;
                    ++k;
                }
                qsort(lay, (size_t)k, sizeof(layer_t), layer_cmp);
                double T = 1.0, c3[3] = {0.0, 0.0, 0.0};
                for (int64_t i = 0; i < k; ++i) {
                    const double a = lay[i].alpha;
                    for (int c = 0; c < 3; ++c) c3[c] += lay[i].g->rgb[c] * a * T;
                    T *= 1.0 - a;
                    if (T < t_min) break;
                }
                const int64_t o = yy * w + xx;
                for (int c = 0; c < 3; ++c)
                    if (out_C) out_C[3 * o + c] = c3[c] + T * P->bg[c];
                if (out_T) out_T[o] = T;
                if (out_amb) out_amb[o] = amb;
            }
        free(lay);
    }
    free_visible(&v);
}

int32_t ora_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
