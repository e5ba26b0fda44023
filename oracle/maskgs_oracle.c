/*
 * FP64 CPU oracle for masked rasterization of 3D Gaussians (MaskGaussian,
 * arXiv 2412.20522).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  It shares no code, header, table or constant
 * generator with the HIP kernels and is used only by the tests, by the smoke
 * check and by the benchmark's CPU-baseline leg.  It is never on the product
 * path.
 *
 * Every floating-point quantity is computed in double precision; inputs are
 * taken as doubles (the FP32 parameters of the GPU path widen exactly), so
 * finite differences in FP64 are meaningful.  Where the method is an exact computation
 * (compositing, its gradients) the code below is the plain definition written
 * out, per pixel, with per-pixel lists held in memory.
 *
 * Sections and what they follow:
 *   activations, 3D covariance, EWA splat, SH colour  -- Sec. 3.1 (a 3D
 *       Gaussian with centre p, opacity o, scales s, quaternion q and SH is
 *       splatted to a 2D Gaussian; alpha_i = o_i * G2D_i(x)).  The exponent
 *       uses the inverse of the 2D covariance (the printed formula omits the
 *       inverse; read as the standard EWA conic).
 *   tile lists and depth order  -- Sec. 3.1 (16x16 tiles, only Gaussians
 *       that intersect the tile and pass the alpha filter take part, in depth
 *       order).
 *   masked forward compositing  -- Eq. (3)-(4), plus the background term of
 *       the supplementary derivation (final transmittance times c_bg).
 *   masked backward compositing -- Eq. (6) with b read as the colour behind
 *       entry i relative to T_{i+1} (the recursion of the supplementary
 *       material), plus the background term derived there; gradients for the
 *       mask reach every entry that passed the alpha filter, whatever its
 *       mask (Sec. 3.3-3.4, Fig. 1 caption).
 *   mask sampling, mask loss    -- Sec. 3.3 (two scores, Gumbel-Softmax),
 *       Eq. (7)-(8).
 *   random numbers -- Philox4x32-10, Salmon, Moraes, Dror and Shaw,
 *       "Parallel random numbers: as easy as 1, 2, 3", SC'11.
 *   optimiser -- Adam, Kingma and Ba, ICLR 2015 (the paper trains with the
 *       3DGS optimiser and does not restate it).
 *
 * Parity pins live in the test suite (closed forms, invariants, finite
 * differences, a dense brute-force reference, SH orthonormality by
 * quadrature, Philox known-answer vectors).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* inputs shared with the Python side through ctypes                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    float viewmat[16]; /* world -> camera, row-major, camera +z forward */
    float fx, fy, cx, cy;
    int32_t width, height;
} orc_camera;

typedef struct {
    int32_t tile_w, tile_h;
    int32_t sh_degree;
    int32_t exact_mode;  /* 1: no alpha_min, no T_min, no Q cut, every valid
                            Gaussian in every tile */
    float alpha_min;     /* 1/255 */
    float alpha_max;     /* 0.99  */
    float t_min;         /* 1e-4  */
    float q_max;         /* 9     */
    float near_plane;    /* 0.2   */
    float dilation;      /* 0.3   */
    float jac_clamp;     /* 1.3   */
    float lambda_floor;  /* 0.1   */
    float bg[3];
    float margin;        /* relative margin for the Q / alpha decision flags, 1e-5 */
    float margin_t;      /* relative margin for the transmittance stop flag, 2e-4
                            (an FP32 transmittance carries a relative rounding
                            error that grows with the number of blended entries) */
} orc_settings;

/* flag bits per pixel */
#define ORC_FLAG_Q     1u
#define ORC_FLAG_AMIN  2u
#define ORC_FLAG_AMAX  4u
#define ORC_FLAG_TMIN  8u

static double eff_alpha_min(const orc_settings* st) { return st->exact_mode ? 0.0 : (double)st->alpha_min; }
static double eff_t_min(const orc_settings* st) { return st->exact_mode ? 0.0 : (double)st->t_min; }
static double eff_q_max(const orc_settings* st) { return st->exact_mode ? INFINITY : (double)st->q_max; }

/* ------------------------------------------------------------------------ */
/* small dense linear algebra, row-major                                     */
/* ------------------------------------------------------------------------ */

static void mat_mul(const double* a, const double* b, double* c, int m, int k, int n) {
    /* c[m x n] = a[m x k] * b[k x n] */
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) {
            double s = 0.0;
            for (int t = 0; t < k; t++) s += a[i * k + t] * b[t * n + j];
            c[i * n + j] = s;
        }
}

static void mat_transpose(const double* a, double* at, int m, int n) {
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) at[j * m + i] = a[i * n + j];
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics, generic in degree                              */
/*                                                                          */
/* For a unit direction (x, y, z) with polar angle theta (cos theta = z) and */
/* azimuth phi, the real SH of degree l and order m are                     */
/*   m = 0 : K(l,0) P_l^0(z)                                                */
/*   m > 0 : sqrt(2) K(l,m) cos(m phi) P_l^m(z)                             */
/*   m < 0 : sqrt(2) K(l,|m|) sin(|m| phi) P_l^|m|(z)                       */
/* with K(l,m) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m the associated */
/* Legendre functions without the Condon-Shortley phase.  Writing           */
/* P_l^m(z) = sin^m(theta) D_l^m(z) and sin^m(theta) e^{i m phi} = (x+iy)^m  */
/* gives a polynomial in (x, y, z) that equals Y on the unit sphere; its    */
/* gradient, projected onto the tangent plane, is the gradient of Y.        */
/* D follows the standard three-term recurrence in l.                        */
/* Index of (l, m) is l*l + l + m.                                          */
/* ------------------------------------------------------------------------ */

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= (double)i;
    return f;
}

/* values[k], grads[k][3] for k < (deg+1)^2; grads may be NULL */
static void sh_basis(int deg, const double dir[3], double* values, double (*grads)[3]) {
    const double x = dir[0], y = dir[1], z = dir[2];
    /* A_m + i B_m = (x + i y)^m and their partials in x, y */
    double A[4], B[4], Ax[4], Ay[4], Bx[4], By[4];
    A[0] = 1.0; B[0] = 0.0; Ax[0] = Ay[0] = Bx[0] = By[0] = 0.0;
    for (int m = 0; m < deg; m++) {
        A[m + 1] = x * A[m] - y * B[m];
        B[m + 1] = x * B[m] + y * A[m];
        Ax[m + 1] = A[m] + x * Ax[m] - y * Bx[m];
        Ay[m + 1] = -B[m] + x * Ay[m] - y * By[m];
        Bx[m + 1] = B[m] + x * Bx[m] + y * Ax[m];
        By[m + 1] = A[m] + x * By[m] + y * Ay[m];
    }
    for (int m = 0; m <= deg; m++) {
        /* D_l^m(z) for l = m..deg and dD/dz */
        double D[4] = {0, 0, 0, 0}, Dz[4] = {0, 0, 0, 0};
        double dfact = 1.0; /* (2m-1)!! */
        for (int i = 1; i <= 2 * m - 1; i += 2) dfact *= (double)i;
        D[m] = dfact;
        Dz[m] = 0.0;
        if (m + 1 <= deg) {
            D[m + 1] = (2.0 * m + 1.0) * z * D[m];
            Dz[m + 1] = (2.0 * m + 1.0) * D[m];
        }
        for (int l = m + 2; l <= deg; l++) {
            D[l] = ((2.0 * l - 1.0) * z * D[l - 1] - (double)(l + m - 1) * D[l - 2]) / (double)(l - m);
            Dz[l] = ((2.0 * l - 1.0) * (D[l - 1] + z * Dz[l - 1]) - (double)(l + m - 1) * Dz[l - 2]) /
                    (double)(l - m);
        }
        for (int l = m; l <= deg; l++) {
            const double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            if (m == 0) {
                const int idx = l * l + l;
                values[idx] = K * D[l];
                if (grads) { grads[idx][0] = 0.0; grads[idx][1] = 0.0; grads[idx][2] = K * Dz[l]; }
            } else {
                const double c = sqrt(2.0) * K;
                const int ip = l * l + l + m, in = l * l + l - m;
                values[ip] = c * A[m] * D[l];
                values[in] = c * B[m] * D[l];
                if (grads) {
                    grads[ip][0] = c * Ax[m] * D[l];
                    grads[ip][1] = c * Ay[m] * D[l];
                    grads[ip][2] = c * A[m] * Dz[l];
                    grads[in][0] = c * Bx[m] * D[l];
                    grads[in][1] = c * By[m] * D[l];
                    grads[in][2] = c * B[m] * Dz[l];
                }
            }
        }
    }
}

ORC_API void orc_sh_basis(int deg, int64_t n, const double* dirs, double* values, double* grads) {
    const int k = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; i++)
        sh_basis(deg, dirs + 3 * i, values + k * i, grads ? (double (*)[3])(grads + 3 * k * i) : NULL);
}

/* ------------------------------------------------------------------------ */
/* projection: activations, 3D covariance, view transform, EWA, SH colour   */
/* ------------------------------------------------------------------------ */

static void quat_rotation(const double q[4], double R[9]) {
    /* unit quaternion (w, x, y, z) -> rotation matrix */
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* derivative of the rotation matrix entries w.r.t. each quaternion component */
static void quat_rotation_partials(const double q[4], double dR[4][9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    const double dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    const double dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    const double dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    memcpy(dR[0], dw, sizeof dw);
    memcpy(dR[1], dx, sizeof dx);
    memcpy(dR[2], dy, sizeof dy);
    memcpy(dR[3], dz, sizeof dz);
}

typedef struct {
    int valid;
    double s[3], qn[4], qnorm, o;
    double Rq[9], Sigma3[9];
    double W[9], tvec[3];
    double t[3];
    float depth_f;
    double sx, sy; int clamp_x, clamp_y; /* clamped t_x/t_z and t_y/t_z */
    double J[6], T[6];
    double cov2[3];  /* a, b, c of the 2D covariance (dilated) */
    double det;
    double conic[3];
    double radius;
    double u, v;
    double campos[3], dirv[3], dnorm, dir[3];
    double color[3];
    int cclamp[3];
} orc_proj_state;

static void load_view(const orc_camera* cam, double W[9], double tvec[3]) {
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) W[3 * i + j] = (double)cam->viewmat[4 * i + j];
        tvec[i] = (double)cam->viewmat[4 * i + 3];
    }
}

/* Forward projection of one Gaussian for one camera, all in FP64. */
static void project_one(const double* mean, const double* log_scale, const double* quat, double opacity_logit,
                        const double* sh, int deg, const orc_camera* cam, const orc_settings* st,
                        orc_proj_state* ps) {
    memset(ps, 0, sizeof *ps);
    /* activations */
    for (int i = 0; i < 3; i++) ps->s[i] = exp(log_scale[i]);
    double qq = 0.0;
    for (int i = 0; i < 4; i++) qq += quat[i] * quat[i];
    ps->qnorm = sqrt(qq);
    for (int i = 0; i < 4; i++) ps->qn[i] = quat[i] / ps->qnorm;
    ps->o = 1.0 / (1.0 + exp(-opacity_logit));
    /* 3D covariance R diag(s^2) R^T */
    quat_rotation(ps->qn, ps->Rq);
    {
        double RS[9], RSt[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) RS[3 * i + j] = ps->Rq[3 * i + j] * ps->s[j];
        mat_transpose(RS, RSt, 3, 3);
        mat_mul(RS, RSt, ps->Sigma3, 3, 3, 3);
    }
    /* view transform; the depth key is the fp32 rounding of the FP64 z */
    load_view(cam, ps->W, ps->tvec);
    const double px = mean[0], py = mean[1], pz = mean[2];
    for (int i = 0; i < 3; i++)
        ps->t[i] = ((ps->W[3 * i + 0] * px + ps->W[3 * i + 1] * py) + ps->W[3 * i + 2] * pz) + ps->tvec[i];
    ps->depth_f = (float)ps->t[2];
    if (!((double)ps->depth_f > (double)st->near_plane)) { ps->valid = 0; return; }
    const double fx = cam->fx, fy = cam->fy;
    const double tx = ps->t[0], ty = ps->t[1], tz = ps->t[2];
    ps->u = fx * tx / tz + (double)cam->cx;
    ps->v = fy * ty / tz + (double)cam->cy;
    /* Jacobian of the perspective map, with the lateral ratio clamped */
    const double limx = (double)st->jac_clamp * (0.5 * (double)cam->width / fx);
    const double limy = (double)st->jac_clamp * (0.5 * (double)cam->height / fy);
    double rx = tx / tz, ry = ty / tz;
    ps->clamp_x = (rx < -limx || rx > limx);
    ps->clamp_y = (ry < -limy || ry > limy);
    ps->sx = rx < -limx ? -limx : (rx > limx ? limx : rx);
    ps->sy = ry < -limy ? -limy : (ry > limy ? limy : ry);
    ps->J[0] = fx / tz; ps->J[1] = 0.0;      ps->J[2] = -fx * ps->sx / tz;
    ps->J[3] = 0.0;     ps->J[4] = fy / tz;  ps->J[5] = -fy * ps->sy / tz;
    mat_mul(ps->J, ps->W, ps->T, 2, 3, 3);
    {
        double TS[6], Tt[6], C2[4];
        mat_mul(ps->T, ps->Sigma3, TS, 2, 3, 3);
        mat_transpose(ps->T, Tt, 2, 3);
        mat_mul(TS, Tt, C2, 2, 3, 2);
        ps->cov2[0] = C2[0] + (double)st->dilation;
        ps->cov2[1] = C2[1];
        ps->cov2[2] = C2[3] + (double)st->dilation;
    }
    ps->det = ps->cov2[0] * ps->cov2[2] - ps->cov2[1] * ps->cov2[1];
    if (!(ps->det > 0.0)) { ps->valid = 0; return; }
    ps->conic[0] = ps->cov2[2] / ps->det;
    ps->conic[1] = -ps->cov2[1] / ps->det;
    ps->conic[2] = ps->cov2[0] / ps->det;
    {
        const double mid = 0.5 * (ps->cov2[0] + ps->cov2[2]);
        double disc = mid * mid - ps->det;
        if (disc < (double)st->lambda_floor) disc = (double)st->lambda_floor;
        const double lmax = mid + sqrt(disc);
        ps->radius = ceil(3.0 * sqrt(lmax));
    }
    if (!(ps->radius > 0.0)) { ps->valid = 0; return; }
    /* colour from SH in the viewing direction (camera centre -> Gaussian) */
    {
        double Wt[9];
        mat_transpose(ps->W, Wt, 3, 3);
        for (int i = 0; i < 3; i++)
            ps->campos[i] = -(Wt[3 * i + 0] * ps->tvec[0] + Wt[3 * i + 1] * ps->tvec[1] + Wt[3 * i + 2] * ps->tvec[2]);
        ps->dirv[0] = px - ps->campos[0];
        ps->dirv[1] = py - ps->campos[1];
        ps->dirv[2] = pz - ps->campos[2];
        ps->dnorm = sqrt(ps->dirv[0] * ps->dirv[0] + ps->dirv[1] * ps->dirv[1] + ps->dirv[2] * ps->dirv[2]);
        for (int i = 0; i < 3; i++) ps->dir[i] = ps->dirv[i] / ps->dnorm;
        double Y[16];
        sh_basis(deg, ps->dir, Y, NULL);
        const int K = (deg + 1) * (deg + 1);
        for (int ch = 0; ch < 3; ch++) {
            double c = 0.5;
            for (int k = 0; k < K; k++) c += sh[3 * k + ch] * Y[k];
            ps->cclamp[ch] = c < 0.0;
            ps->color[ch] = c < 0.0 ? 0.0 : c;
        }
    }
    ps->valid = 1;
}

/* Outputs of the forward projection for n Gaussians and one camera. */
ORC_API void orc_project_fwd(int64_t n, const double* means, const double* log_scales, const double* quats,
                             const double* opacity_logits, const double* sh, const orc_camera* cam,
                             const orc_settings* st, double* mean2d, uint32_t* depth_bits, double* conic,
                             double* cov2d, double* radius, double* opacity, double* color, uint8_t* cclamp,
                             uint8_t* valid) {
    const int deg = st->sh_degree, K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        orc_proj_state ps;
        project_one(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opacity_logits[i], sh + 3 * K * i, deg, cam,
                    st, &ps);
        float df = ps.depth_f;
        uint32_t bits;
        memcpy(&bits, &df, 4);
        depth_bits[i] = bits;
        valid[i] = (uint8_t)ps.valid;
        mean2d[2 * i] = ps.u;
        mean2d[2 * i + 1] = ps.v;
        for (int c = 0; c < 3; c++) {
            conic[3 * i + c] = ps.conic[c];
            cov2d[3 * i + c] = ps.cov2[c];
            color[3 * i + c] = ps.color[c];
            cclamp[3 * i + c] = (uint8_t)ps.cclamp[c];
        }
        radius[i] = ps.radius;
        opacity[i] = ps.o;
        if (!ps.valid) {
            radius[i] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* tiles touched, tile lists in (tile, depth, id) order, tile ranges        */
/* ------------------------------------------------------------------------ */

static void tile_rect(double u, double v, double r, int gw, int gh, const orc_settings* st, int rect[4]) {
    if (st->exact_mode) {
        rect[0] = 0; rect[1] = 0; rect[2] = gw - 1; rect[3] = gh - 1;
        return;
    }
    double x0 = floor((u - r) / st->tile_w), x1 = floor((u + r) / st->tile_w);
    double y0 = floor((v - r) / st->tile_h), y1 = floor((v + r) / st->tile_h);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > gw - 1) x1 = gw - 1;
    if (y1 > gh - 1) y1 = gh - 1;
    if (x0 > x1 || y0 > y1) { rect[0] = 1; rect[1] = 1; rect[2] = 0; rect[3] = 0; return; }
    rect[0] = (int)x0; rect[1] = (int)y0; rect[2] = (int)x1; rect[3] = (int)y1;
}

typedef struct { uint32_t depth_bits; uint32_t id; } orc_entry;

static int entry_cmp(const void* a, const void* b) {
    const orc_entry* x = (const orc_entry*)a;
    const orc_entry* y = (const orc_entry*)b;
    if (x->depth_bits != y->depth_bits) return x->depth_bits < y->depth_bits ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

static int grid_w(const orc_settings* st, int w) { return (w + st->tile_w - 1) / st->tile_w; }
static int grid_h(const orc_settings* st, int h) { return (h + st->tile_h - 1) / st->tile_h; }

ORC_API int64_t orc_total_tiles(int n_views, const int32_t* widths, const int32_t* heights, const orc_settings* st) {
    int64_t t = 0;
    for (int v = 0; v < n_views; v++) t += (int64_t)grid_w(st, widths[v]) * grid_h(st, heights[v]);
    return t;
}

/*
 * Per (view, Gaussian) record r = view * n + g.  Computes tiles touched for
 * each record; when keys != NULL also writes the sorted instance list
 * (key = global tile << 32 | depth bits, value = record) and per-tile
 * [start, end) ranges.  Returns K, the number of instances.
 */
ORC_API int64_t orc_build_lists(int n_views, int64_t n, const int32_t* widths, const int32_t* heights,
                                const double* mean2d, const double* radius, const uint32_t* depth_bits,
                                const uint8_t* valid, const orc_settings* st, int64_t* tiles_touched,
                                uint64_t* keys, uint32_t* vals, int64_t k_cap, uint32_t* ranges) {
    const int64_t total_tiles = orc_total_tiles(n_views, widths, heights, st);
    int64_t* tile_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_views + 1));
    tile_off[0] = 0;
    for (int v = 0; v < n_views; v++)
        tile_off[v + 1] = tile_off[v] + (int64_t)grid_w(st, widths[v]) * grid_h(st, heights[v]);
    int64_t K = 0;
    for (int v = 0; v < n_views; v++) {
        const int gw = grid_w(st, widths[v]), gh = grid_h(st, heights[v]);
        for (int64_t g = 0; g < n; g++) {
            const int64_t r = (int64_t)v * n + g;
            int64_t cnt = 0;
            if (valid[r]) {
                int rect[4];
                tile_rect(mean2d[2 * r], mean2d[2 * r + 1], radius[r], gw, gh, st, rect);
                if (rect[0] <= rect[2] && rect[1] <= rect[3])
                    cnt = (int64_t)(rect[2] - rect[0] + 1) * (rect[3] - rect[1] + 1);
            }
            tiles_touched[r] = cnt;
            K += cnt;
        }
    }
    if (keys == NULL) { free(tile_off); return K; }
    if (K > k_cap) { free(tile_off); return -1; }
    /* bucket instances by global tile, then order each bucket */
    int64_t* bstart = (int64_t*)calloc((size_t)total_tiles + 1, sizeof(int64_t));
    for (int v = 0; v < n_views; v++) {
        const int gw = grid_w(st, widths[v]), gh = grid_h(st, heights[v]);
        for (int64_t g = 0; g < n; g++) {
            const int64_t r = (int64_t)v * n + g;
            if (!tiles_touched[r]) continue;
            int rect[4];
            tile_rect(mean2d[2 * r], mean2d[2 * r + 1], radius[r], gw, gh, st, rect);
            for (int ty = rect[1]; ty <= rect[3]; ty++)
                for (int tx = rect[0]; tx <= rect[2]; tx++) bstart[tile_off[v] + (int64_t)ty * gw + tx + 1]++;
        }
    }
    for (int64_t t = 0; t < total_tiles; t++) bstart[t + 1] += bstart[t];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)total_tiles);
    for (int64_t t = 0; t < total_tiles; t++) fill[t] = bstart[t];
    orc_entry* ent = (orc_entry*)malloc(sizeof(orc_entry) * (size_t)(K > 0 ? K : 1));
    for (int v = 0; v < n_views; v++) {
        const int gw = grid_w(st, widths[v]), gh = grid_h(st, heights[v]);
        for (int64_t g = 0; g < n; g++) {
            const int64_t r = (int64_t)v * n + g;
            if (!tiles_touched[r]) continue;
            int rect[4];
            tile_rect(mean2d[2 * r], mean2d[2 * r + 1], radius[r], gw, gh, st, rect);
            for (int ty = rect[1]; ty <= rect[3]; ty++)
                for (int tx = rect[0]; tx <= rect[2]; tx++) {
                    const int64_t t = tile_off[v] + (int64_t)ty * gw + tx;
                    ent[fill[t]].depth_bits = depth_bits[r];
                    ent[fill[t]].id = (uint32_t)r;
                    fill[t]++;
                }
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < total_tiles; t++) {
        const int64_t s = bstart[t], e = bstart[t + 1];
        if (e - s > 1) qsort(ent + s, (size_t)(e - s), sizeof(orc_entry), entry_cmp);
        for (int64_t i = s; i < e; i++) {
            keys[i] = ((uint64_t)t << 32) | ent[i].depth_bits;
            vals[i] = ent[i].id;
        }
        ranges[2 * t] = (uint32_t)s;
        ranges[2 * t + 1] = (uint32_t)e;
    }
    free(ent);
    free(fill);
    free(bstart);
    free(tile_off);
    return K;
}

/* ------------------------------------------------------------------------ */
/* masked compositing, forward and backward, one pixel at a time            */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double* mean2d;   /* [R, 2]  R = n_views * n records */
    const double* conic;    /* [R, 3] */
    const double* opacity;  /* [R]    */
    const double* color;    /* [R, 3] */
    const double* mask;     /* [n]    shared by all views */
    int64_t n;
} orc_splats;

/* One entry that passed both filters and did not stop the pixel. */
typedef struct {
    uint32_t rec;
    double alpha, G, T, dx, dy;
    int clamped;
} orc_blend;

typedef struct {
    double rgb[3];
    double T;
    int64_t last;       /* list position of the last blended entry, -1 if none */
    int64_t examined;   /* entries examined, up to and including the stop entry */
    int64_t n_blend;
    int stopped;
    int64_t stop_pos;   /* list position of the stop entry when stopped */
    uint32_t flags;
} orc_pixel;

/* Walk one pixel's list (list positions [s, e) of `vals`) front to back. */
static void composite_pixel(const orc_splats* sp, const uint32_t* vals, int64_t s, int64_t e, double pxc,
                            double pyc, const orc_settings* st, orc_blend* out_list, orc_pixel* px) {
    const double amin = eff_alpha_min(st), tmin = eff_t_min(st), qmax = eff_q_max(st);
    const double amax = st->alpha_max, mg = st->margin;
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    px->last = -1;
    px->examined = 0;
    px->n_blend = 0;
    px->stopped = 0;
    px->stop_pos = -1;
    px->flags = 0;
    for (int64_t k = s; k < e; k++) {
        px->examined++;
        const uint32_t r = vals[k];
        const int64_t g = (int64_t)(r % (uint32_t)sp->n);
        const double dx = sp->mean2d[2 * r] - pxc, dy = sp->mean2d[2 * r + 1] - pyc;
        const double a = sp->conic[3 * r], b = sp->conic[3 * r + 1], c = sp->conic[3 * r + 2];
        const double Q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
        if (isfinite(qmax) && fabs(Q - qmax) <= mg * qmax) px->flags |= ORC_FLAG_Q;
        if (Q > qmax) continue;
        const double G = exp(-0.5 * Q);
        const double oG = sp->opacity[r] * G;
        if (fabs(oG - amax) <= mg * amax) px->flags |= ORC_FLAG_AMAX;
        const int clamped = oG > amax;
        const double alpha = clamped ? amax : oG;
        if (amin > 0.0 && fabs(alpha - amin) <= mg * amin) px->flags |= ORC_FLAG_AMIN;
        if (alpha < amin) continue;
        const double M = sp->mask[g];
        const double test = T * (1.0 - M * alpha);
        if (tmin > 0.0 && fabs(test - tmin) <= (double)st->margin_t * tmin) px->flags |= ORC_FLAG_TMIN;
        if (test < tmin) {
            px->stopped = 1;
            px->stop_pos = k;
            break;
        }
        for (int ch = 0; ch < 3; ch++) C[ch] += M * alpha * T * sp->color[3 * r + ch];
        if (out_list) {
            orc_blend* bl = &out_list[px->n_blend];
            bl->rec = r; bl->alpha = alpha; bl->G = G; bl->T = T; bl->dx = dx; bl->dy = dy; bl->clamped = clamped;
        }
        px->n_blend++;
        T = test;
        px->last = k;
    }
    for (int ch = 0; ch < 3; ch++) px->rgb[ch] = C[ch] + T * (double)st->bg[ch];
    px->T = T;
}

typedef struct {
    int64_t view_px_off;     /* offset of the view's first pixel */
    int64_t view_tile_off;   /* offset of the view's first tile */
    int gw, gh, w, h;
} orc_view_geom;

static orc_view_geom* make_geoms(int n_views, const int32_t* widths, const int32_t* heights, const orc_settings* st) {
    orc_view_geom* g = (orc_view_geom*)malloc(sizeof(orc_view_geom) * (size_t)n_views);
    int64_t po = 0, to = 0;
    for (int v = 0; v < n_views; v++) {
        g[v].view_px_off = po;
        g[v].view_tile_off = to;
        g[v].w = widths[v];
        g[v].h = heights[v];
        g[v].gw = grid_w(st, widths[v]);
        g[v].gh = grid_h(st, heights[v]);
        po += (int64_t)widths[v] * heights[v];
        to += (int64_t)g[v].gw * g[v].gh;
    }
    return g;
}

/*
 * Forward over every pixel of every view.  images are packed per view as
 * [3, H_v, W_v]; per-pixel arrays are packed per view as [H_v, W_v].
 */
ORC_API void orc_render_fwd(int n_views, const int32_t* widths, const int32_t* heights, const orc_settings* st,
                            int64_t n, const double* mean2d, const double* conic, const double* opacity,
                            const double* color, const double* mask, const uint32_t* vals, const uint32_t* ranges,
                            double* image, double* t_final, int64_t* last, int64_t* examined, int64_t* n_blend,
                            uint8_t* flags) {
    orc_splats sp = {mean2d, conic, opacity, color, mask, n};
    orc_view_geom* geo = make_geoms(n_views, widths, heights, st);
    for (int v = 0; v < n_views; v++) {
        const orc_view_geom gv = geo[v];
        const int64_t P = (int64_t)gv.w * gv.h;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t p = 0; p < P; p++) {
            const int x = (int)(p % gv.w), y = (int)(p / gv.w);
            const int64_t tile = gv.view_tile_off + (int64_t)(y / st->tile_h) * gv.gw + (x / st->tile_w);
            orc_pixel px;
            composite_pixel(&sp, vals, ranges[2 * tile], ranges[2 * tile + 1], x + 0.5, y + 0.5, st, NULL, &px);
            const int64_t q = gv.view_px_off + p;
            for (int ch = 0; ch < 3; ch++) image[3 * gv.view_px_off + ch * P + p] = px.rgb[ch];
            t_final[q] = px.T;
            last[q] = px.last;
            examined[q] = px.examined;
            n_blend[q] = px.n_blend;
            flags[q] = (uint8_t)px.flags;
        }
    }
    free(geo);
}

/*
 * Importance of every Gaussian from the forward (the alpha_i T_i of
 * score-based pruning, Sec. 2; the factor Eq. 6 carries, Sec. 3.4): over
 * every pixel of every view, the weight M_i alpha_i T_i with which the
 * Gaussian enters the pixel's colour in Eq. 3, summed (imp_sum) and
 * maximised (imp_max), over the entries the pixel blends.  Each thread
 * accumulates pixels of its own static share; the shares are added in
 * thread order.
 */
ORC_API void orc_importance(int n_views, const int32_t* widths, const int32_t* heights, const orc_settings* st,
                            int64_t n, const double* mean2d, const double* conic, const double* opacity,
                            const double* color, const double* mask, const uint32_t* vals, const uint32_t* ranges,
                            double* imp_sum, double* imp_max) {
    orc_splats sp = {mean2d, conic, opacity, color, mask, n};
    orc_view_geom* geo = make_geoms(n_views, widths, heights, st);
#ifdef _OPENMP
    const int nt = omp_get_max_threads();
#else
    const int nt = 1;
#endif
    double* part_sum = (double*)calloc((size_t)nt * (size_t)n + 1, sizeof(double));
    double* part_max = (double*)calloc((size_t)nt * (size_t)n + 1, sizeof(double));
    for (int v = 0; v < n_views; v++) {
        const orc_view_geom gv = geo[v];
        const int64_t P = (int64_t)gv.w * gv.h;
#pragma omp parallel num_threads(nt)
        {
#ifdef _OPENMP
            const int tid = omp_get_thread_num();
#else
            const int tid = 0;
#endif
            double* ps = part_sum + (size_t)tid * (size_t)n;
            double* pm = part_max + (size_t)tid * (size_t)n;
            int64_t cap = 1024;
            orc_blend* list = (orc_blend*)malloc(sizeof(orc_blend) * (size_t)cap);
#pragma omp for schedule(static)
            for (int64_t p = 0; p < P; p++) {
                const int x = (int)(p % gv.w), y = (int)(p / gv.w);
                const int64_t tile = gv.view_tile_off + (int64_t)(y / st->tile_h) * gv.gw + (x / st->tile_w);
                const int64_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
                if (e - s > cap) {
                    cap = e - s;
                    list = (orc_blend*)realloc(list, sizeof(orc_blend) * (size_t)cap);
                }
                orc_pixel px;
                composite_pixel(&sp, vals, s, e, x + 0.5, y + 0.5, st, list, &px);
                for (int64_t i = 0; i < px.n_blend; i++) {
                    const int64_t g = (int64_t)(list[i].rec % (uint32_t)n);
                    const double w = mask[g] * list[i].alpha * list[i].T;
                    ps[g] += w;
                    if (w > pm[g]) pm[g] = w;
                }
            }
            free(list);
        }
    }
    for (int64_t g = 0; g < n; g++) {
        double s = 0.0, m = 0.0;
        for (int t = 0; t < nt; t++) {
            s += part_sum[(size_t)t * (size_t)n + (size_t)g];
            if (part_max[(size_t)t * (size_t)n + (size_t)g] > m) m = part_max[(size_t)t * (size_t)n + (size_t)g];
        }
        imp_sum[g] = s;
        imp_max[g] = m;
    }
    free(part_sum);
    free(part_max);
    free(geo);
}

/*
 * Backward over every pixel of every view.  dL_dimage has the image layout.
 * Gradients are accumulated per record (view, Gaussian) for the 2D
 * quantities and per Gaussian for the mask.  touched_flagged[rec] is set for
 * every record examined by a flagged pixel (and, after a flagged stop, for
 * the entries such a pixel would blend next until one with non-zero mask).
 */
ORC_API void orc_render_bwd(int n_views, const int32_t* widths, const int32_t* heights, const orc_settings* st,
                            int64_t n, const double* mean2d, const double* conic, const double* opacity,
                            const double* color, const double* mask, const uint32_t* vals, const uint32_t* ranges,
                            const double* dl_dimage, double* d_mean2d, double* d_conic, double* d_opacity,
                            double* d_color, double* d_mask, uint8_t* touched_flagged) {
    orc_splats sp = {mean2d, conic, opacity, color, mask, n};
    orc_view_geom* geo = make_geoms(n_views, widths, heights, st);
    const double bg[3] = {st->bg[0], st->bg[1], st->bg[2]};
    for (int v = 0; v < n_views; v++) {
        const orc_view_geom gv = geo[v];
        const int64_t P = (int64_t)gv.w * gv.h;
#pragma omp parallel
        {
            int64_t cap = 1024;
            orc_blend* list = (orc_blend*)malloc(sizeof(orc_blend) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
            for (int64_t p = 0; p < P; p++) {
                const int x = (int)(p % gv.w), y = (int)(p / gv.w);
                const int64_t tile = gv.view_tile_off + (int64_t)(y / st->tile_h) * gv.gw + (x / st->tile_w);
                const int64_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
                if (e - s > cap) {
                    cap = e - s;
                    list = (orc_blend*)realloc(list, sizeof(orc_blend) * (size_t)cap);
                }
                orc_pixel px;
                composite_pixel(&sp, vals, s, e, x + 0.5, y + 0.5, st, list, &px);
                double w[3];
                for (int ch = 0; ch < 3; ch++) w[ch] = dl_dimage[3 * gv.view_px_off + ch * P + p];
                const double wbg = w[0] * bg[0] + w[1] * bg[1] + w[2] * bg[2];
                double bcol[3] = {0.0, 0.0, 0.0}; /* colour behind, relative to T_{i+1} */
                for (int64_t i = px.n_blend - 1; i >= 0; i--) {
                    const orc_blend* bl = &list[i];
                    const uint32_t r = bl->rec;
                    const int64_t g = (int64_t)(r % (uint32_t)n);
                    const double M = mask[g], al = bl->alpha, Ti = bl->T;
                    const double* c = &color[3 * r];
                    const double X = Ti * (w[0] * (c[0] - bcol[0]) + w[1] * (c[1] - bcol[1]) + w[2] * (c[2] - bcol[2])) -
                                     px.T / (1.0 - M * al) * wbg;
                    const double dM = al * X;
                    const double dA = M * X;
                    double dcol[3];
                    for (int ch = 0; ch < 3; ch++) dcol[ch] = M * al * Ti * w[ch];
                    double dO = 0.0, dQ = 0.0;
                    if (!bl->clamped) {
                        dO = bl->G * dA;
                        dQ = -0.5 * opacity[r] * bl->G * dA;
                    }
                    const double a = conic[3 * r], b = conic[3 * r + 1], cc = conic[3 * r + 2];
                    const double du = dQ * 2.0 * (a * bl->dx + b * bl->dy);
                    const double dv = dQ * 2.0 * (b * bl->dx + cc * bl->dy);
                    const double da = dQ * bl->dx * bl->dx;
                    const double db = dQ * 2.0 * bl->dx * bl->dy;
                    const double dc = dQ * bl->dy * bl->dy;
#pragma omp atomic
                    d_mask[g] += dM;
#pragma omp atomic
                    d_opacity[r] += dO;
#pragma omp atomic
                    d_mean2d[2 * r] += du;
#pragma omp atomic
                    d_mean2d[2 * r + 1] += dv;
#pragma omp atomic
                    d_conic[3 * r] += da;
#pragma omp atomic
                    d_conic[3 * r + 1] += db;
#pragma omp atomic
                    d_conic[3 * r + 2] += dc;
                    for (int ch = 0; ch < 3; ch++) {
#pragma omp atomic
                        d_color[3 * r + ch] += dcol[ch];
                    }
                    for (int ch = 0; ch < 3; ch++) bcol[ch] = M * al * c[ch] + (1.0 - M * al) * bcol[ch];
                }
                if (px.flags && touched_flagged) {
                    const int64_t end_mark = px.stopped ? px.stop_pos : e - 1;
                    for (int64_t k = s; k <= end_mark; k++) touched_flagged[vals[k]] = 1;
                    if (px.stopped && (px.flags & ORC_FLAG_TMIN)) {
                        /* entries a non-stopping walk would blend next, up to the next visible one */
                        const double amin = eff_alpha_min(st), qmax = eff_q_max(st);
                        for (int64_t k = px.stop_pos + 1; k < e; k++) {
                            const uint32_t r = vals[k];
                            touched_flagged[r] = 1;
                            const double dx = mean2d[2 * r] - (x + 0.5), dy = mean2d[2 * r + 1] - (y + 0.5);
                            const double Q = conic[3 * r] * dx * dx + 2.0 * conic[3 * r + 1] * dx * dy +
                                             conic[3 * r + 2] * dy * dy;
                            if (Q > qmax) continue;
                            double al = opacity[r] * exp(-0.5 * Q);
                            if (al > st->alpha_max) al = st->alpha_max;
                            if (al < amin) continue;
                            if (mask[r % (uint32_t)n] * al > 0.0) break;
                        }
                    }
                }
            }
            free(list);
        }
    }
    free(geo);
}

/*
 * Direct per-pixel definition, independent of tiles: every valid Gaussian of
 * one view that passes the Q cut and the alpha filter at the pixel, in
 * (depth, id) order, composited with Eq. (3)-(4) and the background.
 * Used to check sampled pixels at sizes where full tile lists are costly.
 */
typedef struct { uint32_t depth_bits; uint32_t id; double alpha, G; } orc_direct;

static int direct_cmp(const void* a, const void* b) {
    const orc_direct* x = (const orc_direct*)a;
    const orc_direct* y = (const orc_direct*)b;
    if (x->depth_bits != y->depth_bits) return x->depth_bits < y->depth_bits ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

ORC_API void orc_render_pixels_direct(int64_t n, const double* mean2d, const double* conic, const double* opacity,
                                      const double* color, const uint32_t* depth_bits, const uint8_t* valid,
                                      const double* mask, const orc_settings* st, int64_t n_px, const int32_t* px_xy,
                                      double* rgb, double* t_final, int64_t* n_blend) {
    const double amin = eff_alpha_min(st), tmin = eff_t_min(st), qmax = eff_q_max(st);
#pragma omp parallel
    {
        int64_t cap = 4096;
        orc_direct* lst = (orc_direct*)malloc(sizeof(orc_direct) * (size_t)cap);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n_px; i++) {
            const double pxc = px_xy[2 * i] + 0.5, pyc = px_xy[2 * i + 1] + 0.5;
            int64_t cnt = 0;
            for (int64_t g = 0; g < n; g++) {
                if (!valid[g]) continue;
                const double dx = mean2d[2 * g] - pxc, dy = mean2d[2 * g + 1] - pyc;
                const double Q = conic[3 * g] * dx * dx + 2.0 * conic[3 * g + 1] * dx * dy + conic[3 * g + 2] * dy * dy;
                if (Q > qmax) continue;
                const double G = exp(-0.5 * Q);
                double al = opacity[g] * G;
                if (al > st->alpha_max) al = st->alpha_max;
                if (al < amin) continue;
                if (cnt == cap) {
                    cap *= 2;
                    lst = (orc_direct*)realloc(lst, sizeof(orc_direct) * (size_t)cap);
                }
                lst[cnt].depth_bits = depth_bits[g];
                lst[cnt].id = (uint32_t)g;
                lst[cnt].alpha = al;
                lst[cnt].G = G;
                cnt++;
            }
            if (cnt > 1) qsort(lst, (size_t)cnt, sizeof(orc_direct), direct_cmp);
            double T = 1.0, C[3] = {0, 0, 0};
            int64_t nb = 0;
            for (int64_t k = 0; k < cnt; k++) {
                const uint32_t g = lst[k].id;
                const double M = mask[g], al = lst[k].alpha;
                const double test = T * (1.0 - M * al);
                if (test < tmin) break;
                for (int ch = 0; ch < 3; ch++) C[ch] += M * al * T * color[3 * g + ch];
                T = test;
                nb++;
            }
            for (int ch = 0; ch < 3; ch++) rgb[3 * i + ch] = C[ch] + T * (double)st->bg[ch];
            t_final[i] = T;
            n_blend[i] = nb;
        }
        free(lst);
    }
}

/* ------------------------------------------------------------------------ */
/* projection backward: chain rule from 2D quantities to Gaussian params    */
/* ------------------------------------------------------------------------ */

static void project_bwd_one(const double* mean, const double* log_scale, const double* quat, double opacity_logit,
                            const double* sh, int deg, const orc_camera* cam, const orc_settings* st,
                            const double* dmean2d, const double* dconic, double dopac, const double* dcolor,
                            double* g_mean, double* g_logscale, double* g_quat, double* g_oplogit, double* g_sh) {
    orc_proj_state ps;
    project_one(mean, log_scale, quat, opacity_logit, sh, deg, cam, st, &ps);
    if (!ps.valid) return;
    const int K = (deg + 1) * (deg + 1);
    const double fx = cam->fx, fy = cam->fy;
    const double tx = ps.t[0], ty = ps.t[1], tz = ps.t[2];

    /* opacity */
    *g_oplogit += dopac * ps.o * (1.0 - ps.o);

    /* colour: SH coefficients and viewing direction */
    double dcol[3];
    for (int ch = 0; ch < 3; ch++) dcol[ch] = ps.cclamp[ch] ? 0.0 : dcolor[ch];
    double Y[16], dY[16][3];
    sh_basis(deg, ps.dir, Y, dY);
    double ddir[3] = {0, 0, 0};
    for (int k = 0; k < K; k++)
        for (int ch = 0; ch < 3; ch++) {
            g_sh[3 * k + ch] += dcol[ch] * Y[k];
            for (int j = 0; j < 3; j++) ddir[j] += dcol[ch] * sh[3 * k + ch] * dY[k][j];
        }
    double dd = ddir[0] * ps.dir[0] + ddir[1] * ps.dir[1] + ddir[2] * ps.dir[2];
    double dp[3];
    for (int j = 0; j < 3; j++) dp[j] = (ddir[j] - ps.dir[j] * dd) / ps.dnorm;

    /* conic -> 2D covariance: d(Sigma^-1) = -Sigma^-1 dSigma Sigma^-1 */
    const double Cm[4] = {ps.conic[0], ps.conic[1], ps.conic[1], ps.conic[2]};
    const double Gc[4] = {dconic[0], 0.5 * dconic[1], 0.5 * dconic[1], dconic[2]};
    double tmp[4], H[4];
    mat_mul(Cm, Gc, tmp, 2, 2, 2);
    mat_mul(tmp, Cm, H, 2, 2, 2);
    for (int i = 0; i < 4; i++) H[i] = -H[i];

    /* 2D covariance T Sigma3 T^T -> Sigma3 and T */
    double Tt[6], HT[6], dSigma3[9], dT[6], HTS[6];
    mat_transpose(ps.T, Tt, 2, 3);
    mat_mul(H, ps.T, HT, 2, 2, 3);
    mat_mul(Tt, HT, dSigma3, 3, 2, 3);
    mat_mul(HT, ps.Sigma3, HTS, 2, 3, 3);
    for (int i = 0; i < 6; i++) dT[i] = 2.0 * HTS[i];
    /* T = J W */
    double Wt[9], dJ[6];
    mat_transpose(ps.W, Wt, 3, 3);
    mat_mul(dT, Wt, dJ, 2, 3, 3);

    /* view-space position: projection of the centre and the Jacobian */
    double dt[3] = {0, 0, 0};
    dt[0] += dmean2d[0] * fx / tz;
    dt[2] += -dmean2d[0] * fx * tx / (tz * tz);
    dt[1] += dmean2d[1] * fy / tz;
    dt[2] += -dmean2d[1] * fy * ty / (tz * tz);
    dt[2] += dJ[0] * (-fx / (tz * tz));
    dt[2] += dJ[4] * (-fy / (tz * tz));
    /* J02 = -fx sx / tz with sx = tx / tz unless clamped */
    if (!ps.clamp_x) {
        dt[0] += dJ[2] * (-fx / (tz * tz));
        dt[2] += dJ[2] * (2.0 * fx * tx / (tz * tz * tz));
    } else {
        dt[2] += dJ[2] * (fx * ps.sx / (tz * tz));
    }
    if (!ps.clamp_y) {
        dt[1] += dJ[5] * (-fy / (tz * tz));
        dt[2] += dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
    } else {
        dt[2] += dJ[5] * (fy * ps.sy / (tz * tz));
    }
    double dmean[3];
    mat_mul(Wt, dt, dmean, 3, 3, 1);
    for (int j = 0; j < 3; j++) g_mean[j] += dmean[j] + dp[j];

    /* Sigma3 = R diag(s^2) R^T */
    double dR[9];
    {
        /* dL/dR_ik = sum_j (G_ij + G_ji) s_k^2 R_jk */
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) {
                double acc = 0.0;
                for (int j = 0; j < 3; j++) acc += (dSigma3[3 * i + j] + dSigma3[3 * j + i]) * ps.s[k] * ps.s[k] * ps.Rq[3 * j + k];
                dR[3 * i + k] = acc;
            }
        /* dL/ds_k = sum_ij G_ij R_ik R_jk 2 s_k */
        for (int k = 0; k < 3; k++) {
            double acc = 0.0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) acc += dSigma3[3 * i + j] * ps.Rq[3 * i + k] * ps.Rq[3 * j + k];
            g_logscale[k] += acc * 2.0 * ps.s[k] * ps.s[k];
        }
    }
    double dRq[4][9], dqn[4];
    quat_rotation_partials(ps.qn, dRq);
    for (int c = 0; c < 4; c++) {
        double acc = 0.0;
        for (int i = 0; i < 9; i++) acc += dR[i] * dRq[c][i];
        dqn[c] = acc;
    }
    double qd = 0.0;
    for (int c = 0; c < 4; c++) qd += ps.qn[c] * dqn[c];
    for (int c = 0; c < 4; c++) g_quat[c] += (dqn[c] - ps.qn[c] * qd) / ps.qnorm;
}

/* Sum over views of the chain rule; 2D gradients are per record (view, g). */
ORC_API void orc_project_bwd(int n_views, int64_t n, const double* means, const double* log_scales,
                             const double* quats, const double* opacity_logits, const double* sh, const orc_camera* cams,
                             const orc_settings* st, const double* d_mean2d, const double* d_conic,
                             const double* d_opacity, const double* d_color, double* g_means, double* g_log_scales,
                             double* g_quats, double* g_opacity_logits, double* g_sh) {
    const int deg = st->sh_degree, K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int v = 0; v < n_views; v++) {
            const int64_t r = (int64_t)v * n + i;
            project_bwd_one(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opacity_logits[i], sh + 3 * K * i, deg,
                            &cams[v], st, d_mean2d + 2 * r, d_conic + 3 * r, d_opacity[r], d_color + 3 * r,
                            g_means + 3 * i, g_log_scales + 3 * i, g_quats + 4 * i, g_opacity_logits + i,
                            g_sh + 3 * K * i);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* random numbers: Philox4x32-10                                             */
/* ------------------------------------------------------------------------ */

ORC_API void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n1 = lo1;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        const uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0, 1): top 24 bits plus one half, times 2^-24 */
static double u01_from_bits(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

/*
 * Straight-through Gumbel-Softmax over the two scores of each Gaussian:
 * hard M = [s0 + g0 > s1 + g1], soft y = softmax((s + g) / tau)_0.
 * Philox counter = (id lo, id hi, step lo, step hi), key = (seed lo, seed hi);
 * output words 0 and 1 give the noise of scores 0 and 1.
 */
ORC_API void orc_sample_masks(int64_t n, const double* scores, double tau, uint64_t seed, uint64_t step,
                              double* m_hard, double* y_soft, double* gumbel) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)step, (uint32_t)(step >> 32)};
        const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        const double g0 = -log(-log(u01_from_bits(out[0])));
        const double g1 = -log(-log(u01_from_bits(out[1])));
        const double z0 = scores[2 * i] + g0, z1 = scores[2 * i + 1] + g1;
        m_hard[i] = z0 > z1 ? 1.0 : 0.0;
        y_soft[i] = 1.0 / (1.0 + exp(-(z0 - z1) / tau));
        if (gumbel) { gumbel[2 * i] = g0; gumbel[2 * i + 1] = g1; }
    }
}

/*
 * Deterministic masks of the straight-through alternative in the ablation of
 * Sec. 4.3: the existence probability sigmoid(s0 - s1), and a hard mask that
 * is 1 exactly when it exceeds the threshold.
 */
ORC_API void orc_threshold_masks(int64_t n, const double* scores, double threshold, double* m_hard, double* y_soft) {
    for (int64_t i = 0; i < n; i++) {
        const double p = 1.0 / (1.0 + exp(scores[2 * i + 1] - scores[2 * i]));
        m_hard[i] = p > threshold ? 1.0 : 0.0;
        y_soft[i] = p;
    }
}

/*
 * Gradient to the two scores through the straight-through mask, including
 * the mask-count loss L_m = (mean M)^2 weighted by lambda_m (Eq. 7-8).
 */
ORC_API void orc_mask_grad(int64_t n, const double* d_mask, const double* m_hard, const double* y_soft, double tau,
                           double lambda_m, double* d_scores, double* loss_m) {
    double sum = 0.0;
    for (int64_t i = 0; i < n; i++) sum += m_hard[i];
    const double mean = n > 0 ? sum / (double)n : 0.0;
    if (loss_m) *loss_m = mean * mean;
    const double dlm = n > 0 ? 2.0 * mean / (double)n : 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double y = y_soft[i];
        const double g = (d_mask[i] + lambda_m * dlm) * y * (1.0 - y) / tau;
        d_scores[2 * i] = g;
        d_scores[2 * i + 1] = -g;
    }
}

/* ------------------------------------------------------------------------ */
/* losses and optimiser                                                      */
/* ------------------------------------------------------------------------ */

/* L1 mean over every element, sign(0) = 0 */
ORC_API double orc_l1_loss(int64_t m, const double* image, const float* target, double* d_image) {
    double acc = 0.0;
    for (int64_t i = 0; i < m; i++) {
        const double d = image[i] - (double)target[i];
        acc += fabs(d);
        if (d_image) d_image[i] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (double)m;
    }
    return acc / (double)m;
}

ORC_API double orc_psnr(int64_t m, const double* a, const double* b) {
    double acc = 0.0;
    for (int64_t i = 0; i < m; i++) acc += (a[i] - b[i]) * (a[i] - b[i]);
    return -10.0 * log10(acc / (double)m);
}

ORC_API void orc_adam(int64_t m, double* params, const double* grads, double* m1, double* m2, double lr, double b1,
                      double b2, double eps, int64_t step) {
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < m; i++) {
        m1[i] = b1 * m1[i] + (1.0 - b1) * grads[i];
        m2[i] = b2 * m2[i] + (1.0 - b2) * grads[i] * grads[i];
        const double mh = m1[i] / c1, vh = m2[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

ORC_API int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

ORC_API void orc_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
