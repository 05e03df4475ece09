/*
 * recogs_oracle.c -- plain FP64 CPU oracle for the select / recolor / splat-render path.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this file's library. It shares no code, header or table
 * with the HIP library; both read the same seeded input arrays.
 *
 * What it computes (paper: ReCoGS, arXiv 2511.18441):
 *   - covariance Sigma = R S S^T R^T                           (Sec. 3.1, eq. 1)
 *   - view-dependent colour from SH coefficients, degree <= 3  (Sec. 3.1, eq. 2)
 *   - per-pixel front-to-back alpha blending                   (Sec. 3.1, eq. 3)
 *   - the tint c* = t c, generalised to an affine 3x3 recolour (Sec. 3.3, eq. 6)
 *   - gradients of the blended image w.r.t. opacity, SH DC and the recolour
 *     matrix                                                    (Sec. 4.1, eq. 8)
 * plus the per-Gaussian screen-disk / colour-ball selection predicate and the
 * (tile, depth) binning whose sorted order the GPU must reproduce exactly.
 *
 * The paper names the original Gaussian-splatting rasterizer (Sec. 4) but states
 * none of its constants; the readings used here (EWA projection with a 0.3 px^2
 * dilation and a 1.3x frustum clamp on the Jacobian, alpha clamp 0.99, skip below
 * 1/255, stop when transmittance would fall below 1e-4, colour = max(0, f + 1/2),
 * real SH with the Condon-Shortley phase) are that rasterizer's published
 * conventions.
 *
 * Everything is evaluated in double precision from the float inputs (which are
 * exact in double). The depth that orders splats is the float32 rounding of the
 * exact camera-space depth, computed with __float128 so the rounding is exact.
 *
 * Tolerance bands. Where a float decides a discrete outcome (an alpha exactly at
 * the 1/255 threshold, transmittance exactly at 1e-4, a tile-rectangle edge) the
 * oracle reports how close the decision was, so a float32 implementation can be
 * graded exactly outside the band and by a computed bound inside it.
 *
 * Parity pins: every function here is checked by CPU tests against closed forms,
 * invariants, scipy's spherical harmonics and finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9];   /* world -> camera rotation, row-major; rows are camera axes */
    double t[3];   /* camera-space position of the world origin */
    double znear;
} orc_camera;

/* ---- per-Gaussian projection record: column indices ------------------------ */
enum {
    P_Z = 0,       /* exact camera depth (double) */
    P_Z32,         /* float32 rounding of the exact depth, as a double */
    P_U, P_V,      /* projected centre, continuous pixel coordinates */
    P_SA, P_SB, P_SC,      /* 2D covariance [[a, b], [b, c]] incl. dilation */
    P_CA, P_CB, P_CC,      /* conic = inverse 2D covariance [[A, B], [B, C]] */
    P_R, P_G, P_B,         /* colour after clamp */
    P_PR, P_PG, P_PB,      /* colour before clamp (after recolour if selected) */
    P_FR, P_FG, P_FB,      /* f + 1/2 before recolour */
    P_SIGMA,               /* activated opacity */
    P_QEXT,                /* extent level 2 ln(255 sigma) + 1/64, or -1 */
    P_EX, P_EY,            /* half-extents of the box q <= QEXT */
    P_DET,                 /* determinant of the 2D covariance */
    P_NCOL
};
enum {
    I_STATUS = 0,          /* 0 visible; 1 depth-culled; 2 degenerate; 3 alpha<1/255 everywhere; 4 off-image */
    I_PXLO, I_PXHI, I_PYLO, I_PYHI,
    I_TXLO, I_TXHI, I_TYLO, I_TYHI,
    I_COUNT,               /* number of tiles overlapped */
    I_FLAG,                /* 1 when a tile/cull decision lies within the rounding band */
    I_Z32BITS,             /* bit pattern of the float32 depth */
    I_SEL,                 /* 1 when the fused recolour was applied */
    I_RULE,                /* extent rule of the tile rectangle: 0 alpha box, 1 3DGS square */
    I_NCOL
};

#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_MIN 1e-4
#define DILATION 0.3
#define FRUSTUM_CLAMP 1.3
#define Q_SLACK (1.0 / 64.0)

/* Bands inside which a float32 evaluation may decide differently.
 * ALPHA_BAND_MAX bounds the per-evaluation relative alpha band (see alpha_band). */
#define ALPHA_BAND_MAX 8e-3
#define TERM_BAND_MIN 1e-5
#define EDGE_BAND_PX 5e-4
#define OPACITY_BAND 1e-6
#define DET_BAND 1e-6

/* ---------------------------------------------------------------------------
 * Real spherical harmonics up to degree 3 (eq. 2), orthonormal on the sphere,
 * Condon-Shortley phase kept, order m = -l..l within band l. With s = sqrt(pi):
 *   l=0: 1/(2s)
 *   l=1: -sqrt3/(2s) y,  sqrt3/(2s) z,  -sqrt3/(2s) x
 *   l=2: sqrt15/(2s) xy, -sqrt15/(2s) yz, sqrt5/(4s)(2z^2-x^2-y^2),
 *        -sqrt15/(2s) xz, sqrt15/(4s)(x^2-y^2)
 *   l=3: -sqrt(35/2)/(4s) y(3x^2-y^2), sqrt105/(2s) xyz, -sqrt(21/2)/(4s) y(4z^2-x^2-y^2),
 *        sqrt7/(4s) z(2z^2-3x^2-3y^2), -sqrt(21/2)/(4s) x(4z^2-x^2-y^2),
 *        sqrt105/(4s) z(x^2-y^2), -sqrt(35/2)/(4s) x(x^2-3y^2)
 * ------------------------------------------------------------------------- */
void orc_sh_basis(int32_t deg, double x, double y, double z, double *out)
{
    const double s = sqrt(M_PI);
    out[0] = 1.0 / (2.0 * s);
    if (deg < 1) return;
    out[1] = -sqrt(3.0) / (2.0 * s) * y;
    out[2] = sqrt(3.0) / (2.0 * s) * z;
    out[3] = -sqrt(3.0) / (2.0 * s) * x;
    if (deg < 2) return;
    out[4] = sqrt(15.0) / (2.0 * s) * x * y;
    out[5] = -sqrt(15.0) / (2.0 * s) * y * z;
    out[6] = sqrt(5.0) / (4.0 * s) * (2.0 * z * z - x * x - y * y);
    out[7] = -sqrt(15.0) / (2.0 * s) * x * z;
    out[8] = sqrt(15.0) / (4.0 * s) * (x * x - y * y);
    if (deg < 3) return;
    out[9] = -sqrt(35.0 / 2.0) / (4.0 * s) * y * (3.0 * x * x - y * y);
    out[10] = sqrt(105.0) / (2.0 * s) * x * y * z;
    out[11] = -sqrt(21.0 / 2.0) / (4.0 * s) * y * (4.0 * z * z - x * x - y * y);
    out[12] = sqrt(7.0) / (4.0 * s) * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    out[13] = -sqrt(21.0 / 2.0) / (4.0 * s) * x * (4.0 * z * z - x * x - y * y);
    out[14] = sqrt(105.0) / (4.0 * s) * z * (x * x - y * y);
    out[15] = -sqrt(35.0 / 2.0) / (4.0 * s) * x * (x * x - 3.0 * y * y);
}

/* ---------------------------------------------------------------------------
 * eq. (1): Sigma = R S S^T R^T with S = diag(exp(log_scale)), R from the unit
 * quaternion (w, x, y, z) (normalised here). Output planes xx, xy, xz, yy, yz, zz.
 * ------------------------------------------------------------------------- */
void orc_covariance(int64_t n, const double *log_scales, const double *quat, double *cov)
{
    for (int64_t i = 0; i < n; ++i) {
        double w = quat[0 * n + i], x = quat[1 * n + i], y = quat[2 * n + i], z = quat[3 * n + i];
        double nq = sqrt(w * w + x * x + y * y + z * z);
        w /= nq; x /= nq; y /= nq; z /= nq;
        double R[3][3] = {
            {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
        double s[3];
        for (int k = 0; k < 3; ++k) s[k] = exp(log_scales[k * n + i]);
        double M[3][3]; /* M = R S */
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[r][c] = R[r][c] * s[c];
        double S[3][3]; /* Sigma = M M^T */
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += M[r][k] * M[c][k];
                S[r][c] = acc;
            }
        cov[0 * n + i] = S[0][0]; cov[1 * n + i] = S[0][1]; cov[2 * n + i] = S[0][2];
        cov[3 * n + i] = S[1][1]; cov[4 * n + i] = S[1][2]; cov[5 * n + i] = S[2][2];
    }
}

/* Exact camera-space depth row . mu + t_z, rounded once to float32. Every product
 * of two float32 values is exact in binary128 and the 4-term sum is exact there for
 * any inputs whose magnitudes span fewer than 60 binades. */
static float depth_f32_exact(const orc_camera *cam, double mx, double my, double mz)
{
    __float128 acc = (__float128)cam->R[6] * (__float128)mx;
    acc += (__float128)cam->R[7] * (__float128)my;
    acc += (__float128)cam->R[8] * (__float128)mz;
    acc += (__float128)cam->t[2];
    return (float)acc;
}

static void camera_centre(const orc_camera *cam, double *c)
{
    for (int k = 0; k < 3; ++k)
        c[k] = -(cam->R[0 * 3 + k] * cam->t[0] + cam->R[1 * 3 + k] * cam->t[1] + cam->R[2 * 3 + k] * cam->t[2]);
}

/* Tile rectangle of a pixel-index box [lo, hi] (inclusive, possibly empty). */
static void rect_from_edges(double ax, double bx, double ay, double by, int32_t W, int32_t H,
                            int32_t tw, int32_t th, int64_t *r /* pxlo pxhi pylo pyhi txlo txhi tylo tyhi count */)
{
    /* pixels whose centre k + 1/2 lies in [u - e, u + e]: k in [ceil(u-e-1/2), floor(u+e-1/2)] */
    double fx0 = ceil(ax), fx1 = floor(bx), fy0 = ceil(ay), fy1 = floor(by);
    if (fx0 < 0) fx0 = 0;
    if (fy0 < 0) fy0 = 0;
    if (fx1 > W - 1) fx1 = W - 1;
    if (fy1 > H - 1) fy1 = H - 1;
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) {
        for (int k = 0; k < 9; ++k) r[k] = (k == 0 || k == 2 || k == 4 || k == 6) ? 0 : -1;
        r[8] = 0;
        return;
    }
    int64_t x0 = (int64_t)fx0, x1 = (int64_t)fx1, y0 = (int64_t)fy0, y1 = (int64_t)fy1;
    r[0] = x0; r[1] = x1; r[2] = y0; r[3] = y1;
    r[4] = x0 / tw; r[5] = x1 / tw; r[6] = y0 / th; r[7] = y1 / th;
    r[8] = (r[5] - r[4] + 1) * (r[7] - r[6] + 1);
}

/* Tile rectangle of the 3DGS rasteriser's square (extent rule 1): a radius of rad
 * pixels around the centre (xc, yc) in pixel-index coordinates (pixel k's centre at
 * k); tiles floor((xc - rad) / tw) up to, not including, floor((xc + rad + tw - 1) / tw),
 * clipped to the grid (the same in y). Empty when either span is. The pixel range
 * written is the one the listed tiles cover inside the image. */
static void rect_square(double xc, double yc, double rad, int32_t W, int32_t H, int32_t tw, int32_t th,
                        int64_t *r /* as rect_from_edges */)
{
    const double ntx = (double)((W + tw - 1) / tw), nty = (double)((H + th - 1) / th);
    double a = floor((xc - rad) / tw), b = floor((xc + rad + tw - 1) / tw);
    double c = floor((yc - rad) / th), d = floor((yc + rad + th - 1) / th);
    a = a < 0 ? 0 : (a > ntx ? ntx : a);
    b = b < 0 ? 0 : (b > ntx ? ntx : b);
    c = c < 0 ? 0 : (c > nty ? nty : c);
    d = d < 0 ? 0 : (d > nty ? nty : d);
    if (!(b > a) || !(d > c)) {
        for (int k = 0; k < 9; ++k) r[k] = (k == 0 || k == 2 || k == 4 || k == 6) ? 0 : -1;
        r[8] = 0;
        return;
    }
    r[4] = (int64_t)a; r[5] = (int64_t)b - 1; r[6] = (int64_t)c; r[7] = (int64_t)d - 1;
    r[0] = r[4] * tw; r[1] = (r[5] + 1) * tw - 1; r[2] = r[6] * th; r[3] = (r[7] + 1) * th - 1;
    if (r[1] > W - 1) r[1] = W - 1;
    if (r[3] > H - 1) r[3] = H - 1;
    r[8] = (r[5] - r[4] + 1) * (r[7] - r[6] + 1);
}

/* Largest eigenvalue of the 2D covariance [[a, b], [b, c]] with the 3DGS rasteriser's
 * floor of 0.1 px^2 under the discriminant: (a + c)/2 + sqrt(max(0.1, ((a - c)/2)^2 + b^2)). */
static double lambda_max_3dgs(double a, double b, double c)
{
    const double hd = 0.5 * (a - c), disc = hd * hd + b * b;
    return 0.5 * (a + c) + sqrt(disc > 0.1 ? disc : 0.1);
}

/* ---------------------------------------------------------------------------
 * Per-Gaussian projection, colour and tile rectangle.
 *   m = R mu + t; cull when float32 depth <= znear (no far plane).
 *   u = fx m_x / z + cx, v = fy m_y / z + cy.
 *   EWA: J = [[fx/z, 0, -fx xh/z^2], [0, fy/z, -fy yh/z^2]] with xh = z clamp(m_x/z,
 *   +-1.3 (W/2)/fx) (same for y); Sigma2D = J R Sigma R^T J^T + 0.3 I; conic = inverse.
 *   colour: f = sum_k C_k Y_k(d), d = (mu - campos)/|mu - campos|; pre = f + 1/2;
 *   if the Gaussian is selected for the fused recolour: pre = M (f + 1/2) + b;
 *   rgb = max(0, pre).
 *   extent: alpha >= 1/255 <=> q <= 2 ln(255 sigma); the box covers q <= that level
 *   plus 1/64 so its edges never decide a pixel; half-extents sqrt(level Sigma_xx),
 *   sqrt(level Sigma_yy); tiles of tw x th pixels.
 *   rule 1 (the 3DGS rasteriser's extent, for comparison with it): the tiles of the
 *   square of radius ceil(3 sqrt(lambda_max)) pixels (rect_square), and a splat then
 *   reaches only the pixels of those tiles (the image depends on the tile shape).
 *   Gaussians with 255 sigma < 1, which can reach no pixel, get no tiles under
 *   either rule.
 * Arrays: means/cov planes (double, [3][n] / [6][n]); opacity [n]; sh [3K][n]
 * (plane k*3+c). mask may be NULL (no recolour), otherwise M (row-major) and b.
 * ------------------------------------------------------------------------- */
void orc_project(int64_t n, const double *means, const double *cov, const double *opacity,
                 const double *sh, int32_t deg, const orc_camera *cam, int32_t tw, int32_t th,
                 const uint8_t *mask, const double *M, const double *b,
                 double *proj /* [n][P_NCOL] */, int64_t *iproj /* [n][I_NCOL] */, int32_t rule)
{
    double campos[3];
    camera_centre(cam, campos);
    const int ncoef = (deg + 1) * (deg + 1);
    const float znear32 = (float)cam->znear;
    for (int64_t i = 0; i < n; ++i) {
        double *p = proj + i * P_NCOL;
        int64_t *q = iproj + i * I_NCOL;
        for (int k = 0; k < P_NCOL; ++k) p[k] = NAN;
        for (int k = 0; k < I_NCOL; ++k) q[k] = 0;
        q[I_RULE] = rule;
        q[I_PXLO] = q[I_PYLO] = q[I_TXLO] = q[I_TYLO] = 0;
        q[I_PXHI] = q[I_PYHI] = q[I_TXHI] = q[I_TYHI] = -1;
        p[P_QEXT] = -1;

        const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
        double m[3];
        for (int r = 0; r < 3; ++r)
            m[r] = cam->R[r * 3 + 0] * mu[0] + cam->R[r * 3 + 1] * mu[1] + cam->R[r * 3 + 2] * mu[2] + cam->t[r];
        const float z32 = depth_f32_exact(cam, mu[0], mu[1], mu[2]);
        uint32_t zb;
        memcpy(&zb, &z32, 4);
        const double z = m[2];
        p[P_Z] = z;
        p[P_Z32] = (double)z32;
        q[I_Z32BITS] = zb;
        if (!(z32 > znear32)) {
            q[I_STATUS] = 1;
            /* one float32 ulp from the plane: the GPU's depth may round the other way */
            if (fabs((double)z32 - (double)znear32) <= 2.0 * ((double)nextafterf(znear32, INFINITY) - (double)znear32))
                q[I_FLAG] = 1;
            continue;
        }
        if (fabs((double)z32 - (double)znear32) <= 2.0 * ((double)nextafterf(znear32, INFINITY) - (double)znear32))
            q[I_FLAG] = 1;
        p[P_U] = cam->fx * m[0] / z + cam->cx;
        p[P_V] = cam->fy * m[1] / z + cam->cy;

        /* EWA 2D covariance */
        const double limx = FRUSTUM_CLAMP * (0.5 * cam->width) / cam->fx;
        const double limy = FRUSTUM_CLAMP * (0.5 * cam->height) / cam->fy;
        double tx = m[0] / z, ty = m[1] / z;
        tx = tx < -limx ? -limx : (tx > limx ? limx : tx);
        ty = ty < -limy ? -limy : (ty > limy ? limy : ty);
        const double xh = tx * z, yh = ty * z;
        const double J[2][3] = {{cam->fx / z, 0.0, -cam->fx * xh / (z * z)},
                                {0.0, cam->fy / z, -cam->fy * yh / (z * z)}};
        double Tm[2][3]; /* J R */
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                Tm[r][c] = J[r][0] * cam->R[0 * 3 + c] + J[r][1] * cam->R[1 * 3 + c] + J[r][2] * cam->R[2 * 3 + c];
        const double S3[3][3] = {{cov[0 * n + i], cov[1 * n + i], cov[2 * n + i]},
                                 {cov[1 * n + i], cov[3 * n + i], cov[4 * n + i]},
                                 {cov[2 * n + i], cov[4 * n + i], cov[5 * n + i]}};
        double S2[2][2];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                double acc = 0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += Tm[r][k] * S3[k][l] * Tm[c][l];
                S2[r][c] = acc;
            }
        const double sa = S2[0][0] + DILATION, sb = S2[0][1], sc = S2[1][1] + DILATION;
        const double det = sa * sc - sb * sb;
        p[P_SA] = sa; p[P_SB] = sb; p[P_SC] = sc; p[P_DET] = det;
        if (!(det > 0) || !isfinite(det)) {
            q[I_STATUS] = 2;
            continue;
        }
        if (det <= DET_BAND * sa * sc) q[I_FLAG] = 1;
        p[P_CA] = sc / det; p[P_CB] = -sb / det; p[P_CC] = sa / det;

        /* colour (eq. 2), optional fused recolour (eq. 6 generalised) */
        double d[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
        const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int k = 0; k < 3; ++k) d[k] /= dn;
        double Y[16];
        orc_sh_basis(deg, d[0], d[1], d[2], Y);
        double f[3];
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < ncoef; ++k) acc += sh[(int64_t)(k * 3 + c) * n + i] * Y[k];
            f[c] = acc + 0.5;
            p[P_FR + c] = f[c];
        }
        const int sel = mask && mask[i];
        q[I_SEL] = sel;
        for (int c = 0; c < 3; ++c) {
            double pre = f[c];
            if (sel) pre = M[c * 3 + 0] * f[0] + M[c * 3 + 1] * f[1] + M[c * 3 + 2] * f[2] + b[c];
            p[P_PR + c] = pre;
            p[P_R + c] = pre > 0 ? pre : 0.0;
        }

        const double sigma = opacity[i];
        p[P_SIGMA] = sigma;
        if (fabs(255.0 * sigma - 1.0) <= OPACITY_BAND) q[I_FLAG] = 1;
        if (!(255.0 * sigma >= 1.0)) {
            q[I_STATUS] = 3;
            continue;
        }
        const double level = 2.0 * log(255.0 * sigma) + Q_SLACK;
        const double ex = sqrt(level * sa), ey = sqrt(level * sc);
        p[P_QEXT] = level; p[P_EX] = ex; p[P_EY] = ey;
        int64_t r0[9];
        if (rule == 1) {
            const double r3 = 3.0 * sqrt(lambda_max_3dgs(sa, sb, sc));
            const double xc = p[P_U] - 0.5, yc = p[P_V] - 0.5;
            rect_square(xc, yc, ceil(r3), cam->width, cam->height, tw, th, r0);
            for (int k = 0; k < 4; ++k) q[I_PXLO + k] = r0[k];
            for (int k = 0; k < 4; ++k) q[I_TXLO + k] = r0[4 + k];
            q[I_COUNT] = r0[8];
            q[I_STATUS] = r0[8] > 0 ? 0 : 4;
            /* flag when a sub-pixel move of the centre, or 3 sqrt(lambda) near an integer
               (its float32 value may round the radius the other way), changes the tiles */
            const double e = EDGE_BAND_PX, er = EDGE_BAND_PX + 1e-5 * r3;
            const double pert[7][3] = {{xc - e, yc, ceil(r3)}, {xc + e, yc, ceil(r3)}, {xc, yc - e, ceil(r3)},
                                       {xc, yc + e, ceil(r3)}, {xc, yc, ceil(r3 - er)}, {xc, yc, ceil(r3 + er)},
                                       {xc, yc, ceil(r3)}};
            for (int k = 0; k < 6; ++k) {
                int64_t r1[9];
                rect_square(pert[k][0], pert[k][1], pert[k][2], cam->width, cam->height, tw, th, r1);
                int same = r1[8] == r0[8];
                if (same && r0[8] > 0)
                    for (int j = 4; j < 8; ++j) same &= r1[j] == r0[j];
                if (!same) q[I_FLAG] = 1;
            }
            continue;
        }
        const double ax = p[P_U] - ex - 0.5, bx = p[P_U] + ex - 0.5;
        const double ay = p[P_V] - ey - 0.5, by = p[P_V] + ey - 0.5;
        rect_from_edges(ax, bx, ay, by, cam->width, cam->height, tw, th, r0);
        q[I_PXLO] = r0[0]; q[I_PXHI] = r0[1]; q[I_PYLO] = r0[2]; q[I_PYHI] = r0[3];
        q[I_TXLO] = r0[4]; q[I_TXHI] = r0[5]; q[I_TYLO] = r0[6]; q[I_TYHI] = r0[7];
        q[I_COUNT] = r0[8];
        q[I_STATUS] = r0[8] > 0 ? 0 : 4;
        /* flag when a sub-pixel move of any edge changes the tile rectangle */
        const double e = EDGE_BAND_PX;
        const double pert[8][4] = {{ax - e, bx, ay, by}, {ax + e, bx, ay, by}, {ax, bx - e, ay, by},
                                   {ax, bx + e, ay, by}, {ax, bx, ay - e, by}, {ax, bx, ay + e, by},
                                   {ax, bx, ay, by - e}, {ax, bx, ay, by + e}};
        for (int k = 0; k < 8; ++k) {
            int64_t r1[9];
            rect_from_edges(pert[k][0], pert[k][1], pert[k][2], pert[k][3], cam->width, cam->height, tw, th, r1);
            int same = r1[8] == r0[8];
            if (same && r0[8] > 0)
                for (int j = 4; j < 8; ++j) same &= r1[j] == r0[j];
            if (!same) q[I_FLAG] = 1;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Selection predicate (per Gaussian; stand-in for the paper's brush selection,
 * Sec. 3.2): selected iff float32 depth > znear, the unclamped projected centre
 * lies in the closed disk (cx, cy, r), and the DC colour Y00 C0 + 1/2 lies in the
 * closed ball (ref, rho). flag = 1 when either inequality is within its band.
 * dc: [3][n] DC coefficients.
 * ------------------------------------------------------------------------- */
void orc_select(int64_t n, const double *means, const double *dc, const orc_camera *cam,
                double scx, double scy, double radius, const double *ref, double color_radius,
                uint8_t *mask, uint8_t *flag)
{
    const double y00 = 1.0 / (2.0 * sqrt(M_PI));
    const float znear32 = (float)cam->znear;
    for (int64_t i = 0; i < n; ++i) {
        const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
        double m[3];
        for (int r = 0; r < 3; ++r)
            m[r] = cam->R[r * 3 + 0] * mu[0] + cam->R[r * 3 + 1] * mu[1] + cam->R[r * 3 + 2] * mu[2] + cam->t[r];
        const float z32 = depth_f32_exact(cam, mu[0], mu[1], mu[2]);
        mask[i] = 0;
        flag[i] = 0;
        if (fabs((double)z32 - (double)znear32) <= 2.0 * ((double)nextafterf(znear32, INFINITY) - (double)znear32))
            flag[i] = 1;
        if (!(z32 > znear32)) continue;
        const double u = cam->fx * m[0] / m[2] + cam->cx, v = cam->fy * m[1] / m[2] + cam->cy;
        const double d2 = (u - scx) * (u - scx) + (v - scy) * (v - scy);
        double c2 = 0;
        for (int c = 0; c < 3; ++c) {
            const double col = y00 * dc[c * n + i] + 0.5 - ref[c];
            c2 += col * col;
        }
        const double r2 = radius * radius, rho2 = color_radius * color_radius;
        if (fabs(d2 - r2) <= 1e-5 * r2 || fabs(c2 - rho2) <= 1e-6) flag[i] = 1;
        mask[i] = (d2 <= r2) && (c2 <= rho2);
    }
}

/* ---------------------------------------------------------------------------
 * Recolour on coefficients (eq. 6 generalised to rgb' = M rgb + b on the displayed
 * colour rgb = f + 1/2): for selected i, C'_k = M C_k for k >= 1 and
 * C'_0 = M C_0 + ((M - I) 1/2 + b) / Y00. Unselected coefficients are copied.
 * sh, out: [3K][n], plane k*3 + c.
 * ------------------------------------------------------------------------- */
void orc_recolor(int64_t n, int32_t ncoef, const double *sh, const uint8_t *mask,
                 const double *M, const double *b, double *out)
{
    const double y00 = 1.0 / (2.0 * sqrt(M_PI));
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < ncoef; ++k) {
            double c_in[3], c_out[3];
            for (int c = 0; c < 3; ++c) c_in[c] = sh[(int64_t)(k * 3 + c) * n + i];
            if (mask[i]) {
                for (int r = 0; r < 3; ++r) {
                    c_out[r] = M[r * 3 + 0] * c_in[0] + M[r * 3 + 1] * c_in[1] + M[r * 3 + 2] * c_in[2];
                    if (k == 0) {
                        const double off = (M[r * 3 + 0] + M[r * 3 + 1] + M[r * 3 + 2] - 1.0) * 0.5 + b[r];
                        c_out[r] += off / y00;
                    }
                }
            } else {
                for (int c = 0; c < 3; ++c) c_out[c] = c_in[c];
            }
            for (int c = 0; c < 3; ++c) out[(int64_t)(k * 3 + c) * n + i] = c_out[c];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Keys of the tile binning: for every Gaussian with a non-empty rectangle, in index
 * order, one entry per overlapped tile in row-major order: (tile id, float32 depth
 * bits, Gaussian index). tiles_x = ceil(W / tw). Returns the number written.
 * ------------------------------------------------------------------------- */
int64_t orc_emit_keys(int64_t n, const int64_t *iproj, int32_t tiles_x, int64_t cap,
                      int64_t *tile, int64_t *zbits, int64_t *idx)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t *q = iproj + i * I_NCOL;
        if (q[I_COUNT] <= 0) continue;
        for (int64_t ty = q[I_TYLO]; ty <= q[I_TYHI]; ++ty)
            for (int64_t tx = q[I_TXLO]; tx <= q[I_TXHI]; ++tx) {
                if (k < cap) {
                    tile[k] = ty * tiles_x + tx;
                    zbits[k] = q[I_Z32BITS];
                    idx[k] = i;
                }
                ++k;
            }
    }
    return k;
}

/* ---------------------------------------------------------------------------
 * Per-pixel compositing (eq. 3) by its definition.
 *
 * For a pixel p with centre (px + 1/2, py + 1/2), the candidates are the visible
 * Gaussians with alpha_i(p) = min(0.99, sigma_i exp(-q_i(p)/2)) >= 1/255, q the
 * squared Mahalanobis distance under the conic. They are taken in ascending
 * (float32 depth, index) order. With T = 1, C = 0: for each candidate,
 * T' = T (1 - alpha); if T' < 1e-4 stop before blending it; else C += rgb alpha T
 * and T = T'. The pixel value is y = C + T bg.
 *
 * Candidate gathering: for each query window the Gaussians whose extent box
 * (q <= 2 ln(255 sigma) + 1/64, which contains every point with alpha >= 1/255 and
 * the whole rounding band below it) meets the window are listed once; with
 * brute != 0 every visible Gaussian is tried for every pixel instead.
 *
 * Also returned per pixel: final T, the index of the last blended Gaussian (-1 if
 * none), the number blended, and `slack`: an upper bound of how much the pixel can
 * move if a float32 evaluation decides any in-band threshold or termination test
 * the other way (sum over those events of the exact change of y, max over channels).
 * ------------------------------------------------------------------------- */
typedef struct {
    double z32;
    int64_t idx;
    double alpha; /* unclamped sigma * G */
    double band;  /* relative rounding band of alpha at this pixel */
} cand_t;

/* Relative error a float32 evaluation of alpha = sigma exp(-q/2) can carry at this
 * pixel: the projected centre is off by up to du = 2^-22 max(W, H) pixels (a few
 * float32 roundings of a coordinate of that size), which moves q by |grad q| du;
 * q itself and exp carry a few float32 ulps. */
static double alpha_band(const double *p, double dx, double dy, double qv, double du)
{
    const double gx = 2.0 * (p[P_CA] * dx + p[P_CB] * dy), gy = 2.0 * (p[P_CB] * dx + p[P_CC] * dy);
    double b = 1e-5 + 4e-6 * qv + 0.5 * sqrt(gx * gx + gy * gy) * du;
    return b < ALPHA_BAND_MAX ? b : ALPHA_BAND_MAX;
}

static int cand_cmp(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->z32 < y->z32) return -1;
    if (x->z32 > y->z32) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int visible_for_pixels(const int64_t *q, const double *p)
{
    /* any Gaussian not culled by depth or degeneracy, with an extent box, may touch pixels */
    return (q[I_STATUS] == 0 || q[I_STATUS] == 4 || q[I_STATUS] == 3) && p[P_SIGMA] * 255.0 >= 1.0 - ALPHA_BAND_MAX;
}

static double box_level(const double *p)
{
    const double s = p[P_SIGMA] * 255.0;
    return 2.0 * log(s) + Q_SLACK;
}

/* 1 when Gaussian q may reach pixel (px, py): always under the alpha-box rule (its
 * box holds every pixel it reaches); under the 3DGS square rule only in its tiles. */
static int tile_reaches(const int64_t *q, int64_t px, int64_t py)
{
    return !q[I_RULE] || (q[I_PXLO] <= px && px <= q[I_PXHI] && q[I_PYLO] <= py && py <= q[I_PYHI]);
}

/* 1 when Gaussian (p, q) may reach a pixel of the window (x0, y0, w, h): its alpha >= 1/255
 * box meets the window and, under the square rule, so does its tiles' pixel range. */
static int window_reaches(const double *p, const int64_t *q, int32_t x0, int32_t y0, int32_t ww, int32_t wh)
{
    const double lev = box_level(p);
    if (!(lev > 0)) return 0;
    const double ex = sqrt(lev * p[P_SA]), ey = sqrt(lev * p[P_SC]);
    /* pixel centres k + 1/2 within [u - ex, u + ex] */
    if (p[P_U] + ex - 0.5 < x0 || p[P_U] - ex - 0.5 > x0 + ww - 1) return 0;
    if (p[P_V] + ey - 0.5 < y0 || p[P_V] - ey - 0.5 > y0 + wh - 1) return 0;
    if (q[I_RULE] && (q[I_PXHI] < x0 || q[I_PXLO] > x0 + ww - 1 || q[I_PYHI] < y0 || q[I_PYLO] > y0 + wh - 1)) return 0;
    return 1;
}

/* The splats of `list` whose alpha at the pixel centre reaches the threshold (less
 * its rounding band), sorted front to back (z32, then index); returns their count. */
static int64_t gather_candidates(int64_t ncand_all, const int64_t *list, const double *proj, const int64_t *iproj,
                                 double pxc, double pyc, double du, cand_t *buf)
{
    int64_t nc = 0;
    const int64_t px = (int64_t)floor(pxc), py = (int64_t)floor(pyc);
    for (int64_t j = 0; j < ncand_all; ++j) {
        const int64_t i = list[j];
        if (!tile_reaches(iproj + i * I_NCOL, px, py)) continue;
        const double *p = proj + i * P_NCOL;
        const double dx = pxc - p[P_U], dy = pyc - p[P_V];
        const double qv = p[P_CA] * dx * dx + 2.0 * p[P_CB] * dx * dy + p[P_CC] * dy * dy;
        const double a = p[P_SIGMA] * exp(-0.5 * qv);
        if (a >= ALPHA_MIN * (1.0 - ALPHA_BAND_MAX)) {
            buf[nc].z32 = p[P_Z32];
            buf[nc].idx = i;
            buf[nc].alpha = a;
            buf[nc].band = alpha_band(p, dx, dy, qv, du);
            ++nc;
        }
    }
    qsort(buf, (size_t)nc, sizeof(cand_t), cand_cmp);
    return nc;
}

static void composite_pixel(int64_t ncand_all, const int64_t *list, const double *proj, const int64_t *iproj,
                            double pxc, double pyc, double du, const double *bg, cand_t *buf,
                            double *out_rgb, double *out_T, int64_t *out_last, int64_t *out_nb,
                            double *out_slack)
{
    const int64_t nc = gather_candidates(ncand_all, list, proj, iproj, pxc, pyc, du, buf);

    /* forward pass */
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t last = -1, nb = 0, stop = nc;
    for (int64_t k = 0; k < nc; ++k) {
        const double a = buf[k].alpha < ALPHA_MAX ? buf[k].alpha : ALPHA_MAX;
        if (buf[k].alpha < ALPHA_MIN) continue;
        const double Tn = T * (1.0 - a);
        if (Tn < T_MIN) { stop = k; break; }
        const double *p = proj + buf[k].idx * P_NCOL;
        for (int c = 0; c < 3; ++c) C[c] += p[P_R + c] * a * T;
        T = Tn;
        last = buf[k].idx;
        ++nb;
    }
    double y[3];
    for (int c = 0; c < 3; ++c) y[c] = C[c] + T * bg[c];

    /* slack pass: replay, measuring what each in-band decision could change */
    double slack[3] = {0, 0, 0};
    double Tk = 1.0, A[3] = {0, 0, 0};
    double relT = TERM_BAND_MIN; /* relative uncertainty of the float32 transmittance */
    for (int64_t k = 0; k < nc && k <= stop; ++k) {
        const double *p = proj + buf[k].idx * P_NCOL;
        const double araw = buf[k].alpha;
        const double a = araw < ALPHA_MAX ? araw : ALPHA_MAX;
        const int near_thr = fabs(araw * 255.0 - 1.0) <= buf[k].band;
        if (araw < ALPHA_MIN) {
            /* skipped; if blended instead: y changes by a (rgb T - R), R = y - A */
            if (near_thr)
                for (int c = 0; c < 3; ++c) slack[c] += fabs(a * (p[P_R + c] * Tk - (y[c] - A[c])));
            continue;
        }
        const double Tn = Tk * (1.0 - a);
        if (araw < ALPHA_MAX) relT += buf[k].band * a / (1.0 - a);
        if (k == stop) {
            /* stopped here; if continued instead: at most this splat plus Tn times the brightest later colour */
            if (fabs(Tn / T_MIN - 1.0) <= relT) {
                double mx = bg[0] > bg[1] ? bg[0] : bg[1];
                mx = mx > bg[2] ? mx : bg[2];
                for (int64_t j = k + 1; j < nc; ++j) {
                    const double *pj = proj + buf[j].idx * P_NCOL;
                    for (int c = 0; c < 3; ++c) mx = pj[P_R + c] > mx ? pj[P_R + c] : mx;
                }
                for (int c = 0; c < 3; ++c) slack[c] += fabs(a * Tk * p[P_R + c]) + Tn * mx + Tk * bg[c];
            }
            break;
        }
        if (fabs(Tn / T_MIN - 1.0) <= relT) {
            /* blended here; if stopped instead: y = A + Tk bg */
            for (int c = 0; c < 3; ++c) slack[c] += fabs(y[c] - A[c] - Tk * bg[c]);
        }
        if (near_thr) {
            /* blended; if skipped instead: y changes by a (rgb T - R / (1 - a)), R behind it */
            for (int c = 0; c < 3; ++c) {
                const double R = y[c] - A[c] - p[P_R + c] * a * Tk;
                slack[c] += fabs(a * (p[P_R + c] * Tk - R / (1.0 - a)));
            }
        }
        for (int c = 0; c < 3; ++c) A[c] += p[P_R + c] * a * Tk;
        Tk = Tn;
    }
    for (int c = 0; c < 3; ++c) out_rgb[c] = y[c];
    *out_T = T;
    *out_last = last;
    *out_nb = nb;
    double s = slack[0] > slack[1] ? slack[0] : slack[1];
    *out_slack = s > slack[2] ? s : slack[2];
}

void orc_render_windows(int64_t n, const double *proj, const int64_t *iproj, int32_t width, int32_t height,
                        const double *bg,
                        int64_t nwin, const int32_t *win /* [nwin][4]: x0 y0 w h */, int32_t brute,
                        double *out_rgb, double *out_T, int64_t *out_last, int64_t *out_nb, double *out_slack)
{
    int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nwin + 1));
    offs[0] = 0;
    for (int64_t w = 0; w < nwin; ++w) offs[w + 1] = offs[w] + (int64_t)win[w * 4 + 2] * win[w * 4 + 3];

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t w = 0; w < nwin; ++w) {
        const int32_t x0 = win[w * 4 + 0], y0 = win[w * 4 + 1], ww = win[w * 4 + 2], wh = win[w * 4 + 3];
        int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t nl = 0;
        const double du = ldexp((double)(width > height ? width : height), -22);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t *q = iproj + i * I_NCOL;
            const double *p = proj + i * P_NCOL;
            if (!visible_for_pixels(q, p)) continue;
            if (!brute && !window_reaches(p, q, x0, y0, ww, wh)) continue;
            list[nl++] = i;
        }
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(nl > 0 ? nl : 1));
        for (int32_t yy = 0; yy < wh; ++yy)
            for (int32_t xx = 0; xx < ww; ++xx) {
                const int64_t o = offs[w] + (int64_t)yy * ww + xx;
                composite_pixel(nl, list, proj, iproj, x0 + xx + 0.5, y0 + yy + 0.5, du, bg, buf,
                                out_rgb + 3 * o, out_T + o, out_last + o, out_nb + o, out_slack + o);
            }
        free(buf);
        free(list);
    }
    free(offs);
}

/* Rough depth map (Sec. 3.2): following eq. 3's front-to-back order, the depth of the
 * blended splat whose blending takes the transmittance below tau; 0 where it never
 * falls below tau (before the pixel stops). The depth is the splat's float32 depth
 * (z32, the sort key). flag = 1 where a float32 evaluation could decide differently:
 * an alpha near 1/255, or the transmittance within its rounding band of tau, at one of
 * the splats up to and including the crossing. */
static void depth_pixel(int64_t ncand_all, const int64_t *list, const double *proj, const int64_t *iproj, double pxc,
                        double pyc, double du, double tau, cand_t *buf, double *out_depth, int32_t *out_flag)
{
    const int64_t nc = gather_candidates(ncand_all, list, proj, iproj, pxc, pyc, du, buf);
    double T = 1.0, relT = TERM_BAND_MIN;
    double depth = 0.0;
    int32_t flag = 0;
    for (int64_t k = 0; k < nc; ++k) {
        const double araw = buf[k].alpha;
        const double a = araw < ALPHA_MAX ? araw : ALPHA_MAX;
        if (fabs(araw * 255.0 - 1.0) <= buf[k].band) flag = 1;
        if (araw < ALPHA_MIN) continue;
        const double Tn = T * (1.0 - a);
        if (araw < ALPHA_MAX) relT += buf[k].band * a / (1.0 - a);
        if (fabs(Tn / T_MIN - 1.0) <= relT) flag = 1;
        if (Tn < T_MIN) break;  /* not blended: the pixel stops */
        if (fabs(Tn / tau - 1.0) <= relT) flag = 1;
        if (Tn < tau) {
            depth = buf[k].z32;
            break;
        }
        T = Tn;
    }
    *out_depth = depth;
    *out_flag = flag;
}

void orc_depth_windows(int64_t n, const double *proj, const int64_t *iproj, int32_t width, int32_t height, double tau,
                       int64_t nwin, const int32_t *win /* [nwin][4]: x0 y0 w h */, double *out_depth,
                       int32_t *out_flag)
{
    int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nwin + 1));
    offs[0] = 0;
    for (int64_t w = 0; w < nwin; ++w) offs[w + 1] = offs[w] + (int64_t)win[w * 4 + 2] * win[w * 4 + 3];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t w = 0; w < nwin; ++w) {
        const int32_t x0 = win[w * 4 + 0], y0 = win[w * 4 + 1], ww = win[w * 4 + 2], wh = win[w * 4 + 3];
        int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t nl = 0;
        const double du = ldexp((double)(width > height ? width : height), -22);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t *q = iproj + i * I_NCOL;
            const double *p = proj + i * P_NCOL;
            if (!visible_for_pixels(q, p) || !window_reaches(p, q, x0, y0, ww, wh)) continue;
            list[nl++] = i;
        }
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(nl > 0 ? nl : 1));
        for (int32_t yy = 0; yy < wh; ++yy)
            for (int32_t xx = 0; xx < ww; ++xx) {
                const int64_t o = offs[w] + (int64_t)yy * ww + xx;
                depth_pixel(nl, list, proj, iproj, x0 + xx + 0.5, y0 + yy + 0.5, du, tau, buf, out_depth + o,
                            out_flag + o);
            }
        free(buf);
        free(list);
    }
    free(offs);
}

/* ---------------------------------------------------------------------------
 * Backward of the per-pixel compositing and of the colour/recolour step (eq. 8,
 * restricted to opacity, SH DC and the recolour matrix).
 *
 * Given g = dL/dy for every pixel of the image (HWC), for each pixel and each
 * blended Gaussian i (in blending order, T_i its transmittance, R_i the colour
 * of everything behind it including the background):
 *   dL/drgb_i  += alpha_i T_i g
 *   dL/dalpha_i = g . (rgb_i T_i - R_i / (1 - alpha_i))
 *   dL/dsigma_i += dL/dalpha_i G_i(p) when sigma_i G_i(p) < 0.99 (0 where clamped)
 * then per Gaussian, with gh = dL/drgb masked where the pre-clamp colour <= 0:
 *   selected:   dL/dC0 = Y00 M^T gh,  dL/dM += gh (f + 1/2)^T
 *   unselected: dL/dC0 = Y00 gh
 * Skipped and terminated splats receive nothing. Single-threaded.
 * ------------------------------------------------------------------------- */

/* One pixel's terms, over the candidate Gaussians list[0..nl) (a superset of the
 * Gaussians with alpha >= 1/255 at the pixel), accumulated into dsigma and drgb. */
static void backward_pixel(int64_t nl, const int64_t *list, const double *proj, const int64_t *iproj, int64_t px,
                           int64_t py, const double *bg, const double *g, cand_t *buf, double *Tl, double *dsigma,
                           double *drgb)
{
    const double pxc = px + 0.5, pyc = py + 0.5;
    int64_t nc = 0;
    for (int64_t j = 0; j < nl; ++j) {
        const int64_t i = list[j];
        if (!tile_reaches(iproj + i * I_NCOL, px, py)) continue;
        const double *p = proj + i * P_NCOL;
        const double dx = pxc - p[P_U], dy = pyc - p[P_V];
        const double qv = p[P_CA] * dx * dx + 2.0 * p[P_CB] * dx * dy + p[P_CC] * dy * dy;
        const double a = p[P_SIGMA] * exp(-0.5 * qv);
        if (a >= ALPHA_MIN) {
            buf[nc].z32 = p[P_Z32];
            buf[nc].idx = i;
            buf[nc].alpha = a;
            ++nc;
        }
    }
    qsort(buf, (size_t)nc, sizeof(cand_t), cand_cmp);
    /* forward: which are blended, and their T */
    double T = 1.0, y[3] = {0, 0, 0};
    int64_t nbl = 0;
    for (int64_t k = 0; k < nc; ++k) {
        const double a = buf[k].alpha < ALPHA_MAX ? buf[k].alpha : ALPHA_MAX;
        const double Tn = T * (1.0 - a);
        if (Tn < T_MIN) break;
        const double *p = proj + buf[k].idx * P_NCOL;
        for (int c = 0; c < 3; ++c) y[c] += p[P_R + c] * a * T;
        Tl[k] = T;
        T = Tn;
        ++nbl;
    }
    for (int c = 0; c < 3; ++c) y[c] += T * bg[c];
    double Acc[3] = {0, 0, 0};
    for (int64_t k = 0; k < nbl; ++k) {
        const int64_t i = buf[k].idx;
        const double *p = proj + i * P_NCOL;
        const double araw = buf[k].alpha;
        const double a = araw < ALPHA_MAX ? araw : ALPHA_MAX;
        const double Ti = Tl[k];
        double dalpha = 0;
        for (int c = 0; c < 3; ++c) {
            const double contrib = p[P_R + c] * a * Ti;
            const double R = y[c] - Acc[c] - contrib;
            drgb[i * 3 + c] += a * Ti * g[c];
            dalpha += g[c] * (p[P_R + c] * Ti - R / (1.0 - a));
            Acc[c] += contrib;
        }
        if (araw < ALPHA_MAX) dsigma[i] += dalpha * (araw / p[P_SIGMA]);
    }
}

static void backward_zero(int64_t n, double *dsigma, double *drgb, double *dc0, double *dM)
{
    for (int64_t i = 0; i < n; ++i) {
        dsigma[i] = 0;
        for (int c = 0; c < 3; ++c) drgb[i * 3 + c] = 0, dc0[c * n + i] = 0;
    }
    for (int k = 0; k < 9; ++k) dM[k] = 0;
}

/* the per-Gaussian chain through the clamp, the fused recolour and the DC term */
static void backward_chain(int64_t n, const double *proj, const int64_t *iproj, const double *M, const double *drgb,
                           double *dc0, double *dM)
{
    const double y00 = 1.0 / (2.0 * sqrt(M_PI));
    for (int64_t i = 0; i < n; ++i) {
        const double *p = proj + i * P_NCOL;
        const int64_t *q = iproj + i * I_NCOL;
        if (!visible_for_pixels(q, p)) continue;
        double gh[3];
        for (int c = 0; c < 3; ++c) gh[c] = p[P_PR + c] > 0 ? drgb[i * 3 + c] : 0.0;
        if (q[I_SEL]) {
            for (int c = 0; c < 3; ++c)
                dc0[c * n + i] = y00 * (M[0 * 3 + c] * gh[0] + M[1 * 3 + c] * gh[1] + M[2 * 3 + c] * gh[2]);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) dM[r * 3 + c] += gh[r] * p[P_FR + c];
        } else {
            for (int c = 0; c < 3; ++c) dc0[c * n + i] = y00 * gh[c];
        }
    }
}

/* Whole image, every visible Gaussian tried at every pixel. */
void orc_backward(int64_t n, const double *proj, const int64_t *iproj, int32_t W, int32_t H,
                  const double *bg, const double *M, const double *dldy /* [H][W][3] */,
                  double *dsigma /* [n] */, double *drgb /* [n][3] */, double *dc0 /* [3][n] */,
                  double *dM /* [9] */)
{
    backward_zero(n, dsigma, drgb, dc0, dM);
    int64_t nl = 0;
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        if (visible_for_pixels(iproj + i * I_NCOL, proj + i * P_NCOL)) list[nl++] = i;
    cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(nl > 0 ? nl : 1));
    double *Tl = (double *)malloc(sizeof(double) * (size_t)(nl > 0 ? nl : 1));
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px)
            backward_pixel(nl, list, proj, iproj, px, py, bg, dldy + ((int64_t)py * W + px) * 3, buf, Tl, dsigma,
                           drgb);
    backward_chain(n, proj, iproj, M, drgb, dc0, dM);
    free(Tl);
    free(buf);
    free(list);
}

/* The same where dL/dy is zero outside the given windows (x0, y0, w, h): only their
 * pixels are visited, each with the Gaussians whose alpha >= 1/255 box (as in
 * orc_render_windows) meets the window as candidates. Windows in order, pixels
 * row-major inside each. */
void orc_backward_windows(int64_t n, const double *proj, const int64_t *iproj, int32_t W, int32_t H,
                          const double *bg, const double *M, const double *dldy /* [H][W][3] */,
                          int64_t nwin, const int32_t *win /* [nwin][4] */,
                          double *dsigma, double *drgb, double *dc0, double *dM)
{
    (void)H;
    backward_zero(n, dsigma, drgb, dc0, dM);
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t w = 0; w < nwin; ++w) {
        const int32_t x0 = win[w * 4 + 0], y0 = win[w * 4 + 1], ww = win[w * 4 + 2], wh = win[w * 4 + 3];
        int64_t nl = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t *q = iproj + i * I_NCOL;
            const double *p = proj + i * P_NCOL;
            if (!visible_for_pixels(q, p) || !window_reaches(p, q, x0, y0, ww, wh)) continue;
            list[nl++] = i;
        }
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(nl > 0 ? nl : 1));
        double *Tl = (double *)malloc(sizeof(double) * (size_t)(nl > 0 ? nl : 1));
        for (int32_t yy = 0; yy < wh; ++yy)
            for (int32_t xx = 0; xx < ww; ++xx) {
                const int64_t px = x0 + xx, py = y0 + yy;
                backward_pixel(nl, list, proj, iproj, px, py, bg, dldy + (py * W + px) * 3, buf, Tl, dsigma, drgb);
            }
        free(Tl);
        free(buf);
    }
    backward_chain(n, proj, iproj, M, drgb, dc0, dM);
    free(list);
}

/* Library self-description for the Python wrapper. */
int32_t orc_ncols(int32_t which) { return which == 0 ? P_NCOL : I_NCOL; }
