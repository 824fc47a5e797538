/*
 * FP64 CPU oracle for the non-rectified variational fisheye stereo method of
 * Roxas & Oishi, "Real-Time Variational Fisheye Stereo without Rectification
 * and Undistortion" (arXiv 1909.07545).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark load this file's shared library; the product
 * library never includes, links, loads or calls it, and it shares no code,
 * header, table or constant generator with the GPU path.
 *
 * Style: plain loops in double precision, one function per step of the
 * method, each naming the passage of the paper it follows.  Every sweep is a
 * Jacobi sweep (reads old arrays, writes new ones), so the OpenMP row
 * parallelism gives bitwise identical results for any thread count.
 *
 * Layout: images are row-major H x W arrays, pixel (i = row, j = column) at
 * index i*W + j, with integer coordinates at pixel centres.  Vector fields
 * are interleaved: w[2*idx + c]; the TGV dual q is (dx v1, dy v1, dx v2,
 * dy v2) at q[4*idx + c]; the tensor is (t11, t12, t22) at T[3*idx + c].
 *
 * Where the paper is silent, garbled or inconsistent, the reading taken is
 * stated next to the code that implements it.
 *
 * What pins each function (the checks it is held to, other than itself) is
 * listed in the header of oracle/__init__.py.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

enum { OR_PINHOLE = 0, OR_EQUIDISTANT = 1, OR_KANNALA_BRANDT = 2, OR_UNIFIED = 3, OR_EUCM = 4 };
enum { OR_TGV = 0, OR_TV = 1 };
enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_MODEL = -4, OR_E_DEGENERATE = -5 };

typedef struct {
    int model;          /* OR_PINHOLE, OR_EQUIDISTANT, OR_KANNALA_BRANDT, OR_UNIFIED, OR_EUCM */
    int width, height;
    double fx, fy, cx, cy;
    double k[4];        /* Kannala-Brandt k1..k4; unified: k[0] = xi; enhanced unified: k[0] = alpha,
                           k[1] = beta (ignored otherwise) */
    double fov_deg;     /* full field of view of the circular mask */
} or_camera;

typedef struct {
    int levels, warps, iters, reg;
    double lambda, alpha0, alpha1, beta, eta, du_max, theta_gamma;
    int data_term;      /* 0: brightness, 1: rank transform of radius 2 (census variant),
                           2: gradient magnitude */
} or_params;

/* ------------------------------------------------------------------------ */
/* Camera models.  The method needs only a defined projection pi and, for   */
/* depth, its inverse (Sec. III-B; Sec. III-D last paragraph, which names    */
/* the unified and enhanced unified models as ones with a closed-form        */
/* inverse).  Every model here is radially symmetric: a ray at angle theta   */
/* from the axis lands at normalised radius r_d(theta).                      */
/*  Kannala-Brandt: r_d = theta + k1 theta^3 + k2 theta^5 + k3 theta^7 +     */
/*    k4 theta^9 (equidistant is k = 0, pinhole is r_d = tan theta).         */
/*  Unified (xi): the point is projected from the centre of a unit sphere    */
/*    moved by xi along the axis, m = (x, y) / (xi |X| + z), so               */
/*    r_d = sin theta / (xi + cos theta)  (xi = 0 is the pinhole).           */
/*  Enhanced unified (alpha, beta): m = (x, y) / (alpha rho + (1 - alpha) z), */
/*    rho = sqrt(beta (x^2 + y^2) + z^2), so                                  */
/*    r_d = sin theta / (alpha sqrt(beta sin^2 + cos^2) + (1 - alpha) cos)    */
/*    (alpha = 0 is the pinhole; beta = 1 is the unified model with           */
/*    xi = alpha / (1 - alpha) and focal length scaled by 1 / (1 - alpha)).   */
/* ------------------------------------------------------------------------ */

/* Denominator of the unified models' radial map (> 0 where it is defined). */
static double or_unified_den(const or_camera *c, double th)
{
    double s = sin(th), co = cos(th);
    if (c->model == OR_UNIFIED) return c->k[0] + co;
    return c->k[0] * sqrt(c->k[1] * s * s + co * co) + (1.0 - c->k[0]) * co;
}

static double or_theta_d(const or_camera *c, double th)
{
    if (c->model == OR_PINHOLE) return tan(th);
    if (c->model == OR_EQUIDISTANT) return th;
    if (c->model == OR_UNIFIED || c->model == OR_EUCM) return sin(th) / or_unified_den(c, th);
    double t3 = th * th * th, t5 = t3 * th * th, t7 = t5 * th * th, t9 = t7 * th * th;
    return th + c->k[0] * t3 + c->k[1] * t5 + c->k[2] * t7 + c->k[3] * t9;
}

static double or_dtheta_d(const or_camera *c, double th)
{
    if (c->model == OR_PINHOLE) { double cs = cos(th); return 1.0 / (cs * cs); }
    if (c->model == OR_EQUIDISTANT) return 1.0;
    if (c->model == OR_UNIFIED || c->model == OR_EUCM) {
        /* quotient rule on sin / D */
        double s = sin(th), co = cos(th), D = or_unified_den(c, th), dD;
        if (c->model == OR_UNIFIED) {
            dD = -s;
        } else {
            double a = c->k[0], b = c->k[1], g = sqrt(b * s * s + co * co);
            dD = a * (b - 1.0) * s * co / g - (1.0 - a) * s;
        }
        return (co * D - s * dD) / (D * D);
    }
    double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
    return 1.0 + 3.0 * c->k[0] * t2 + 5.0 * c->k[1] * t4 + 7.0 * c->k[2] * t6 + 9.0 * c->k[3] * t8;
}

/* Largest angle of the grid i*pi/4096 up to which r_d(theta) is increasing;
 * the inverse of the radial map is taken on [0, that angle] and saturates
 * beyond it.  Pinhole: just below pi/2. */
double or_theta_limit(const or_camera *c)
{
    if (c->model == OR_PINHOLE) return 0.5 * OR_PI * (1.0 - 1e-9);
    if (c->model == OR_EQUIDISTANT) return OR_PI;
    int unified = c->model == OR_UNIFIED || c->model == OR_EUCM;
    for (int i = 1; i <= 4096; ++i) {
        double th = OR_PI * (double)i / 4096.0;
        if (unified && !(or_unified_den(c, th) > 0.0)) return OR_PI * (double)(i - 1) / 4096.0;
        if (!(or_dtheta_d(c, th) > 0.0)) return OR_PI * (double)(i - 1) / 4096.0;
    }
    return OR_PI;
}

/* Inverse of the radial map by safeguarded Newton iteration (Sec. III-D:
 * Kannala-Brandt needs a non-linear solve for its unprojection). */
static double or_theta_of_rd(const or_camera *c, double th_lim, double rd)
{
    if (rd <= 0.0) return 0.0;
    if (c->model == OR_EQUIDISTANT) return rd < th_lim ? rd : th_lim;
    if (c->model == OR_PINHOLE) return atan(rd);
    if (rd >= or_theta_d(c, th_lim)) return th_lim;
    double lo = 0.0, hi = th_lim, th = rd < th_lim ? rd : 0.5 * th_lim;
    for (int it = 0; it < 200; ++it) {
        double f = or_theta_d(c, th) - rd;
        if (f == 0.0) return th;
        if (f > 0.0) hi = th; else lo = th;
        double nt = th - f / or_dtheta_d(c, th);
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        if (fabs(nt - th) < 1e-15) return nt;
        th = nt;
    }
    return th;
}

/* pi: 3-D point in the camera frame -> pixel.  Returns 0 if it has no image
 * (pinhole behind the camera). */
static int or_project(const or_camera *c, const double X[3], double x[2])
{
    if (c->model == OR_PINHOLE) {
        if (!(X[2] > 0.0)) return 0;
        x[0] = c->cx + c->fx * X[0] / X[2];
        x[1] = c->cy + c->fy * X[1] / X[2];
        return 1;
    }
    double rho = sqrt(X[0] * X[0] + X[1] * X[1]);
    double th = atan2(rho, X[2]);
    double rd = or_theta_d(c, th);
    if (rho > 0.0) {
        x[0] = c->cx + c->fx * rd * X[0] / rho;
        x[1] = c->cy + c->fy * rd * X[1] / rho;
    } else {
        x[0] = c->cx;
        x[1] = c->cy;
    }
    return 1;
}

/* pi^-1: pixel -> unit ray in the camera frame.  The unified models use
 * their closed forms: unified, the ray (lambda m, lambda - xi) with lambda =
 * (xi + sqrt(1 + (1 - xi^2) r^2)) / (1 + r^2), which has unit length;
 * enhanced unified, normalise(m, m_z) with m_z = (1 - beta alpha^2 r^2) /
 * (alpha sqrt(1 - (2 alpha - 1) beta r^2) + 1 - alpha).  Beyond the angle
 * limit the radius is clamped to r_d(th_lim), as for the other models. */
static void or_unproject(const or_camera *c, double th_lim, double px, double py, double r[3])
{
    double mx = (px - c->cx) / c->fx, my = (py - c->cy) / c->fy;
    if (c->model == OR_PINHOLE) {
        double n = sqrt(mx * mx + my * my + 1.0);
        r[0] = mx / n; r[1] = my / n; r[2] = 1.0 / n;
        return;
    }
    if (c->model == OR_UNIFIED || c->model == OR_EUCM) {
        double rr = sqrt(mx * mx + my * my);
        if (th_lim < OR_PI) {
            double rmax = or_theta_d(c, th_lim);
            if (rr > rmax) {
                mx *= rmax / rr;
                my *= rmax / rr;
                rr = rmax;
            }
        }
        double r2 = rr * rr, X[3];
        if (c->model == OR_UNIFIED) {
            double xi = c->k[0];
            double disc = 1.0 + (1.0 - xi * xi) * r2;
            double lam = (xi + sqrt(disc > 0.0 ? disc : 0.0)) / (1.0 + r2);
            X[0] = lam * mx; X[1] = lam * my; X[2] = lam - xi;
        } else {
            double a = c->k[0], b = c->k[1];
            double disc = 1.0 - (2.0 * a - 1.0) * b * r2;
            X[0] = mx; X[1] = my;
            X[2] = (1.0 - b * a * a * r2) / (a * sqrt(disc > 0.0 ? disc : 0.0) + 1.0 - a);
        }
        double n = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
        r[0] = X[0] / n; r[1] = X[1] / n; r[2] = X[2] / n;
        return;
    }
    double rd = sqrt(mx * mx + my * my);
    double th = or_theta_of_rd(c, th_lim, rd);
    if (rd > 0.0) {
        double s = sin(th) / rd;
        r[0] = s * mx; r[1] = s * my; r[2] = cos(th);
    } else {
        r[0] = 0.0; r[1] = 0.0; r[2] = 1.0;
    }
}

/* Level-l intrinsics of the coarse-to-fine pyramid with scale 1/2
 * (Sec. IV-B): f_l = f / 2^l, c_l = (c + 1/2) / 2^l - 1/2 (pixel centres). */
static or_camera or_level_camera(const or_camera *c, int l)
{
    or_camera o = *c;
    double s = ldexp(1.0, -l);
    o.fx = c->fx * s; o.fy = c->fy * s;
    o.cx = (c->cx + 0.5) * s - 0.5; o.cy = (c->cy + 0.5) * s - 0.5;
    o.width = c->width >> l; o.height = c->height >> l;
    return o;
}

/* Model validity: the radial map must be increasing on [0, FOV/2]. */
int or_camera_check(const or_camera *c)
{
    if (c->width <= 0 || c->height <= 0 || !(c->fx > 0.0) || !(c->fy > 0.0)) return OR_E_INVALID;
    if (c->model < OR_PINHOLE || c->model > OR_EUCM) return OR_E_INVALID;
    if (c->model == OR_UNIFIED && !(c->k[0] >= 0.0)) return OR_E_INVALID;
    if (c->model == OR_EUCM && !(c->k[0] >= 0.0 && c->k[0] <= 1.0 && c->k[1] > 0.0)) return OR_E_INVALID;
    double half = 0.5 * c->fov_deg * OR_PI / 180.0;
    if (!(half > 0.0)) return OR_E_INVALID;
    if (c->model == OR_PINHOLE && !(half < 0.5 * OR_PI)) return OR_E_MODEL;
    if (half > OR_PI) return OR_E_MODEL;
    if (c->model >= OR_KANNALA_BRANDT && or_theta_limit(c) < half) return OR_E_MODEL;
    return OR_OK;
}

/* Batched helpers for tests. */
void or_project_points(const or_camera *c, int n, const double *X, double *x, unsigned char *ok)
{
    for (int i = 0; i < n; ++i) ok[i] = (unsigned char)or_project(c, X + 3 * i, x + 2 * i);
}

void or_unproject_points(const or_camera *c, int n, const double *x, double *r)
{
    double th_lim = or_theta_limit(c);
    for (int i = 0; i < n; ++i) or_unproject(c, th_lim, x[2 * i], x[2 * i + 1], r + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Masks (Sec. IV-B): circular FOV mask at level 0, nearest-neighbour      */
/* scaled per level: M_l(i,j) = M_0(2^l i + 2^(l-1), 2^l j + 2^(l-1)).      */
/* ------------------------------------------------------------------------ */

void or_mask0(const or_camera *c, unsigned char *m)
{
    int W = c->width, H = c->height;
    double rmax = or_theta_d(c, 0.5 * c->fov_deg * OR_PI / 180.0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double mx = (j - c->cx) / c->fx, my = (i - c->cy) / c->fy;
            m[i * W + j] = (unsigned char)(sqrt(mx * mx + my * my) <= rmax);
        }
}

void or_level_mask(const unsigned char *m0, int W, int H, int l, unsigned char *ml)
{
    int Wl = W >> l, Hl = H >> l, off = l > 0 ? (1 << (l - 1)) : 0;
    for (int i = 0; i < Hl; ++i)
        for (int j = 0; j < Wl; ++j)
            ml[i * Wl + j] = m0[((i << l) + off) * W + (j << l) + off];
}

/* ------------------------------------------------------------------------ */
/* Calibration field and pre-rotation (Sec. IV-A).  A surface is projected  */
/* into both cameras with zero translation; the flow x1 - x0 is the field.  */
/* The unit sphere (range 1) stands in for "a surface of arbitrary depth"   */
/* (it has an image at every angle, also beyond 180 degrees).               */
/* valid_c: the direction lies inside camera 1's field of view.             */
/* ------------------------------------------------------------------------ */

void or_calibration_field(const or_camera *c0, const or_camera *c1, const double R[9],
                          double *cf, unsigned char *valid)
{
    int W = c0->width, H = c0->height;
    double lim0 = or_theta_limit(c0);
    double half1 = 0.5 * c1->fov_deg * OR_PI / 180.0;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double r0[3], X1[3], x0[2], x1[2];
            or_unproject(c0, lim0, j, i, r0);
            for (int a = 0; a < 3; ++a) X1[a] = R[3 * a] * r0[0] + R[3 * a + 1] * r0[1] + R[3 * a + 2] * r0[2];
            int ok0 = or_project(c0, r0, x0);
            int ok1 = or_project(c1, X1, x1);
            size_t idx = (size_t)i * W + j;
            if (ok0 && ok1) {
                cf[2 * idx] = x1[0] - x0[0];
                cf[2 * idx + 1] = x1[1] - x0[1];
            } else {
                cf[2 * idx] = 0.0;
                cf[2 * idx + 1] = 0.0;
            }
            double th1 = atan2(sqrt(X1[0] * X1[0] + X1[1] * X1[1]), X1[2]);
            valid[idx] = (unsigned char)(ok0 && ok1 && th1 <= half1);
        }
}

/* Bilinear interpolation with clamp-to-edge taps. */
static double or_bilinear(const double *I, int W, int H, double x, double y)
{
    double fx0 = floor(x), fy0 = floor(y);
    double ax = x - fx0, ay = y - fy0;
    int x0 = (int)fx0, y0 = (int)fy0, x1 = x0 + 1, y1 = y0 + 1;
    x0 = x0 < 0 ? 0 : (x0 > W - 1 ? W - 1 : x0);
    x1 = x1 < 0 ? 0 : (x1 > W - 1 ? W - 1 : x1);
    y0 = y0 < 0 ? 0 : (y0 > H - 1 ? H - 1 : y0);
    y1 = y1 < 0 ? 0 : (y1 > H - 1 ? H - 1 : y1);
    return (1.0 - ax) * (1.0 - ay) * I[(size_t)y0 * W + x0] + ax * (1.0 - ay) * I[(size_t)y0 * W + x1]
         + (1.0 - ax) * ay * I[(size_t)y1 * W + x0] + ax * ay * I[(size_t)y1 * W + x1];
}

/* Pre-rotation warp, done once per pair: I1'(x) = I1(x + c(x)). */
/* ------------------------------------------------------------------------ */
/* Rank transform (a census variant; the paper allows any image I in its     */
/* data term, Sec. III-A, and mentions census matching among the rectified   */
/* comparisons): the share of the (2r+1)^2 - 1 neighbours of a pixel that    */
/* are strictly darker than it, neighbours outside the image taken at the    */
/* nearest edge pixel.  Any strictly increasing change of the intensities    */
/* leaves it unchanged.                                                      */
/* ------------------------------------------------------------------------ */

void or_rank_transform(const double *I, int W, int H, int r, double *out)
{
    const double n = (double)((2 * r + 1) * (2 * r + 1) - 1);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const double c = I[(size_t)i * W + j];
            int count = 0;
            for (int di = -r; di <= r; ++di)
                for (int dj = -r; dj <= r; ++dj) {
                    if (!di && !dj) continue;
                    int y = i + di, x = j + dj;
                    y = y < 0 ? 0 : (y >= H ? H - 1 : y);
                    x = x < 0 ? 0 : (x >= W ? W - 1 : x);
                    count += I[(size_t)y * W + x] < c;
                }
            out[(size_t)i * W + j] = count / n;
        }
}

/* ------------------------------------------------------------------------ */
/* Rectification to a virtual pinhole view and back (Sec. V-A compares the   */
/* method with the same energy run on images rectified to a pinhole view of */
/* a chosen field of view, and shows its errors on the fisheye image).      */
/* The virtual orientation: x along the baseline t' = R^T t (camera 0's      */
/* frame), y perpendicular to x and to the mean of the two optical axes,    */
/* z = x cross y; Rv0 maps camera-0 vectors, Rv1 = Rv0 R^T camera-1 vectors. */
/* Then X_v1 = X_v0 + (|t|, 0, 0): a pinhole pair translated along x.       */
/* ------------------------------------------------------------------------ */

/* Positions within this distance (pixels) outside the image still count as */
/* inside: they arise from rounding at the border (taps are clamped).        */
#define OR_EDGE 1e-6

static void or_cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void or_unit(double a[3])
{
    double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= n; a[1] /= n; a[2] /= n;
}

int or_rectify_rotations(const double R[9], const double t[3], double Rv0[9], double Rv1[9], double *baseline)
{
    double x[3], axis[3], y[3], z[3];
    for (int k = 0; k < 3; ++k) {
        x[k] = 0.0;
        for (int a = 0; a < 3; ++a) x[k] += R[3 * a + k] * t[a];       /* (R^T t)_k */
        axis[k] = 0.5 * ((k == 2) + R[3 * 2 + k]);                    /* camera 1's axis is R^T e_z */
    }
    *baseline = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    if (!(*baseline > 0.0)) return OR_E_INVALID;
    or_unit(x);
    or_cross(axis, x, y);
    if (!(sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]) > 1e-9)) return OR_E_MODEL;
    or_unit(y);
    or_cross(x, y, z);
    for (int k = 0; k < 3; ++k) {
        Rv0[k] = x[k];
        Rv0[3 + k] = y[k];
        Rv0[6 + k] = z[k];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += Rv0[3 * i + k] * R[3 * j + k];
            Rv1[3 * i + j] = acc;
        }
    return OR_OK;
}

/* Pinhole view of a camera image: pixel p of the view sees the ray         */
/* Rv^T ((p - c)/f, 1); it takes the bilinear sample of the image where the */
/* camera sees that ray, if the camera's circular mask holds it (else 0,   */
/* valid 0).  Images row-major, pitch = width.                              */
void or_rectify(const or_camera *cam, const double Rv[9], const or_camera *pin, const double *src, double *dst,
                unsigned char *valid)
{
    double half = 0.5 * cam->fov_deg * OR_PI / 180.0;
    double rmax = or_theta_d(cam, half);
    int Wp = pin->width, Hp = pin->height;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Hp; ++i)
        for (int j = 0; j < Wp; ++j) {
            double v[3] = {(j - pin->cx) / pin->fx, (i - pin->cy) / pin->fy, 1.0}, X[3], x[2];
            for (int a = 0; a < 3; ++a) X[a] = Rv[a] * v[0] + Rv[3 + a] * v[1] + Rv[6 + a] * v[2];
            size_t o = (size_t)i * Wp + j;
            dst[o] = 0.0;
            valid[o] = 0;
            if (!or_project(cam, X, x)) continue;
            double theta = atan2(sqrt(X[0] * X[0] + X[1] * X[1]), X[2]);
            double mx = (x[0] - cam->cx) / cam->fx, my = (x[1] - cam->cy) / cam->fy;
            if (theta > half || sqrt(mx * mx + my * my) > rmax) continue;
            if (x[0] < -OR_EDGE || x[0] > cam->width - 1.0 + OR_EDGE || x[1] < -OR_EDGE ||
                x[1] > cam->height - 1.0 + OR_EDGE)
                continue;
            dst[o] = or_bilinear(src, cam->width, cam->height, x[0], x[1]);
            valid[o] = 1;
        }
}

/* The way back: camera pixel q inside its mask sees pi^-1(q); rotated by   */
/* Rv it lands in the pinhole view at p; if p is inside the view and the    */
/* four bilinear taps around p are valid, the field's bilinear sample there */
/* (else 0, valid 0).                                                       */
void or_unrectify(const or_camera *cam, const double Rv[9], const or_camera *pin, const double *field,
                  const unsigned char *field_valid, double *dst, unsigned char *valid)
{
    double half = 0.5 * cam->fov_deg * OR_PI / 180.0;
    double rmax = or_theta_d(cam, half), th_lim = or_theta_limit(cam);
    int W = cam->width, H = cam->height, Wp = pin->width, Hp = pin->height;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t o = (size_t)i * W + j;
            dst[o] = 0.0;
            valid[o] = 0;
            double mx = (j - cam->cx) / cam->fx, my = (i - cam->cy) / cam->fy;
            if (sqrt(mx * mx + my * my) > rmax) continue;
            double r[3], V[3];
            or_unproject(cam, th_lim, j, i, r);
            for (int a = 0; a < 3; ++a) V[a] = Rv[3 * a] * r[0] + Rv[3 * a + 1] * r[1] + Rv[3 * a + 2] * r[2];
            if (!(V[2] > 0.0)) continue;
            double px = pin->cx + pin->fx * V[0] / V[2], py = pin->cy + pin->fy * V[1] / V[2];
            if (px < -OR_EDGE || px > Wp - 1.0 + OR_EDGE || py < -OR_EDGE || py > Hp - 1.0 + OR_EDGE) continue;
            int x0 = (int)floor(px), y0 = (int)floor(py), x1 = x0 + 1, y1 = y0 + 1;
            x0 = x0 < 0 ? 0 : (x0 > Wp - 1 ? Wp - 1 : x0);
            y0 = y0 < 0 ? 0 : (y0 > Hp - 1 ? Hp - 1 : y0);
            x1 = x1 < 0 ? 0 : (x1 > Wp - 1 ? Wp - 1 : x1);
            y1 = y1 < 0 ? 0 : (y1 > Hp - 1 ? Hp - 1 : y1);
            if (field_valid && !(field_valid[(size_t)y0 * Wp + x0] && field_valid[(size_t)y0 * Wp + x1] &&
                                 field_valid[(size_t)y1 * Wp + x0] && field_valid[(size_t)y1 * Wp + x1]))
                continue;
            dst[o] = or_bilinear(field, Wp, Hp, px, py);
            valid[o] = 1;
        }
}

/* ------------------------------------------------------------------------ */
/* Gradient magnitude (gradient constancy; the paper allows any image I in   */
/* its data term, Sec. III-A): sqrt(Ix^2 + Iy^2) with central differences    */
/* (I(x+1) - I(x-1)) / 2, pixels outside the image taken at the nearest edge */
/* pixel.  Adding a constant to the intensities leaves it unchanged.         */
/* ------------------------------------------------------------------------ */

void or_gradient_magnitude(const double *I, int W, int H, double *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            int jl = j > 0 ? j - 1 : 0, jr = j < W - 1 ? j + 1 : W - 1;
            int iu = i > 0 ? i - 1 : 0, id = i < H - 1 ? i + 1 : H - 1;
            double gx = 0.5 * (I[(size_t)i * W + jr] - I[(size_t)i * W + jl]);
            double gy = 0.5 * (I[(size_t)id * W + j] - I[(size_t)iu * W + j]);
            out[(size_t)i * W + j] = sqrt(gx * gx + gy * gy);
        }
}

void or_prerotate(const double *I1, int W, int H, const double *cf, double *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            out[idx] = or_bilinear(I1, W, H, j + cf[2 * idx], i + cf[2 * idx + 1]);
        }
}

/* ------------------------------------------------------------------------ */
/* Trajectory field (Sec. III-B, Eqs. (6)-(7)).  Points of a surface are    */
/* projected into camera 0 and into a camera translated by a vanishing      */
/* eps * t'/|t'| (images pre-rotated, so the motion is X -> X + t' with     */
/* t' = R^T t); the normalised flow w/|w| is the tangent gamma'(0).  Within  */
/* 2 degrees of the epipoles (+-t') the tangent is undefined: gamma' = 0    */
/* and the pixel is flagged.                                                */
/* ------------------------------------------------------------------------ */

static const double OR_TRAJ_EPS = 1e-6;
static const double OR_EPI_GUARD_DEG = 2.0;

/* t' / |t'| with t' = R^T t; 0 if t = 0. */
static int or_unit_translation(const double R[9], const double t[3], double tp[3])
{
    for (int a = 0; a < 3; ++a) tp[a] = R[a] * t[0] + R[3 + a] * t[1] + R[6 + a] * t[2];
    double tn = sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
    if (!(tn > 0.0)) return 0;
    for (int a = 0; a < 3; ++a) tp[a] /= tn;
    return 1;
}

/* Tangent gamma'(x) at one point x of the image of camera c; returns the
 * epipole flag. */
static int or_tangent(const or_camera *c, double lim, const double tp[3], double cos_guard,
                      double px, double py, double g[2])
{
    double r0[3], X1[3], x0[2], x1[2];
    or_unproject(c, lim, px, py, r0);
    for (int a = 0; a < 3; ++a) X1[a] = r0[a] + OR_TRAJ_EPS * tp[a];
    double ct = r0[0] * tp[0] + r0[1] * tp[1] + r0[2] * tp[2];
    int e = fabs(ct) > cos_guard;
    int ok = or_project(c, r0, x0) && or_project(c, X1, x1);
    g[0] = 0.0;
    g[1] = 0.0;
    if (ok && !e) {
        double gx = x1[0] - x0[0], gy = x1[1] - x0[1];
        double n = sqrt(gx * gx + gy * gy);
        if (n > 0.0) { g[0] = gx / n; g[1] = gy / n; }
    }
    return e;
}

int or_trajectory_field(const or_camera *c0, const double R[9], const double t[3], int l,
                        double *gamma, unsigned char *epi)
{
    double tp[3];
    if (!or_unit_translation(R, t, tp)) return OR_E_DEGENERATE;
    or_camera cl = or_level_camera(c0, l);
    double lim = or_theta_limit(c0);
    double cos_guard = cos(OR_EPI_GUARD_DEG * OR_PI / 180.0);
    int W = cl.width, H = cl.height;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            epi[idx] = (unsigned char)or_tangent(&cl, lim, tp, cos_guard, j, i, gamma + 2 * idx);
        }
    return OR_OK;
}

/* The same tangent at arbitrary level-0 points (test hook). */
int or_trajectory_at(const or_camera *c0, const double R[9], const double t[3], int n, const double *pts,
                     double *gamma, unsigned char *epi)
{
    double tp[3];
    if (!or_unit_translation(R, t, tp)) return OR_E_DEGENERATE;
    double lim = or_theta_limit(c0);
    double cos_guard = cos(OR_EPI_GUARD_DEG * OR_PI / 180.0);
    for (int i = 0; i < n; ++i)
        epi[i] = (unsigned char)or_tangent(c0, lim, tp, cos_guard, pts[2 * i], pts[2 * i + 1], gamma + 2 * i);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Pyramid (Sec. IV-B): scale 1/2 by a 2x2 box average.                     */
/* ------------------------------------------------------------------------ */

void or_downsample(const double *J, int W, int H, double *out)
{
    int Wc = W / 2, Hc = H / 2;
    for (int i = 0; i < Hc; ++i)
        for (int j = 0; j < Wc; ++j)
            out[(size_t)i * Wc + j] = 0.25 * (J[(size_t)(2 * i) * W + 2 * j] + J[(size_t)(2 * i) * W + 2 * j + 1]
                                            + J[(size_t)(2 * i + 1) * W + 2 * j] + J[(size_t)(2 * i + 1) * W + 2 * j + 1]);
}

/* ------------------------------------------------------------------------ */
/* Tensor, Eq. (12): T^(1/2) = exp(-beta |grad I0|^eta) n n^T + nperp nperp^T */
/* with n = grad I0 / |grad I0| (the printed |I0| is read as |grad I0|;      */
/* the printed matrix is used as is, no square root is taken).  Gradient by */
/* central differences, one-sided where a neighbour leaves the image or the */
/* mask; T = I where the gradient vanishes or the pixel is masked out.      */
/* ------------------------------------------------------------------------ */

static int or_in_mask(const unsigned char *m, int W, int H, int i, int j)
{
    return i >= 0 && i < H && j >= 0 && j < W && m[(size_t)i * W + j];
}

void or_tensor(const double *J0, const unsigned char *m, int W, int H, double beta, double eta, double *T)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            double *t = T + 3 * idx;
            t[0] = 1.0; t[1] = 0.0; t[2] = 1.0;
            if (!m[idx]) continue;
            double c = J0[idx], gx = 0.0, gy = 0.0;
            int l = or_in_mask(m, W, H, i, j - 1), r = or_in_mask(m, W, H, i, j + 1);
            if (l && r) gx = 0.5 * (J0[idx + 1] - J0[idx - 1]);
            else if (r) gx = J0[idx + 1] - c;
            else if (l) gx = c - J0[idx - 1];
            int u = or_in_mask(m, W, H, i - 1, j), d = or_in_mask(m, W, H, i + 1, j);
            if (u && d) gy = 0.5 * (J0[idx + W] - J0[idx - W]);
            else if (d) gy = J0[idx + W] - c;
            else if (u) gy = c - J0[idx - W];
            double g = sqrt(gx * gx + gy * gy);
            if (g < 1e-12) continue;
            double nx = gx / g, ny = gy / g, e = exp(-beta * pow(g, eta));
            t[0] = e * nx * nx + ny * ny;
            t[1] = (e - 1.0) * nx * ny;
            t[2] = e * ny * ny + nx * nx;
        }
}

/* ------------------------------------------------------------------------ */
/* Differential operators with the mask boundary condition (Sec. IV-B):     */
/* forward differences whose component is zero when the neighbour leaves    */
/* the image or the mask (Neumann); div is the negative adjoint (Dirichlet).*/
/* mx(P) = M(P) M(P+x) [P+x inside]; my likewise.                           */
/* ------------------------------------------------------------------------ */

static int or_mx(const unsigned char *m, int W, int H, int i, int j)
{
    return or_in_mask(m, W, H, i, j) && or_in_mask(m, W, H, i, j + 1);
}

static int or_my(const unsigned char *m, int W, int H, int i, int j)
{
    return or_in_mask(m, W, H, i, j) && or_in_mask(m, W, H, i + 1, j);
}

/* grad of a scalar field: g[2*idx] = mx (u(P+x) - u(P)), g[2*idx+1] = my (u(P+y) - u(P)). */
void or_grad(const double *u, const unsigned char *m, int W, int H, double *g)
{
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            g[2 * idx] = or_mx(m, W, H, i, j) ? u[idx + 1] - u[idx] : 0.0;
            g[2 * idx + 1] = or_my(m, W, H, i, j) ? u[idx + W] - u[idx] : 0.0;
        }
}

/* div of a 2-vector field (component a at stride s, offset o): the negative adjoint of or_grad. */
static double or_div_at(const double *p, int s, int o, const unsigned char *m, int W, int H, int i, int j)
{
    size_t idx = (size_t)i * W + j;
    double d = 0.0;
    if (or_mx(m, W, H, i, j)) d += p[s * idx + o];
    if (j > 0 && or_mx(m, W, H, i, j - 1)) d -= p[s * (idx - 1) + o];
    if (or_my(m, W, H, i, j)) d += p[s * idx + o + 1];
    if (i > 0 && or_my(m, W, H, i - 1, j)) d -= p[s * (idx - W) + o + 1];
    return d;
}

void or_div(const double *p, const unsigned char *m, int W, int H, double *d)
{
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) d[(size_t)i * W + j] = or_div_at(p, 2, 0, m, W, H, i, j);
}

/* ------------------------------------------------------------------------ */
/* Step sizes: diagonal preconditioning with alpha = 1 (Sec. III-D, after   */
/* Eq. (11)): sigma = 1 / row sums, tau = 1 / column sums of |K| for        */
/* K = [[alpha1 T grad, -alpha1 I], [0, alpha0 grad]].  sigma_p takes the   */
/* smaller of p's two rows so that the projection stays Euclidean; sigma_q  */
/* = 1/(2 alpha0) for all four rows of q.                                    */
/* ------------------------------------------------------------------------ */

void or_steps(const double *T, const unsigned char *m, int W, int H, double alpha0, double alpha1, int reg,
              double *sig_p, double *tau_u, double *tau_v)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            const double *t = T + 3 * idx;
            double mx = or_mx(m, W, H, i, j), my = or_my(m, W, H, i, j);
            double mxl = j > 0 ? or_mx(m, W, H, i, j - 1) : 0.0;
            double myu = i > 0 ? or_my(m, W, H, i - 1, j) : 0.0;
            double vrow = reg == OR_TV ? 0.0 : alpha1;   /* the -alpha1 v entry of each p row */
            double s1 = alpha1 * (fabs(t[0] * mx + t[1] * my) + fabs(t[0]) * mx + fabs(t[1]) * my) + vrow;
            double s2 = alpha1 * (fabs(t[1] * mx + t[2] * my) + fabs(t[1]) * mx + fabs(t[2]) * my) + vrow;
            double smax = s1 > s2 ? s1 : s2;
            sig_p[idx] = smax > 0.0 ? 1.0 / smax : 1.0 / alpha1;
            double cu = fabs(t[0] * mx + t[1] * my) + fabs(t[1] * mx + t[2] * my);
            if (j > 0) { const double *tl = T + 3 * (idx - 1); cu += (fabs(tl[0]) + fabs(tl[1])) * mxl; }
            if (i > 0) { const double *tu = T + 3 * (idx - W); cu += (fabs(tu[1]) + fabs(tu[2])) * myu; }
            tau_u[idx] = cu > 0.0 ? 1.0 / (alpha1 * cu) : 1.0 / alpha1;
            tau_v[idx] = 1.0 / (alpha1 + alpha0 * (mx + my + mxl + myu));
        }
}

/* ------------------------------------------------------------------------ */
/* Projections onto the unit balls, P(phi) = phi / max(1, |phi|) (Eq. (11)). */
/* ------------------------------------------------------------------------ */

static void or_project_ball(double *phi, int n)
{
    double s = 0.0;
    for (int a = 0; a < n; ++a) s += phi[a] * phi[a];
    double nrm = sqrt(s);
    if (nrm > 1.0)
        for (int a = 0; a < n; ++a) phi[a] /= nrm;
}

void or_project_balls(double *phi, int count, int n)
{
    for (int i = 0; i < count; ++i) or_project_ball(phi + (size_t)n * i, n);
}

/* Resolvent of the linearised data term, Eq. (13), with the third case read
 * as u_hat - rho_bar / I_u (the sign that zeroes rho_bar); rho_bar =
 * rho_c + u_hat I_u is the linearised residual of Eq. (3) with rho_c =
 * I1(x, u_w) - I0(x) - u_w I_u.  I_u = 0 leaves u_hat unchanged. */
double or_threshold(double uhat, double rho_c, double Iu, double tau, double lambda)
{
    double rb = rho_c + uhat * Iu;
    double a = tau * lambda * Iu;
    if (rb < -a * Iu) return uhat + a;
    if (rb > a * Iu) return uhat - a;
    if (Iu == 0.0) return uhat;
    return uhat - rb / Iu;
}

void or_threshold_many(int n, const double *uhat, const double *rho_c, const double *Iu, const double *tau,
                       double lambda, double *out)
{
    for (int i = 0; i < n; ++i) out[i] = or_threshold(uhat[i], rho_c[i], Iu[i], tau[i], lambda);
}

/* ------------------------------------------------------------------------ */
/* Linearised energy of Eq. (10) at fixed (I_u, rho_c):                      */
/* sum_M lambda |rho_c + u I_u| + alpha1 |T grad u - v| + alpha0 |grad v|_F.  */
/* ------------------------------------------------------------------------ */

double or_energy(int W, int H, const or_params *pp, const double *T, const unsigned char *m,
                 const double *Iu, const double *rho, const double *u, const double *v)
{
    double E = 0.0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            if (!m[idx]) continue;
            const double *t = T + 3 * idx;
            double mx = or_mx(m, W, H, i, j), my = or_my(m, W, H, i, j);
            double gx = mx ? u[idx + 1] - u[idx] : 0.0, gy = my ? u[idx + W] - u[idx] : 0.0;
            double v1 = 0.0, v2 = 0.0;
            if (pp->reg == OR_TGV) { v1 = v[2 * idx]; v2 = v[2 * idx + 1]; }
            double a1 = t[0] * gx + t[1] * gy - v1, a2 = t[1] * gx + t[2] * gy - v2;
            E += pp->lambda * fabs(rho[idx] + u[idx] * Iu[idx]) + pp->alpha1 * sqrt(a1 * a1 + a2 * a2);
            if (pp->reg == OR_TGV) {
                double d11 = mx ? v[2 * (idx + 1)] - v1 : 0.0, d12 = my ? v[2 * (idx + W)] - v1 : 0.0;
                double d21 = mx ? v[2 * (idx + 1) + 1] - v2 : 0.0, d22 = my ? v[2 * (idx + W) + 1] - v2 : 0.0;
                E += pp->alpha0 * sqrt(d11 * d11 + d12 * d12 + d21 * d21 + d22 * d22);
            }
        }
    return E;
}

/* ------------------------------------------------------------------------ */
/* Primal-dual iterations, Eq. (11), read as the Chambolle-Pock iteration   */
/* for Eq. (10) with K = [[alpha1 T grad, -alpha1 I], [0, alpha0 grad]]:    */
/*   p <- P(p + sigma_p alpha1 (T grad ubar - vbar))                        */
/*   q <- P(q + sigma_q alpha0 grad vbar)                                    */
/*   u' = resolvent(u + tau_u alpha1 div(T p))                               */
/*   v' = v + tau_v (alpha1 p + alpha0 div q)                                */
/*   ubar = u' + theta (u' - u), vbar = v' + theta (v' - v)                  */
/* (alpha1, alpha0 in the primal lines and the over-relaxation against the  */
/* previous iterate are the readings that make this Chambolle-Pock; "u_n"   */
/* is read as u_k).  theta = 1 unless theta_gamma > 0, which selects the     */
/* accelerated schedule theta = 1/sqrt(1 + 2 gamma s), tau <- theta tau,    */
/* sigma <- sigma / theta on scalar factors s of the preconditioned steps.  */
/* Pixels outside the mask are left unchanged.  TV mode: v = 0, no q.        */
/* energy (optional, K+1 entries): the linearised energy before each         */
/* iteration and after the last.                                             */
/* ------------------------------------------------------------------------ */

void or_pd_iterations(int W, int H, const or_params *pp, const double *T, const unsigned char *m,
                      const double *sig_p, const double *tau_u, const double *tau_v,
                      const double *Iu, const double *rho,
                      double *u, double *ubar, double *v, double *vbar, double *p, double *q,
                      int K, double *energy)
{
    size_t n = (size_t)W * H;
    int tgv = pp->reg == OR_TGV;
    double *unew = malloc(n * sizeof(double)), *vnew = malloc(2 * n * sizeof(double));
    double s = 1.0;   /* scalar step factor of the accelerated schedule */
    for (int k = 0; k < K; ++k) {
        if (energy) energy[k] = or_energy(W, H, pp, T, m, Iu, rho, u, v);
        double theta = 1.0, s_next = 1.0;
        if (pp->theta_gamma > 0.0) {
            theta = 1.0 / sqrt(1.0 + 2.0 * pp->theta_gamma * s);
            s_next = theta * s;
        }
        /* dual ascent */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                size_t idx = (size_t)i * W + j;
                if (!m[idx]) continue;
                const double *t = T + 3 * idx;
                int mx = or_mx(m, W, H, i, j), my = or_my(m, W, H, i, j);
                double gx = mx ? ubar[idx + 1] - ubar[idx] : 0.0;
                double gy = my ? ubar[idx + W] - ubar[idx] : 0.0;
                double sp = sig_p[idx] / s;
                double vb1 = tgv ? vbar[2 * idx] : 0.0, vb2 = tgv ? vbar[2 * idx + 1] : 0.0;
                double ph[2];
                ph[0] = p[2 * idx] + sp * pp->alpha1 * (t[0] * gx + t[1] * gy - vb1);
                ph[1] = p[2 * idx + 1] + sp * pp->alpha1 * (t[1] * gx + t[2] * gy - vb2);
                or_project_ball(ph, 2);
                p[2 * idx] = ph[0];
                p[2 * idx + 1] = ph[1];
                if (tgv) {
                    double sq = 1.0 / (2.0 * pp->alpha0) / s, qh[4];
                    qh[0] = q[4 * idx] + sq * pp->alpha0 * (mx ? vbar[2 * (idx + 1)] - vb1 : 0.0);
                    qh[1] = q[4 * idx + 1] + sq * pp->alpha0 * (my ? vbar[2 * (idx + W)] - vb1 : 0.0);
                    qh[2] = q[4 * idx + 2] + sq * pp->alpha0 * (mx ? vbar[2 * (idx + 1) + 1] - vb2 : 0.0);
                    qh[3] = q[4 * idx + 3] + sq * pp->alpha0 * (my ? vbar[2 * (idx + W) + 1] - vb2 : 0.0);
                    or_project_ball(qh, 4);
                    for (int a = 0; a < 4; ++a) q[4 * idx + a] = qh[a];
                }
            }
        /* primal descent: the resolvent for u, explicit step for v */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                size_t idx = (size_t)i * W + j;
                unew[idx] = u[idx];
                if (tgv) {
                    vnew[2 * idx] = v[2 * idx];
                    vnew[2 * idx + 1] = v[2 * idx + 1];
                }
                if (!m[idx]) continue;
                /* div(T p) built from the products (T p)(P) at P, P-x, P-y */
                double dtp = 0.0;
                if (or_mx(m, W, H, i, j)) {
                    const double *t = T + 3 * idx;
                    dtp += t[0] * p[2 * idx] + t[1] * p[2 * idx + 1];
                }
                if (j > 0 && or_mx(m, W, H, i, j - 1)) {
                    const double *t = T + 3 * (idx - 1);
                    dtp -= t[0] * p[2 * (idx - 1)] + t[1] * p[2 * (idx - 1) + 1];
                }
                if (or_my(m, W, H, i, j)) {
                    const double *t = T + 3 * idx;
                    dtp += t[1] * p[2 * idx] + t[2] * p[2 * idx + 1];
                }
                if (i > 0 && or_my(m, W, H, i - 1, j)) {
                    const double *t = T + 3 * (idx - W);
                    dtp -= t[1] * p[2 * (idx - W)] + t[2] * p[2 * (idx - W) + 1];
                }
                double tu = tau_u[idx] * s;
                double uhat = u[idx] + tu * pp->alpha1 * dtp;
                unew[idx] = or_threshold(uhat, rho[idx], Iu[idx], tu, pp->lambda);
                if (tgv) {
                    double tv = tau_v[idx] * s;
                    double dq1 = or_div_at(q, 4, 0, m, W, H, i, j);
                    double dq2 = or_div_at(q, 4, 2, m, W, H, i, j);
                    vnew[2 * idx] = v[2 * idx] + tv * (pp->alpha1 * p[2 * idx] + pp->alpha0 * dq1);
                    vnew[2 * idx + 1] = v[2 * idx + 1] + tv * (pp->alpha1 * p[2 * idx + 1] + pp->alpha0 * dq2);
                }
            }
        /* over-relaxation */
        for (size_t idx = 0; idx < n; ++idx) {
            ubar[idx] = unew[idx] + theta * (unew[idx] - u[idx]);
            u[idx] = unew[idx];
            if (tgv)
                for (int a = 0; a < 2; ++a) {
                    vbar[2 * idx + a] = vnew[2 * idx + a] + theta * (vnew[2 * idx + a] - v[2 * idx + a]);
                    v[2 * idx + a] = vnew[2 * idx + a];
                }
        }
        s = s_next;
    }
    if (energy) energy[K] = or_energy(W, H, pp, T, m, Iu, rho, u, v);
    free(unew);
    free(vnew);
}

/* ------------------------------------------------------------------------ */
/* Warping (Sec. III-A, Eqs. (3), (5); Sec. III-B; Algorithm 1).             */
/* At the warped point y = x + w the tangent gamma'_w is the bicubic (Keys, */
/* a = -1/2, clamp-to-edge) sample g of the trajectory field divided by     */
/* max(|g|, 1/2): unit length wherever the sample is at least half a unit   */
/* long, shorter only where its taps reach an epipole, around which the    */
/* tangents turn through every direction (Sec. III-B) and a unit            */
/* renormalisation of the short sum would be discontinuous in y;            */
/* I_u = I1(y + gamma'_w) - I1(y) is a forward difference of one pixel       */
/* along it (Eq. (5)); rho_c = I1(y) - I0(x) - u_w I_u.  The data term is   */
/* off (I_u = rho_c = 0) where dvalid is 0 (outside the mask, outside       */
/* camera 1's view after pre-rotation, or near an epipole).                 */
/* ------------------------------------------------------------------------ */

static void or_keys_weights(double t, double w[4])
{
    const double a = -0.5;
    double s0 = 1.0 + t, s1 = t, s2 = 1.0 - t, s3 = 2.0 - t;
    w[0] = a * s0 * s0 * s0 - 5.0 * a * s0 * s0 + 8.0 * a * s0 - 4.0 * a;
    w[1] = (a + 2.0) * s1 * s1 * s1 - (a + 3.0) * s1 * s1 + 1.0;
    w[2] = (a + 2.0) * s2 * s2 * s2 - (a + 3.0) * s2 * s2 + 1.0;
    w[3] = a * s3 * s3 * s3 - 5.0 * a * s3 * s3 + 8.0 * a * s3 - 4.0 * a;
}

static void or_bicubic2(const double *g, int W, int H, double x, double y, double out[2])
{
    double fx0 = floor(x), fy0 = floor(y), wx[4], wy[4];
    or_keys_weights(x - fx0, wx);
    or_keys_weights(y - fy0, wy);
    int x0 = (int)fx0, y0 = (int)fy0;
    out[0] = 0.0; out[1] = 0.0;
    for (int b = 0; b < 4; ++b) {
        int yy = y0 - 1 + b;
        yy = yy < 0 ? 0 : (yy > H - 1 ? H - 1 : yy);
        for (int a = 0; a < 4; ++a) {
            int xx = x0 - 1 + a;
            xx = xx < 0 ? 0 : (xx > W - 1 ? W - 1 : xx);
            size_t idx = (size_t)yy * W + xx;
            out[0] += wy[b] * wx[a] * g[2 * idx];
            out[1] += wy[b] * wx[a] * g[2 * idx + 1];
        }
    }
}

void or_sample_trajectory(const double *gamma, int W, int H, int n, const double *pts, double *out)
{
    for (int i = 0; i < n; ++i) or_bicubic2(gamma, W, H, pts[2 * i], pts[2 * i + 1], out + 2 * i);
}

void or_linearise(int W, int H, const double *J0, const double *J1, const double *gamma,
                  const unsigned char *dvalid, const double *u, const double *w,
                  double *u_w, double *gamma_w, double *Iu, double *rho)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            double yx = j + w[2 * idx], yy = i + w[2 * idx + 1], g[2];
            u_w[idx] = u[idx];
            or_bicubic2(gamma, W, H, yx, yy, g);
            double n = sqrt(g[0] * g[0] + g[1] * g[1]);
            if (n < 0.5) n = 0.5;
            g[0] /= n;
            g[1] /= n;
            gamma_w[2 * idx] = g[0];
            gamma_w[2 * idx + 1] = g[1];
            if (!dvalid[idx]) { Iu[idx] = 0.0; rho[idx] = 0.0; continue; }
            double i1 = or_bilinear(J1, W, H, yx, yy);
            double i1s = or_bilinear(J1, W, H, yx + g[0], yy + g[1]);
            Iu[idx] = i1s - i1;
            rho[idx] = i1 - J0[idx] - u[idx] * Iu[idx];
        }
}

/* Clip and accumulate (Sec. III-C, Eqs. (8)-(9); Algorithm 1): the increment
 * du = u - u_w is clamped elementwise to +-du_max; u = u_w + du and
 * w = w + du gamma'_w. */
void or_clip_accumulate(int W, int H, double du_max, const double *u_w, const double *gamma_w,
                        double *u, double *w)
{
    for (size_t idx = 0; idx < (size_t)W * H; ++idx) {
        double du = u[idx] - u_w[idx];
        if (du > du_max) du = du_max;
        if (du < -du_max) du = -du_max;
        u[idx] = u_w[idx] + du;
        w[2 * idx] += du * gamma_w[2 * idx];
        w[2 * idx + 1] += du * gamma_w[2 * idx + 1];
    }
}

/* Coarse-to-fine transfer (Sec. IV-B): u and w are upscaled by 2 with a
 * bilinear sample at ((j + 1/2)/2 - 1/2, (i + 1/2)/2 - 1/2) whose taps
 * outside the coarse mask get weight 0 (the rest renormalised; 0 if none),
 * and multiplied by 2. */
void or_upsample(int Wc, int Hc, const unsigned char *mc, const double *uc, const double *wc,
                 int Wf, int Hf, double *uf, double *wf)
{
    for (int i = 0; i < Hf; ++i)
        for (int j = 0; j < Wf; ++j) {
            double x = (j + 0.5) * 0.5 - 0.5, y = (i + 0.5) * 0.5 - 0.5;
            double fx0 = floor(x), fy0 = floor(y), ax = x - fx0, ay = y - fy0;
            int xs[2] = { (int)fx0, (int)fx0 + 1 }, ys[2] = { (int)fy0, (int)fy0 + 1 };
            double wxs[2] = { 1.0 - ax, ax }, wys[2] = { 1.0 - ay, ay };
            double sw = 0.0, su = 0.0, s1 = 0.0, s2 = 0.0;
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int xx = xs[a] < 0 ? 0 : (xs[a] > Wc - 1 ? Wc - 1 : xs[a]);
                    int yy = ys[b] < 0 ? 0 : (ys[b] > Hc - 1 ? Hc - 1 : ys[b]);
                    size_t cidx = (size_t)yy * Wc + xx;
                    if (!mc[cidx]) continue;
                    double wt = wxs[a] * wys[b];
                    sw += wt;
                    su += wt * uc[cidx];
                    s1 += wt * wc[2 * cidx];
                    s2 += wt * wc[2 * cidx + 1];
                }
            size_t fidx = (size_t)i * Wf + j;
            if (sw > 0.0) {
                uf[fidx] = 2.0 * su / sw;
                wf[2 * fidx] = 2.0 * s1 / sw;
                wf[2 * fidx + 1] = 2.0 * s2 / sw;
            } else {
                uf[fidx] = 0.0;
                wf[2 * fidx] = 0.0;
                wf[2 * fidx + 1] = 0.0;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Depth (Sec. III-D, last paragraph): the rays a = pi0^-1(x) from the      */
/* origin and b = pi0^-1(x + w) from the pre-rotated camera-1 centre        */
/* C = -t' are triangulated by their closest approach:                      */
/*   d0 = (a.C - (a.b)(b.C)) / (1 - (a.b)^2),                               */
/*   d1 = ((a.b)(a.C) - b.C) / (1 - (a.b)^2).                               */
/* depth = d0 (range along the unit ray), Z = d0 a_z.  Invalid (depth and Z  */
/* = +inf, valid = 0) unless 1 - (a.b)^2 > 1e-12, d0 > 0, d1 > 0 and the    */
/* data term was on at x.                                                    */
/* ------------------------------------------------------------------------ */

int or_triangulate(const or_camera *c0, const double R[9], const double t[3], const double *w,
                   const unsigned char *dvalid, double *depth, double *Z, unsigned char *valid)
{
    int W = c0->width, H = c0->height;
    double C[3];
    for (int a = 0; a < 3; ++a) C[a] = -(R[a] * t[0] + R[3 + a] * t[1] + R[6 + a] * t[2]);
    double lim = or_theta_limit(c0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t idx = (size_t)i * W + j;
            double a[3], b[3];
            or_unproject(c0, lim, j, i, a);
            or_unproject(c0, lim, j + w[2 * idx], i + w[2 * idx + 1], b);
            double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
            double aC = a[0] * C[0] + a[1] * C[1] + a[2] * C[2];
            double bC = b[0] * C[0] + b[1] * C[1] + b[2] * C[2];
            double den = 1.0 - ab * ab;
            depth[idx] = INFINITY;
            Z[idx] = INFINITY;
            valid[idx] = 0;
            if (!(den > 1e-12) || !dvalid[idx]) continue;
            double d0 = (aC - ab * bC) / den, d1 = (ab * aC - bC) / den;
            if (!(d0 > 0.0) || !(d1 > 0.0)) continue;
            depth[idx] = d0;
            Z[idx] = d0 * a[2];
            valid[idx] = 1;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole method: Algorithm 1 inside the coarse-to-fine scheme of Sec. IV-B, */
/* after the pre-rotation of Sec. IV-A.                                      */
/*   for l = L-1 .. 0: tensor, steps, (u, w) from level l+1 (or 0),          */
/*     v = p = q = 0; for each warp: linearise, ubar = u, vbar = v,          */
/*     K primal-dual iterations, clip and accumulate;                        */
/*   then triangulate at level 0.                                            */
/* betas/etas: optional per-call override of the tensor parameters.         */
/* level_u/level_w (optional): u and w at the end of every level, level      */
/* l stored at offset sum_{m<l} H_m W_m (times 2 for w).                     */
/* ------------------------------------------------------------------------ */

int or_solve(const or_camera *c0, const or_camera *c1, const double R[9], const double t[3],
             const or_params *pp, const double *I0, const double *I1,
             double *u_out, double *w_out, double *depth, double *Z, unsigned char *valid,
             double *level_u, double *level_w)
{
    int W = c0->width, H = c0->height, L = pp->levels;
    if (L < 1 || pp->warps < 0 || pp->iters < 0) return OR_E_INVALID;
    if (pp->data_term < 0 || pp->data_term > 2) return OR_E_INVALID;
    if (c1->width != W || c1->height != H) return OR_E_INVALID;
    if ((W % (1 << (L - 1))) || (H % (1 << (L - 1)))) return OR_E_INVALID;
    int st = or_camera_check(c0);
    if (st) return st;
    st = or_camera_check(c1);
    if (st) return st;
    size_t n0 = (size_t)W * H;

    /* per-pair setup: masks, calibration field, pre-rotation, pyramids */
    unsigned char *m0 = malloc(n0), *vc = malloc(n0), *d0 = malloc(n0);
    double *cf = malloc(2 * n0 * sizeof(double));
    or_mask0(c0, m0);
    or_calibration_field(c0, c1, R, cf, vc);
    for (size_t i = 0; i < n0; ++i) d0[i] = m0[i] && vc[i];
    double **J0 = malloc(L * sizeof(double *)), **J1 = malloc(L * sizeof(double *));
    J0[0] = malloc(n0 * sizeof(double));
    J1[0] = malloc(n0 * sizeof(double));
    memcpy(J0[0], I0, n0 * sizeof(double));
    or_prerotate(I1, W, H, cf, J1[0]);
    for (int l = 1; l < L; ++l) {
        size_t nl = (size_t)(W >> l) * (H >> l);
        J0[l] = malloc(nl * sizeof(double));
        J1[l] = malloc(nl * sizeof(double));
        or_downsample(J0[l - 1], W >> (l - 1), H >> (l - 1), J0[l]);
        or_downsample(J1[l - 1], W >> (l - 1), H >> (l - 1), J1[l]);
    }

    /* per-level state, sized for level 0 */
    double *u = calloc(n0, sizeof(double)), *w = calloc(2 * n0, sizeof(double));
    double *uc = calloc(n0, sizeof(double)), *wc = calloc(2 * n0, sizeof(double));
    double *ubar = malloc(n0 * sizeof(double)), *v = malloc(2 * n0 * sizeof(double));
    double *vbar = malloc(2 * n0 * sizeof(double)), *p = malloc(2 * n0 * sizeof(double));
    double *q = malloc(4 * n0 * sizeof(double)), *T = malloc(3 * n0 * sizeof(double));
    double *sp = malloc(n0 * sizeof(double)), *tu = malloc(n0 * sizeof(double)), *tv = malloc(n0 * sizeof(double));
    double *uw = malloc(n0 * sizeof(double)), *gw = malloc(2 * n0 * sizeof(double));
    double *Iu = malloc(n0 * sizeof(double)), *rho = malloc(n0 * sizeof(double));
    double *gam = malloc(2 * n0 * sizeof(double));
    unsigned char *ml = malloc(n0), *dl = malloc(n0), *el = malloc(n0), *mprev = malloc(n0);
    unsigned char *dv0 = malloc(n0);
    double *R0 = pp->data_term != 0 ? malloc(n0 * sizeof(double)) : NULL;
    double *R1 = pp->data_term != 0 ? malloc(n0 * sizeof(double)) : NULL;
    size_t lvl_off = 0;
    for (int l = 0; l < L - 1; ++l) lvl_off += (size_t)(W >> l) * (H >> l);

    int Wp = 0, Hp = 0;
    for (int l = L - 1; l >= 0; --l) {
        int Wl = W >> l, Hl = H >> l;
        size_t nl = (size_t)Wl * Hl;
        st = or_trajectory_field(c0, R, t, l, gam, el);
        if (st) break;
        or_level_mask(m0, W, H, l, ml);
        or_level_mask(d0, W, H, l, dl);
        for (size_t i = 0; i < nl; ++i) dl[i] = ml[i] && dl[i] && !el[i];
        if (l == 0) memcpy(dv0, dl, n0);
        or_tensor(J0[l], ml, Wl, Hl, pp->beta, pp->eta, T);
        if (R0) {
            /* rank / gradient data term: the linearisation of this level
               sees the transforms of the level's images; the tensor keeps
               the intensities */
            if (pp->data_term == 1) {
                or_rank_transform(J0[l], Wl, Hl, 2, R0);
                or_rank_transform(J1[l], Wl, Hl, 2, R1);
            } else {
                or_gradient_magnitude(J0[l], Wl, Hl, R0);
                or_gradient_magnitude(J1[l], Wl, Hl, R1);
            }
        }
        or_steps(T, ml, Wl, Hl, pp->alpha0, pp->alpha1, pp->reg, sp, tu, tv);
        if (l == L - 1) {
            memset(u, 0, nl * sizeof(double));
            memset(w, 0, 2 * nl * sizeof(double));
        } else {
            or_upsample(Wp, Hp, mprev, uc, wc, Wl, Hl, u, w);
        }
        memset(v, 0, 2 * nl * sizeof(double));
        memset(p, 0, 2 * nl * sizeof(double));
        memset(q, 0, 4 * nl * sizeof(double));
        for (int ww = 0; ww < pp->warps; ++ww) {
            or_linearise(Wl, Hl, R0 ? R0 : J0[l], R0 ? R1 : J1[l], gam, dl, u, w, uw, gw, Iu, rho);
            memcpy(ubar, u, nl * sizeof(double));
            memcpy(vbar, v, 2 * nl * sizeof(double));
            or_pd_iterations(Wl, Hl, pp, T, ml, sp, tu, tv, Iu, rho, u, ubar, v, vbar, p, q, pp->iters, NULL);
            or_clip_accumulate(Wl, Hl, pp->du_max, uw, gw, u, w);
        }
        if (level_u) memcpy(level_u + lvl_off, u, nl * sizeof(double));
        if (level_w) memcpy(level_w + 2 * lvl_off, w, 2 * nl * sizeof(double));
        if (l > 0) lvl_off -= (size_t)(W >> (l - 1)) * (H >> (l - 1));
        memcpy(uc, u, nl * sizeof(double));
        memcpy(wc, w, 2 * nl * sizeof(double));
        memcpy(mprev, ml, nl);
        Wp = Wl;
        Hp = Hl;
    }
    if (!st) {
        memcpy(u_out, u, n0 * sizeof(double));
        memcpy(w_out, w, 2 * n0 * sizeof(double));
        or_triangulate(c0, R, t, w, dv0, depth, Z, valid);
    }

    free(R0);
    free(R1);
    for (int l = 0; l < L; ++l) { free(J0[l]); free(J1[l]); }
    free(J0); free(J1); free(m0); free(vc); free(d0); free(cf);
    free(u); free(w); free(uc); free(wc); free(ubar); free(v); free(vbar); free(p); free(q); free(T);
    free(sp); free(tu); free(tv); free(uw); free(gw); free(Iu); free(rho); free(gam);
    free(ml); free(dl); free(el); free(mprev); free(dv0);
    return st;
}
