/*
 * The oracle behind the calls of the product library, taking host pointers:
 * vfso_params_default, vfso_rig_create / vfso_rig_destroy, vfso_rig_field,
 * vfso_solve, vfso_solve_batch and vfso_energy, each a thin entry point over
 * the oracle functions of vfs_oracle.c (whole method: Algorithm 1 in the
 * pyramid of Sec. IV-B after the pre-rotation of Sec. IV-A, triangulation
 * of Sec. III-D; fields of Sec. III-B).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of the oracle: loaded by the tests
 * and the CPU baseline, never by the product library, and written against
 * the oracle's own types (or_camera, or_params) -- no header of the product
 * is included.  Images are row-major H x W doubles with no padding; vector
 * fields interleave their components.  The product's stream, storage,
 * pass-schedule and serving parameters have no meaning here and are not
 * taken.  Every call returns 0 or a negative status (-1 invalid argument,
 * -2 out of host memory, -4 camera model, -5 zero baseline).
 */
#include <stdlib.h>
#include <string.h>

typedef struct {
    int model;
    int width, height;
    double fx, fy, cx, cy;
    double k[4];
    double fov_deg;
} or_camera;

typedef struct {
    int levels, warps, iters, reg;
    double lambda, alpha0, alpha1, beta, eta, du_max, theta_gamma;
    int data_term;
} or_params;

/* oracle functions (vfs_oracle.c) */
int or_camera_check(const or_camera *c);
void or_mask0(const or_camera *c, unsigned char *m);
void or_level_mask(const unsigned char *m0, int W, int H, int l, unsigned char *ml);
void or_calibration_field(const or_camera *c0, const or_camera *c1, const double R[9], double *cf,
                          unsigned char *valid);
int or_trajectory_field(const or_camera *c0, const double R[9], const double t[3], int l, double *gamma,
                        unsigned char *epi);
double or_energy(int W, int H, const or_params *pp, const double *T, const unsigned char *m, const double *Iu,
                 const double *rho, const double *u, const double *v);
int or_solve(const or_camera *c0, const or_camera *c1, const double R[9], const double t[3], const or_params *pp,
             const double *I0, const double *I1, double *u_out, double *w_out, double *depth, double *Z,
             unsigned char *valid, double *level_u, double *level_w);

typedef struct vfso_rig {
    or_camera c0, c1;
    double R[9], t[3];
    int levels;
} vfso_rig;

/* The parameters printed in Sec. IV-C (alpha0 = 17, alpha1 = 1.2, beta = 9,
 * eta = 0.85, 0.2 px clip), lambda = 50, TGV, theta = 1, brightness data
 * term; levels = 5, warps = 10, iters = 100. */
int vfso_params_default(or_params *out)
{
    if (!out) return -1;
    memset(out, 0, sizeof(*out));
    out->levels = 5;
    out->warps = 10;
    out->iters = 100;
    out->reg = 0;
    out->lambda = 50.0;
    out->alpha0 = 17.0;
    out->alpha1 = 1.2;
    out->beta = 9.0;
    out->eta = 0.85;
    out->du_max = 0.2;
    out->theta_gamma = 0.0;
    out->data_term = 0;
    return 0;
}

/* A rig: the calibration (X1 = R X0 + t, R row-major) and the level count. */
int vfso_rig_create(const or_camera *c0, const or_camera *c1, const double R[9], const double t[3], int levels,
                    vfso_rig **out)
{
    if (!out) return -1;
    *out = NULL;
    if (!c0 || !c1 || !R || !t || levels < 1) return -1;
    if (c0->width != c1->width || c0->height != c1->height) return -1;
    if ((c0->width % (1 << (levels - 1))) || (c0->height % (1 << (levels - 1)))) return -1;
    int st = or_camera_check(c0);
    if (st) return st;
    st = or_camera_check(c1);
    if (st) return st;
    if (t[0] == 0.0 && t[1] == 0.0 && t[2] == 0.0) return -5;
    vfso_rig *r = malloc(sizeof(*r));
    if (!r) return -2;
    r->c0 = *c0;
    r->c1 = *c1;
    memcpy(r->R, R, sizeof(r->R));
    memcpy(r->t, t, sizeof(r->t));
    r->levels = levels;
    *out = r;
    return 0;
}

void vfso_rig_destroy(vfso_rig *r) { free(r); }

/* One level of a rig field into dst (H_l x W_l, no padding):
 *   which = 0: trajectory field, 2 doubles per pixel (zero in the epipole guard);
 *   which = 1: calibration field (level 0 only), 2 doubles per pixel;
 *   which = 2: the level's circular mask, 1 double (0 or 1) per pixel. */
int vfso_rig_field(const vfso_rig *r, int level, int which, double *dst)
{
    if (!r || !dst || level < 0 || level >= r->levels || which < 0 || which > 2) return -1;
    if (which == 1 && level != 0) return -1;
    const int W = r->c0.width, H = r->c0.height, Wl = W >> level, Hl = H >> level;
    const size_t n0 = (size_t)W * H, nl = (size_t)Wl * Hl;
    if (which == 0) {
        unsigned char *epi = malloc(nl);
        if (!epi) return -2;
        const int st = or_trajectory_field(&r->c0, r->R, r->t, level, dst, epi);
        free(epi);
        return st;
    }
    if (which == 1) {
        unsigned char *v = malloc(n0);
        if (!v) return -2;
        or_calibration_field(&r->c0, &r->c1, r->R, dst, v);
        free(v);
        return 0;
    }
    unsigned char *m0 = malloc(n0), *ml = malloc(nl);
    if (!m0 || !ml) {
        free(m0);
        free(ml);
        return -2;
    }
    or_mask0(&r->c0, m0);
    or_level_mask(m0, W, H, level, ml);
    for (size_t i = 0; i < nl; ++i) dst[i] = ml[i] ? 1.0 : 0.0;
    free(m0);
    free(ml);
    return 0;
}

/* The whole method on n pairs of a rig; per pair b: u_out[b] (H x W),
 * w_out[b] (2 per pixel), depth_out[b] (+inf where invalid), z_out[b] and
 * valid_out[b] (may be NULL arrays or entries).  betas / etas (may be NULL)
 * override params->beta / eta per pair.  params->levels must be the rig's. */
int vfso_solve_batch(vfso_rig *r, int n, const double *const *I0, const double *const *I1, double *const *u_out,
                     double *const *w_out, double *const *depth_out, double *const *z_out,
                     unsigned char *const *valid_out, const or_params *params, const double *betas,
                     const double *etas)
{
    if (!r || n < 1 || !I0 || !I1 || !u_out || !w_out || !depth_out || !params) return -1;
    if (params->levels != r->levels) return -1;
    const size_t n0 = (size_t)r->c0.width * r->c0.height;
    for (int b = 0; b < n; ++b) {
        if (!I0[b] || !I1[b] || !u_out[b] || !w_out[b] || !depth_out[b]) return -1;
        or_params p = *params;
        if (betas) p.beta = betas[b];
        if (etas) p.eta = etas[b];
        double *z = z_out && z_out[b] ? z_out[b] : malloc(n0 * sizeof(double));
        unsigned char *v = valid_out && valid_out[b] ? valid_out[b] : malloc(n0);
        int st = (!z || !v) ? -2 : or_solve(&r->c0, &r->c1, r->R, r->t, &p, I0[b], I1[b], u_out[b], w_out[b],
                                            depth_out[b], z, v, NULL, NULL);
        if (!(z_out && z_out[b])) free(z);
        if (!(valid_out && valid_out[b])) free(v);
        if (st) return st;
    }
    return 0;
}

int vfso_solve(vfso_rig *r, const double *I0, const double *I1, double *u_out, double *w_out, double *depth_out,
               double *z_out, unsigned char *valid_out, const or_params *params)
{
    return vfso_solve_batch(r, 1, &I0, &I1, &u_out, &w_out, &depth_out, z_out ? &z_out : NULL,
                            valid_out ? &valid_out : NULL, params, NULL, NULL);
}

/* The linearised energy of Eq. (10) of a state at one level (W x H): tensor
 * T (3 per pixel), mask m (bytes), I_u, rho_c, u, v (2 per pixel; NULL in
 * TV mode); *out receives it. */
int vfso_energy(int W, int H, const or_params *params, const double *T, const unsigned char *m, const double *Iu,
                const double *rho, const double *u, const double *v, double *out)
{
    if (W < 1 || H < 1 || !params || !T || !m || !Iu || !rho || !u || !out || (params->reg == 0 && !v)) return -1;
    *out = or_energy(W, H, params, T, m, Iu, rho, u, v);
    return 0;
}
