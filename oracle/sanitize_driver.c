/*
 * Exercise of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure: built and run by tests/test_sanitizers.py).  A small
 * Kannala-Brandt rig (64 x 48, 180 degrees, 2 degrees of rotation), a pair
 * of band-limited textures, and every entry point of vfso.c plus the whole
 * method in both regularisers and all three data terms; exits 0 when every
 * call returns its expected status.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int model, width, height;
    double fx, fy, cx, cy, k[4], fov_deg;
} or_camera;

typedef struct {
    int levels, warps, iters, reg;
    double lambda, alpha0, alpha1, beta, eta, du_max, theta_gamma;
    int data_term;
} or_params;

typedef struct vfso_rig vfso_rig;
int vfso_params_default(or_params *out);
int vfso_rig_create(const or_camera *c0, const or_camera *c1, const double R[9], const double t[3], int levels,
                    vfso_rig **out);
void vfso_rig_destroy(vfso_rig *r);
int vfso_rig_field(const vfso_rig *r, int level, int which, double *dst);
int vfso_solve(vfso_rig *r, const double *I0, const double *I1, double *u, double *w, double *depth, double *z,
               unsigned char *valid, const or_params *params);
int vfso_energy(int W, int H, const or_params *params, const double *T, const unsigned char *m, const double *Iu,
                const double *rho, const double *u, const double *v, double *out);

static double tex(double x, double y)
{
    return 0.5 + 0.15 * cos(0.31 * x + 0.17 * y) + 0.1 * cos(0.11 * x - 0.43 * y + 1.0) + 0.05 * sin(0.7 * y);
}

int main(void)
{
    const int W = 64, H = 48, L = 3;
    or_camera c = {2, W, H, 20.0, 20.0, 31.5, 23.5, {0.01, -0.005, 0.0, 0.0}, 180.0};
    const double a = 2.0 * 3.14159265358979323846 / 180.0;
    double R[9] = {cos(a), 0, sin(a), 0, 1, 0, -sin(a), 0, cos(a)}, t[3] = {0.1, 0.0, 0.0}, z3[3] = {0, 0, 0};
    vfso_rig *rig = NULL;
    if (vfso_rig_create(&c, &c, R, z3, L, &rig) != -5) return 1;
    if (vfso_rig_create(&c, &c, R, t, 6, &rig) != -1) return 2;  /* 48 is not divisible by 32 */
    if (vfso_rig_create(&c, &c, R, t, L, &rig) != 0) return 3;
    size_t n = (size_t)W * H;
    double *I0 = malloc(n * sizeof(double)), *I1 = malloc(n * sizeof(double));
    double *u = malloc(n * sizeof(double)), *w = malloc(2 * n * sizeof(double)), *d = malloc(n * sizeof(double));
    double *zz = malloc(n * sizeof(double)), *f = malloc(2 * n * sizeof(double));
    unsigned char *valid = malloc(n), *m = malloc(n);
    double *T = malloc(3 * n * sizeof(double)), *v = malloc(2 * n * sizeof(double));
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            I0[i * W + j] = tex(j, i);
            I1[i * W + j] = tex(j - 0.8, i);
        }
    or_params p;
    if (vfso_params_default(&p)) return 4;
    p.levels = L;
    p.warps = 2;
    p.iters = 10;
    for (int reg = 0; reg < 2; ++reg)
        for (int dt = 0; dt < 3; ++dt) {
            p.reg = reg;
            p.data_term = dt;
            p.theta_gamma = dt == 1 ? 0.3 : 0.0;
            if (vfso_solve(rig, I0, I1, u, w, d, zz, valid, &p)) return 5;
        }
    for (int l = 0; l < L; ++l) {
        if (vfso_rig_field(rig, l, 0, f)) return 6;
        if (vfso_rig_field(rig, l, 2, f)) return 7;
    }
    if (vfso_rig_field(rig, 0, 1, f)) return 8;
    if (vfso_rig_field(rig, 1, 1, f) != -1) return 9;
    for (size_t i = 0; i < n; ++i) {
        m[i] = 1;
        T[3 * i] = 1.0;
        T[3 * i + 1] = 0.1;
        T[3 * i + 2] = 0.9;
        v[2 * i] = 0.01 * (double)(i % 7);
        v[2 * i + 1] = -0.02;
        d[i] = 0.05 * cos(0.3 * (double)i);      /* I_u */
        zz[i] = 0.02 * sin(0.2 * (double)i);     /* rho_c */
    }
    double e = 0.0;
    p.reg = 0;
    if (vfso_energy(W, H, &p, T, m, d, zz, u, v, &e) || !(e == e) || !(e < 1e300)) return 10;
    vfso_rig_destroy(rig);
    free(I0); free(I1); free(u); free(w); free(d); free(zz); free(f); free(valid); free(m); free(T); free(v);
    printf("oracle sanitized run: ok\n");
    return 0;
}
