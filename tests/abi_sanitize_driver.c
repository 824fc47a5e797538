/*
 * Host-side argument validation of every entry point of include/vfs.h,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
 * code (tests/test_sanitizers.py builds and runs it, without a GPU): each
 * call below is rejected before any device work and must return the stated
 * status; vfs_rectify_rotations, which is host-only, also runs on valid
 * input.  Exits 0 when every status is as expected.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "vfs.h"

static int fails = 0;
#define EXPECT(call, want)                                                                   \
    do {                                                                                     \
        const int got_ = (int)(call);                                                        \
        if (got_ != (want)) {                                                                \
            fprintf(stderr, "%s:%d: %s returned %d, expected %d (%s)\n", __FILE__, __LINE__, \
                    #call, got_, (int)(want), vfs_last_error());                             \
            ++fails;                                                                         \
        }                                                                                    \
    } while (0)

int main(void)
{
    vfs_params p;
    EXPECT(vfs_params_default(&p), VFS_OK);
    EXPECT(vfs_params_default(NULL), VFS_E_INVALID);
    p.levels = 3;
    vfs_camera c = {VFS_KANNALA_BRANDT, 64, 48, 20.0, 20.0, 31.5, 23.5, {0.01, -0.005, 0.0, 0.0}, 180.0};
    vfs_camera bad = c;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[3] = {0.1, 0, 0}, t0[3] = {0, 0, 0};
    vfs_rig* rig = NULL;
    EXPECT(vfs_rig_create(&c, &c, R, t0, 3, NULL, &rig), VFS_E_DEGENERATE);
    EXPECT(vfs_rig_create(&c, &c, R, t, 6, NULL, &rig), VFS_E_INVALID);
    EXPECT(vfs_rig_create(&c, &c, R, t, 0, NULL, &rig), VFS_E_INVALID);
    EXPECT(vfs_rig_create(NULL, &c, R, t, 3, NULL, &rig), VFS_E_INVALID);
    EXPECT(vfs_rig_create(&c, &c, R, t, 3, NULL, NULL), VFS_E_INVALID);
    bad.k[3] = -0.05;
    bad.fov_deg = 200.0;
    EXPECT(vfs_rig_create(&bad, &c, R, t, 3, NULL, &rig), VFS_E_MODEL);
    bad = c;
    bad.model = VFS_PINHOLE;
    EXPECT(vfs_rig_create(&bad, &bad, R, t, 3, NULL, &rig), VFS_E_MODEL);
    bad = c;
    bad.width = 32;
    EXPECT(vfs_rig_create(&c, &bad, R, t, 3, NULL, &rig), VFS_E_INVALID);
    bad = c;
    bad.model = VFS_ENHANCED_UNIFIED;
    bad.k[0] = 1.5;
    EXPECT(vfs_rig_create(&bad, &bad, R, t, 3, NULL, &rig), VFS_E_INVALID);
    double Rn[9] = {NAN, 0, 0, 0, 1, 0, 0, 0, 1};
    EXPECT(vfs_rig_create(&c, &c, Rn, t, 3, NULL, &rig), VFS_E_INVALID);
    EXPECT(vfs_rig_field(NULL, 0, 0, (void*)16, 64, NULL), VFS_E_INVALID);
    EXPECT(vfs_rig_graphs(NULL, 1), VFS_E_INVALID);

    const float* img[1] = {(const float*)16};
    float* out[1] = {(float*)16};
    EXPECT(vfs_solve_batch(NULL, 1, img, img, 256, out, out, out, NULL, NULL, &p, NULL, NULL, NULL), VFS_E_INVALID);
    EXPECT(vfs_solve(NULL, img[0], img[0], 256, out[0], out[0], out[0], NULL, NULL, &p, NULL), VFS_E_INVALID);
    EXPECT(vfs_solve_batch_noalloc(NULL, 1, img, img, 256, out, out, out, NULL, NULL, &p, NULL, NULL, NULL),
           VFS_E_INVALID);
    vfs_probe pr;
    memset(&pr, 0, sizeof(pr));
    EXPECT(vfs_solve_probe(NULL, 1, img, img, 256, &p, NULL, NULL, &pr, NULL), VFS_E_INVALID);

    void* d = (void*)16;
    EXPECT(vfs_step_tensor(0, 4, 4, d, d, 9.0, 0.85, d, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_tensor(8, 4, 4, d, d, 9.0, 0.85, d, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_tensor(8, 4, 8, d, d, -1.0, 0.85, d, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_rank(8, 4, 4, d, d, d, d, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_gradient(8, 4, 8, NULL, d, d, d, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_linearise(8, 4, 8, d, d, d, d, d, d, d, d, d, d, 1, 0, 0.0, NULL), VFS_E_INVALID);
    vfs_params pb = p;
    pb.alpha1 = 0.0;
    EXPECT(vfs_step_pd(8, 8, 8, d, d, d, d, d, d, d, d, d, d, d, &pb, 3, NULL), VFS_E_INVALID);
    pb = p;
    pb.pass_iters = 5;
    EXPECT(vfs_step_pd(8, 8, 8, d, d, d, d, d, d, d, d, d, d, d, &pb, 3, NULL), VFS_E_INVALID);
    pb = p;
    pb.storage = 7;
    EXPECT(vfs_step_pd(8, 8, 8, d, d, d, d, d, d, d, d, d, d, d, &pb, 3, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_pd(8, 8, 8, d, d, d, d, NULL, d, d, d, d, d, d, &p, 3, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_upsample(4, 4, 2, d, d, d, 8, d, d, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_triangulate(NULL, 8, d, d, d, d, NULL), VFS_E_INVALID);
    double e;
    EXPECT(vfs_step_energy(8, 8, 8, d, d, d, d, NULL, &p, &e, NULL), VFS_E_INVALID);
    EXPECT(vfs_step_pd_energy(8, 8, 8, d, d, d, d, d, d, d, d, d, d, d, &p, 0, &e, NULL), VFS_E_INVALID);
    EXPECT(vfs_diff_stats(0, 8, 8, d, d, NULL, NULL, NULL, NULL, NULL), VFS_E_INVALID);
    EXPECT(vfs_profile_enable(NULL, 1), VFS_E_INVALID);
    EXPECT(vfs_profile_read(NULL, NULL, NULL, NULL, 0), VFS_E_INVALID);

    /* host-only: the rectifying orientation of a rotated rig */
    const double a = 0.05;
    double Rr[9] = {cos(a), 0, sin(a), 0, 1, 0, -sin(a), 0, cos(a)}, Rv0[9], Rv1[9], b = 0.0;
    EXPECT(vfs_rectify_rotations(Rr, t, Rv0, Rv1, &b), VFS_OK);
    if (fabs(b - 0.1) > 1e-15) ++fails;
    EXPECT(vfs_rectify_rotations(Rr, t0, Rv0, Rv1, &b), VFS_E_INVALID);
    double tz[3] = {0, 0, 0.1};
    EXPECT(vfs_rectify_rotations(R, tz, Rv0, Rv1, &b), VFS_E_MODEL);
    EXPECT(vfs_rectify(NULL, Rv0, &c, d, 64, d, 64, NULL, NULL), VFS_E_INVALID);
    vfs_camera pin = c;
    pin.model = VFS_PINHOLE;
    pin.fov_deg = 90.0;
    EXPECT(vfs_unrectify(&c, Rv0, &c, d, NULL, 64, d, 64, NULL, NULL), VFS_E_INVALID);
    EXPECT(vfs_rectify(&c, Rv0, &pin, NULL, 64, d, 64, NULL, NULL), VFS_E_INVALID);

    vfs_server_config cfg;
    EXPECT(vfs_server_config_default(&cfg), VFS_OK);
    vfs_server* sv = NULL;
    vfs_server_config bc = cfg;
    bc.max_slots = 0;
    EXPECT(vfs_server_create(&bc, &p, &sv), VFS_E_INVALID);
    bc = cfg;
    bc.mode = 2;
    EXPECT(vfs_server_create(&bc, &p, &sv), VFS_E_INVALID);
    bc = cfg;
    bc.hbm_budget_bytes = 0;
    EXPECT(vfs_server_create(&bc, &p, &sv), VFS_E_INVALID);
    pb = p;
    pb.warps = 0;
    EXPECT(vfs_server_create(&cfg, &pb, &sv), VFS_E_INVALID);
    EXPECT(vfs_server_create(&cfg, &p, NULL), VFS_E_INVALID);
    unsigned long long tk;
    EXPECT(vfs_server_submit(NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 9.0, 0.85, &tk), VFS_E_INVALID);
    int done;
    EXPECT(vfs_server_poll(NULL, 1, &done, NULL), VFS_E_INVALID);
    EXPECT(vfs_server_times(NULL, 1, NULL, NULL), VFS_E_INVALID);
    EXPECT(vfs_server_wait_all(NULL, 1.0), VFS_E_INVALID);
    vfs_server_counters cn;
    EXPECT(vfs_server_stats(NULL, &cn), VFS_E_INVALID);
    size_t bytes;
    EXPECT(vfs_server_request_bytes(NULL, NULL, &bytes), VFS_E_INVALID);
    if (fails) return 1;
    printf("library argument validation under sanitizers: ok\n");
    return 0;
}
