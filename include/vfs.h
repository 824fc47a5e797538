/*
 * vfs.h -- C ABI of the MI355X (gfx950) implementation of non-rectified
 * variational fisheye stereo (Roxas & Oishi, "Real-Time Variational Fisheye
 * Stereo without Rectification and Undistortion", arXiv 1909.07545).
 *
 * The calls follow the paper's statement of the problem: a calibration
 * (fisheye intrinsics of both cameras and the pose X1 = R X0 + t) becomes a
 * rig holding the trajectory fields (Sec. III-B) and the calibration field
 * (Sec. IV-A); an image pair becomes the scalar displacement u along the
 * epipolar curves, the warping vectors w (Sec. III-C, Eqs. (8)-(9)) and the
 * triangulated depth (Sec. III-D, last paragraph), by Algorithm 1 run inside
 * the coarse-to-fine scheme of Sec. IV-B.
 *
 * Conventions shared by every call:
 *  - Images are row-major float32, intensities in [0, 1]; pixel (i = row,
 *    j = column) sits at integer coordinates (j, i) (pixel centres).
 *  - Every pointer argument marked "device" is memory of the current HIP
 *    device (for example a torch CUDA tensor's data_ptr()); "host" pointers
 *    are ordinary process memory.  Pitches are in bytes.
 *  - Work is enqueued asynchronously on the hip_stream argument (a
 *    hipStream_t; NULL means the default stream).  No call synchronises the
 *    stream except where stated.  Device faults surface at the caller's next
 *    synchronisation.
 *  - Every call returns a vfs_status; arguments are validated before any
 *    device work is enqueued, and nothing is enqueued on error.  The message
 *    of the last error of the calling thread is vfs_last_error().
 *  - The library owns rig handles and their device memory (freed by
 *    vfs_rig_destroy); the caller owns every image and output buffer and must
 *    keep them alive until the enqueued work completes.
 */
#ifndef VFS_H
#define VFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VFS_OK = 0,
    VFS_E_INVALID = -1,     /* bad argument: null pointer, size, pitch, count */
    VFS_E_NOMEM = -2,       /* device allocation failed */
    VFS_E_BUDGET = -3,      /* request exceeds a configured memory budget */
    VFS_E_MODEL = -4,       /* camera model not invertible on its field of view */
    VFS_E_DEGENERATE = -5,  /* zero baseline: no trajectory field (Sec. III-B needs |t| != 0) */
    VFS_E_DEVICE = -6       /* a HIP runtime call failed */
} vfs_status;

typedef enum {
    VFS_PINHOLE = 0,
    VFS_EQUIDISTANT = 1,
    VFS_KANNALA_BRANDT = 2,
    VFS_UNIFIED = 3,            /* k[0] = xi */
    VFS_ENHANCED_UNIFIED = 4    /* k[0] = alpha, k[1] = beta */
} vfs_model;
typedef enum { VFS_TGV = 0, VFS_TV = 1 } vfs_reg;
/* Image the data term compares (Sec. III-A allows any image I): the
 * intensities; or at every pyramid level the rank transform of the level's
 * images (the share of the 5x5 neighbours strictly darker than the pixel; a
 * census variant, unchanged by any increasing change of the intensities,
 * e.g. gain, offset, gamma); or the gradient magnitude of the level's images
 * (sqrt(Ix^2 + Iy^2), central differences; gradient constancy, unchanged by
 * an added constant).  The tensor of Eq. (12) keeps the intensities.  Both
 * transformed images call for their own lambda (rank: about 15). */
typedef enum { VFS_DATA_BRIGHTNESS = 0, VFS_DATA_RANK = 1, VFS_DATA_GRADIENT = 2 } vfs_data_term;
/* Storage of the dual variables and of the tensor pack (T^(1/2) of Eq. (12)
 * and I_u): 32-bit float, IEEE half or bfloat16; every update is computed in
 * FP32 and u, v, rho_c stay FP32 (rho_c is formed from I_u as stored). */
typedef enum { VFS_F32 = 0, VFS_F16 = 1, VFS_BF16 = 2 } vfs_storage;

/* Camera (Sec. III-B: any model with a defined projection; Sec. III-D names
 * the unified and enhanced unified models for their closed-form inverse):
 * pixel = (cx, cy) + (fx, fy) r_d(theta) (cos phi, sin phi) for a ray at
 * angle theta from the axis and azimuth phi, with
 *   Kannala-Brandt  r_d = theta + k1 theta^3 + k2 theta^5 + k3 theta^7 + k4 theta^9
 *                   (equidistant is k = 0; pinhole r_d = tan theta),
 *   unified         r_d = sin theta / (xi + cos theta)            (k[0] = xi >= 0),
 *   enh. unified    r_d = sin theta / (alpha sqrt(beta sin^2 theta + cos^2 theta)
 *                                      + (1 - alpha) cos theta)   (k[0] = alpha in [0, 1], k[1] = beta > 0).
 * fov_deg is the full field of view of the circular mask of Sec. IV-B; the
 * radial map must be defined and increasing up to half of it. */
typedef struct {
    int model;             /* vfs_model */
    int width, height;
    double fx, fy, cx, cy;
    double k[4];
    double fov_deg;
} vfs_camera;

/* Solver parameters.  Defaults (vfs_params_default) are the values printed
 * in Sec. IV-C: alpha0 = 17, alpha1 = 1.2, beta = 9, eta = 0.85, and the
 * 0.2 px clip of Sec. III-C; lambda (not printed) defaults to 50;
 * theta_gamma = 0 selects the constant over-relaxation theta = 1, > 0 the
 * accelerated schedule theta_k = 1/sqrt(1 + 2 gamma s_k) on the scalar
 * factor s_k of the preconditioned steps. */
typedef struct {
    int levels, warps, iters;  /* pyramid levels (scale 1/2), warps per level, primal-dual iterations per warp */
    int reg;                   /* vfs_reg: TGV-L1 of Eq. (10), or TV-L1 (v = 0) */
    double lambda, alpha0, alpha1, beta, eta, du_max, theta_gamma;
    int storage;               /* vfs_storage */
    int pass_iters;            /* primal-dual iterations per pass over memory of the dominant launches:
                                  0 = chosen by the library from the pair size and storage (from 2 M
                                  level-0 pixels: 4 in FP32, 3 with 16-bit storage; else 3), or 2,
                                  3, 4; the choice changes only the rounding points of 16-bit
                                  storage and the speed */
    int data_term;             /* vfs_data_term */
} vfs_params;

typedef struct vfs_rig vfs_rig;

/* Fill *out with the defaults above and levels = 5, warps = 10, iters = 100. */
vfs_status vfs_params_default(vfs_params* out);

/* Rig set-up, once per calibration and resolution (Sec. III-B, Sec. IV-A,
 * Sec. IV-B).  cam0 and cam1 (host) must have equal width and height, both
 * divisible by 2^(levels-1), width at most 2^20; R (host, 9 doubles, row-major) and t (host, 3
 * doubles) give X1 = R X0 + t.  Computes in double precision on the device,
 * for every level l: the trajectory field gamma'_l (unit tangents of the
 * epipolar curves of the pre-rotated pair, by projecting the unit sphere
 * into camera 0 and into camera 0 moved by a vanishing step along
 * t' = R^T t), the circular mask M_l (nearest-neighbour scaled), the
 * epipole guard (2 degrees around +-t'), and at level 0 the calibration
 * field c(x) = pi1(R r0(x)) - pi0(r0(x)).  The rig keeps them in device
 * memory.  Synchronises hip_stream before returning.
 * Errors: VFS_E_INVALID, VFS_E_MODEL (radial map not increasing on
 * [0, FOV/2], or pinhole FOV >= 180), VFS_E_DEGENERATE (t = 0),
 * VFS_E_NOMEM, VFS_E_DEVICE. */
vfs_status vfs_rig_create(const vfs_camera* cam0, const vfs_camera* cam1, const double R[9],
                          const double t[3], int levels, void* hip_stream, vfs_rig** out);

void vfs_rig_destroy(vfs_rig* rig);

/* Copy a rig field of one level into dst (device), rows of pitch_bytes:
 *   which = 0: trajectory field, float32 pairs (gx, gy) per pixel;
 *   which = 1: calibration field (level 0 only), float32 pairs;
 *   which = 2: flags, one byte per pixel: bit0 mask M, bit1 mx (M at P and
 *              P+x), bit2 my, bit3 data term on (mask, inside camera 1's
 *              view after pre-rotation, not near an epipole), bit4 epipole.
 * Errors: VFS_E_INVALID (level / which / pitch), VFS_E_DEVICE. */
vfs_status vfs_rig_field(const vfs_rig* rig, int level, int which, void* dst, size_t pitch_bytes,
                         void* hip_stream);

/* Whole method on n image pairs of one rig (Algorithm 1 in the pyramid of
 * Sec. IV-B, after the pre-rotation of Sec. IV-A, then triangulation).
 * I0[b], I1[b] (device) are H x W float32 images with row pitch
 * pitch_bytes; outputs (device, row pitch pitch_bytes for u/depth/z,
 * 2*pitch_bytes for w, pitch_bytes/4 for valid) per pair b:
 *   u_out[b]     displacement along the epipolar curve (level-0 pixels),
 *   w_out[b]     warping vectors, float32 pairs (wx, wy),
 *   depth_out[b] range along the camera-0 ray (+inf where invalid),
 *   z_out[b]     its z coordinate (may be NULL),
 *   valid_out[b] 1 where the depth is valid (may be NULL).
 * betas / etas (host, n doubles each, may be NULL): per-pair tensor
 * parameters overriding params->beta / eta (Eq. (12)).  params (host) must
 * have params->levels equal to the rig's.  The library keeps one device
 * workspace per rig, grown on demand (allocation happens here, outside the
 * enqueued work); n <= VFS_MAX_BATCH.
 * Errors: VFS_E_INVALID, VFS_E_NOMEM, VFS_E_DEVICE. */
#define VFS_MAX_BATCH 32
vfs_status vfs_solve_batch(vfs_rig* rig, int n, const float* const* I0, const float* const* I1,
                           size_t pitch_bytes, float* const* u_out, float* const* w_out,
                           float* const* depth_out, float* const* z_out, uint8_t* const* valid_out,
                           const vfs_params* params, const double* betas, const double* etas,
                           void* hip_stream);

/* Graph replay of the direct solves (the fixed iteration counts of Sec. IV-C
 * make a solve one fixed sequence of launches).  With enable = 1 (the
 * default) the first vfs_solve / vfs_solve_batch of a launch configuration
 * (batch size n and every solver parameter but beta and eta) on a rig
 * captures its launches into a HIP graph, and later solves of that
 * configuration replay it: one graph launch on hip_stream, after the pairs'
 * descriptors are written.  Results are the same as eager launches, bit for
 * bit.  The rig keeps up to 8 graphs (all dropped when a ninth is needed)
 * until vfs_rig_destroy; enable = 0 drops them and launches eagerly.  Solves
 * with profiling on (vfs_profile_enable) always launch eagerly.
 * Errors: VFS_E_INVALID (NULL rig). */
vfs_status vfs_rig_graphs(vfs_rig* rig, int enable);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * vfs_solve_batch with the same arguments, kernels and results, but the
 * pairs' solve state and descriptors live in a fixed device array of the
 * library (VFS_NOALLOC_SCRATCH_BYTES, held on each device the call runs on
 * until the process ends) instead of the rig's workspace; no device memory
 * is allocated or freed.  The state of n pairs must fit: n x (about 149
 * bytes per level-0 pixel in FP32, 109 with 16-bit storage) plus 16 KB of
 * descriptors, e.g. one 640x480 FP32 pair or 26 128x128 pairs; a larger
 * request returns VFS_E_BUDGET before any device work.  Every call on a
 * device shares that device's array: calls that overlap on one device (on
 * different streams or threads) race and must not be made.  The solve
 * writes every state value before reading it, so nothing carries over from
 * the previous call.  Errors: those of vfs_solve_batch, VFS_E_BUDGET. */
#define VFS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vfs_status vfs_solve_batch_noalloc(vfs_rig* rig, int n, const float* const* I0, const float* const* I1,
                                   size_t pitch_bytes, float* const* u_out, float* const* w_out,
                                   float* const* depth_out, float* const* z_out, uint8_t* const* valid_out,
                                   const vfs_params* params, const double* betas, const double* etas,
                                   void* hip_stream);

/* One pair: vfs_solve_batch with n = 1. */
vfs_status vfs_solve(vfs_rig* rig, const float* I0, const float* I1, size_t pitch_bytes, float* u_out,
                     float* w_out, float* depth_out, float* z_out, uint8_t* valid_out,
                     const vfs_params* params, void* hip_stream);

/* ---- Test hook: the state of a whole solve part-way through, for checking
 * one warp of Algorithm 1 (the linearisation of Eqs. (3), (5); the
 * iterations of Eq. (11) with the resolvent of Eq. (13); the clip and
 * accumulation of Sec. III-C) against a reference started from exactly this
 * state.
 *
 * vfs_solve_probe enqueues the launches of vfs_solve_batch on the same n
 * pairs (same kernels, grids and batch) up to the end of warp `warp`
 * (0 <= warp < params->warps) of pyramid level `level` (0 <= level <
 * params->levels), copies pair `pair`'s state at three points of that warp,
 * and stops there: no later warp or level, no triangulation, no outputs.
 * Every destination is device memory with rows of `pitch` pixels (row bytes
 * = pitch x the plane's bytes per pixel); NULL skips a plane.  Planes are
 * level-l sized, H_l x W_l with W_l = W >> level, H_l = H >> level:
 *   after the warp's linearisation, before its iterations:
 *     J0, J1    float32: the level's pyramid images (J1 pre-rotated),
 *     u         float32: u after the previous warp's clip (= u_w),
 *     w         float32 pairs: warping vectors after that clip,
 *     v         float32 pairs (TGV): the warm-started primal v,
 *     p, q      2 and 4 values per pixel (q: TGV): the warm-started duals,
 *     tpack     4 values per pixel: (t11, t12, t22) of Eq. (12) and I_u,
 *     rho       float32: rho_c,
 *     gw        float32 pairs: the tangent at the warped point;
 *   after the iterations, before the clip: u_pd, v_pd, p_pd, q_pd;
 *   after the clip: u_next, w_next.
 * p, q and tpack (and p_pd, q_pd) hold params->storage's values: float32
 * (8, 16, 16 bytes per pixel), or IEEE half / bfloat16 (4, 8, 8 bytes).
 * Allocates like vfs_solve_batch (the rig's workspace); synchronises
 * hip_stream before returning.
 * Errors: those of vfs_solve_batch; VFS_E_INVALID for a NULL probe, level,
 * warp or pair out of range, or pitch < W_l. */
typedef struct {
    int level, warp, pair;
    size_t pitch;
    float *J0, *J1, *u, *w, *v;
    void *p, *q, *tpack;
    float *rho, *gw;
    float *u_pd, *v_pd;
    void *p_pd, *q_pd;
    float *u_next, *w_next;
} vfs_probe;
vfs_status vfs_solve_probe(vfs_rig* rig, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                           const vfs_params* params, const double* betas, const double* etas,
                           const vfs_probe* probe, void* hip_stream);

/* ---- Steps of the method on caller buffers (device), for step-by-step use
 * and testing; they use FP32 storage whatever params->storage says, except
 * vfs_step_pd, which takes its duals and tensor pack in params->storage's
 * format.  They
 * synchronise hip_stream before returning (they allocate a small temporary
 * descriptor, and vfs_step_upsample / vfs_step_triangulate temporary planes).
 * Layout: row-major with a common row pitch of `pitch`
 * ELEMENTS (not bytes) for every plane; vector planes interleave their
 * components (float2 (x, y) per pixel for w, gamma, v, p; float4 for q and
 * for the tensor pack (t11, t12, t22, I_u)).  flags as in vfs_rig_field. */

/* Eq. (12): tensor from the level image J0 and the flags (mask bit), written
 * to tpack.xyz (tpack.w set to 0).  Central differences, one-sided where a
 * neighbour leaves the image or the mask; T = I where the gradient is below
 * 1e-12 or the pixel is masked out. */
vfs_status vfs_step_tensor(int width, int height, size_t pitch, const float* J0, const uint8_t* flags,
                           double beta, double eta, float* tpack, void* hip_stream);

/* Rank transforms (VFS_DATA_RANK) of two planes: R = the share of the 5x5
 * neighbours strictly darker than each pixel, neighbours outside the plane
 * taken at the nearest edge pixel. */
vfs_status vfs_step_rank(int width, int height, size_t pitch, const float* I0, const float* I1, float* R0,
                         float* R1, void* hip_stream);

/* Gradient magnitudes (VFS_DATA_GRADIENT) of two planes: G = sqrt(Ix^2 +
 * Iy^2) with Ix = (I(x+1) - I(x-1)) / 2 and likewise Iy, neighbours outside
 * the plane taken at the nearest edge pixel.  Same arguments, layout and
 * errors as vfs_step_rank. */
vfs_status vfs_step_gradient(int width, int height, size_t pitch, const float* I0, const float* I1, float* G0,
                             float* G1, void* hip_stream);

/* Eqs. (3), (5), Sec. III-B, Algorithm 1: with clip != 0 first clip and
 * accumulate the previous warp (du = clamp(u - u_w, +-du_max), u = u_w + du,
 * w += du gamma_w); then (unless clip_only) linearise at y = x + w:
 * gamma_w = bicubic (Keys, a = -1/2) sample g of the trajectory field over
 * max(|g|, 1/2) (unit length except next to an epipole), I_u = I1(y +
 * gamma_w) - I1(y) into tpack.w, rho_c = I1(y) - I0(x) - u I_u, both 0
 * where the data term is off (flags bit3); u_w = u.  With the rank or
 * gradient data term the solver passes those planes as J0, J1. */
vfs_status vfs_step_linearise(int width, int height, size_t pitch, const float* J0, const float* J1,
                              const float* gamma, const uint8_t* flags, float* u, float* u_w, float* w,
                              float* gamma_w, float* tpack, float* rho, int clip, int clip_only,
                              double du_max, void* hip_stream);

/* Eq. (11): `iters` primal-dual iterations from a warp start (ubar = u,
 * vbar = v), with the preconditioned steps of Sec. III-D recomputed from
 * tpack and flags, the resolvent of Eq. (13), and theta per
 * params->theta_gamma, run by the kernels and pass schedule of the solves
 * (params->pass_iters).  u, v, p, q are read and overwritten; scratch_* are
 * caller buffers of the same shapes used as the second copy of the state
 * (the iteration reads one copy and writes the other).  p, q, tpack and
 * their scratch hold params->storage's values: float32 (2, 4, 4 per pixel),
 * or IEEE half / bfloat16 (2, 4, 4 16-bit values per pixel), rounded each
 * time a launch stores them; u, v, rho stay float32.  TV mode ignores v, q
 * and their scratch (may be NULL).  width at most 2^20 (VFS_E_INVALID). */
vfs_status vfs_step_pd(int width, int height, size_t pitch, const void* tpack, const float* rho,
                       const uint8_t* flags, float* u, float* v, void* p, void* q, float* scratch_u,
                       float* scratch_v, void* scratch_p, void* scratch_q, const vfs_params* params,
                       int iters, void* hip_stream);

/* Sec. IV-B: mask-aware x2 bilinear upsampling of (u, w) from a coarse level
 * (width_c x height_c, pitch_c elements, mask = flags_c bit0) to the fine
 * level (2 width_c x 2 height_c, pitch_f), multiplied by 2. */
vfs_status vfs_step_upsample(int width_c, int height_c, size_t pitch_c, const uint8_t* flags_c,
                             const float* u_c, const float* w_c, size_t pitch_f, float* u_f, float* w_f,
                             void* hip_stream);

/* Sec. III-D: triangulate level-0 warping vectors w of a rig (closest
 * approach of the rays pi0^-1(x) and pi0^-1(x + w) from -t'), in double
 * precision.  Outputs as in vfs_solve_batch. */
vfs_status vfs_step_triangulate(const vfs_rig* rig, size_t pitch, const float* w, float* depth, float* z,
                                uint8_t* valid, void* hip_stream);

/* Linearised energy of Eq. (10) at one level (A9):
 *   E = sum over the mask of lambda |rho_c + u I_u| + alpha1 |T grad u - v|_2
 *       + alpha0 |grad v|_F   (TV: v = 0, no last term),
 * with the masked forward differences of the primal-dual iteration (flags
 * bits 0-2).  Per-pixel terms in FP32, accumulated in FP64 in a fixed order
 * (the same value on every run).  *energy (host) receives E. */
vfs_status vfs_step_energy(int width, int height, size_t pitch, const float* tpack, const float* rho,
                           const uint8_t* flags, const float* u, const float* v, const vfs_params* params,
                           double* energy, void* hip_stream);

/* vfs_step_pd with the energy trace: energy (host, iters + 1 doubles)
 * receives E(x^0), E(x^1), ..., E(x^iters) of the primal iterates.  Runs one
 * iteration per launch (the same iteration as vfs_step_pd; iters >= 1). */
vfs_status vfs_step_pd_energy(int width, int height, size_t pitch, const float* tpack, const float* rho,
                              const uint8_t* flags, float* u, float* v, float* p, float* q, float* scratch_u,
                              float* scratch_v, float* scratch_p, float* scratch_q, const vfs_params* params,
                              int iters, double* energy, void* hip_stream);

/* Difference statistics of two float planes (device, pitch in elements) over
 * the pixels whose flags bit 0 is set (all pixels if flags is NULL): mean and
 * max of |a - b| and the pixel count (host outputs, each may be NULL); FP64
 * fixed-order reduction on the device. */
vfs_status vfs_diff_stats(int width, int height, size_t pitch, const float* a, const float* b,
                          const uint8_t* flags, double* mean_abs, double* max_abs, long long* count,
                          void* hip_stream);

/* ---- Rectification, for comparison with a rectified pipeline (Sec. V-A
 * runs the same energy on images rectified to a pinhole view of a chosen
 * field of view and maps its errors back onto the fisheye image).
 *
 * vfs_rectify_rotations (host only, no device work): for a rig with
 * X1 = R X0 + t (R row-major 9 doubles, t 3 doubles), rotations Rv0, Rv1
 * (row-major, caller's 9 doubles each) of a shared virtual orientation:
 * X_v = Rv0 X0 = Rv1 X1 - (b, 0, 0) with b = |t| returned in *baseline
 * (may be NULL).  Virtual x runs along R^T t, virtual y is perpendicular to
 * it and to the mean of the two optical axes, z = x cross y.  The virtual
 * pair is the pinhole rig R = I, t = (b, 0, 0), whose trajectory field is
 * (1, 0) everywhere.  VFS_E_INVALID for t = 0, VFS_E_MODEL if t lies along
 * the mean optical axis. */
vfs_status vfs_rectify_rotations(const double R[9], const double t[3], double Rv0[9], double Rv1[9],
                                 double* baseline);

/* Virtual pinhole view of a camera image: for each pixel p of `pinhole`
 * (host, model VFS_PINHOLE; its width x height is the output size), the ray
 * Rv^T ((p - c) / f, 1) is projected into `cam` (host, any model); inside
 * cam's circular mask (fov_deg) dst = bilinear sample of src there (taps
 * clamped) and valid = 1, elsewhere dst = 0 and valid = 0.  src: device,
 * cam->height rows of src_pitch floats; dst and valid (device, valid may be
 * NULL): pinhole->height rows of dst_pitch elements.  Geometry in FP64,
 * samples in FP32.  Asynchronous on hip_stream. */
vfs_status vfs_rectify(const vfs_camera* cam, const double Rv[9], const vfs_camera* pinhole, const float* src,
                       size_t src_pitch, float* dst, size_t dst_pitch, uint8_t* valid, void* hip_stream);

/* The way back: for each pixel q of `cam` inside its circular mask, the ray
 * pi^-1(q) rotated by Rv; if it lands at a point p inside the pinhole view
 * (in front of it, within [0, W-1] x [0, H-1]) and the four bilinear taps
 * around p are valid (field_valid, device, may be NULL = all valid), dst =
 * bilinear sample of field at p and valid = 1; else dst = 0, valid = 0.
 * field / field_valid: pinhole->height rows of field_pitch elements; dst /
 * valid (valid may be NULL): cam->height rows of dst_pitch elements. */
vfs_status vfs_unrectify(const vfs_camera* cam, const double Rv[9], const vfs_camera* pinhole, const float* field,
                         const uint8_t* field_valid, size_t field_pitch, float* dst, size_t dst_pitch,
                         uint8_t* valid, void* hip_stream);

/* ---- Measurement: when enabled, vfs_solve_batch records HIP events on its
 * stream around the level-0 primal-dual launches that each carry several
 * iterations of Eq. (11) in one pass over memory (the dominant kernel) and
 * accumulates their elapsed time.  vfs_profile_read synchronises the stream
 * of the last solve and returns the accumulated milliseconds, the number of
 * those launches (counts since the last reset) and the iterations each
 * launch carries (host outputs, each may be NULL). */
vfs_status vfs_profile_enable(vfs_rig* rig, int enable);
vfs_status vfs_profile_read(vfs_rig* rig, double* pd0_ms, long long* pd0_launches, int* iters_per_launch,
                            int reset);

/* ---- Serving: a request loop that batches stereo pairs of different
 * sizes and rigs as they arrive (continuous batching).
 *
 * Requests are grouped by image size and level count into buckets of up to
 * max_slots concurrent requests.  Each request admitted to a bucket owns a
 * slot and its solve state from a device pool of hbm_budget_bytes; a
 * request waits (in arrival order) until its bucket has a free slot and the
 * pool has room, and its memory returns to the pool when it completes.  A
 * bucket advances its requests together one warp step at a time: one step
 * (a "tick") is one replay of a HIP graph captured at the bucket's creation
 * (use_graphs = 1) or the same launches issued eagerly (use_graphs = 0);
 * within a tick every request runs the stages of Algorithm 1 it needs at its
 * own pyramid level and warp, so a request that arrives while others are
 * mid-solve joins at the next tick.  Buckets run on their own streams and
 * overlap on the device.  Each request's arithmetic is that of vfs_solve
 * with the server's params (its levels are its rig's), so its outputs are
 * the same as solving it alone.  Mode VFS_SERVE_PLAIN is the baseline: one
 * request at a time in arrival order, eager launches.
 *
 * A scheduler thread owned by the server does all device work (on the
 * device current at vfs_server_create).  submit / poll / times / wait_all /
 * stats may be called from any thread.  The caller keeps the rigs, images
 * and outputs of a request alive, and does not touch the outputs, until
 * the request is done. */
typedef struct vfs_server vfs_server;
typedef enum { VFS_SERVE_BATCHED = 0, VFS_SERVE_PLAIN = 1 } vfs_serve_mode;
typedef struct {
    int mode;                  /* vfs_serve_mode */
    size_t hbm_budget_bytes;   /* device pool for per-request solve state (batched mode) */
    int max_slots;             /* concurrent requests per bucket, 1 .. VFS_MAX_BATCH */
    int use_graphs;            /* batched mode: replay captured graphs (1) or launch eagerly (0) */
} vfs_server_config;
typedef struct {
    long long ticks;           /* ticks (batched) or solves (plain) so far */
    long long peak_active;     /* most requests in flight at once */
    size_t pool_peak_bytes;    /* high-water mark of the pool (batched) */
    int buckets;
    long long joins;           /* admissions into a bucket whose other requests were mid-solve */
    long long full_ticks;      /* ticks that ran start / level-change / finish stages */
} vfs_server_counters;

/* Defaults: batched, 1 GiB budget, 16 slots per bucket, graphs on. */
vfs_status vfs_server_config_default(vfs_server_config* out);

/* Create a server (and its scheduler thread).  params (host) holds the
 * solver settings of every request (params->levels is ignored: each
 * request uses its rig's level count); warps and iters must be >= 1.
 * Batched mode allocates the pool here.
 * Errors: VFS_E_INVALID, VFS_E_NOMEM, VFS_E_DEVICE. */
vfs_status vfs_server_create(const vfs_server_config* cfg, const vfs_params* params, vfs_server** out);

/* Device bytes of one request's solve state for a rig under this server. */
vfs_status vfs_server_request_bytes(const vfs_server* server, const vfs_rig* rig, size_t* bytes);

/* Queue one pair (device buffers as in vfs_solve; u_out, w_out, z_out and
 * valid_out may be NULL) with its tensor parameters (Eq. (12)); the arrival
 * time is stamped here.  *ticket (host) receives the request's id.
 * Errors: VFS_E_INVALID, VFS_E_BUDGET (one request larger than the budget),
 * or the error that stopped the server. */
vfs_status vfs_server_submit(vfs_server* server, vfs_rig* rig, const float* I0, const float* I1,
                             size_t pitch_bytes, float* u_out, float* w_out, float* depth_out, float* z_out,
                             uint8_t* valid_out, double beta, double eta, unsigned long long* ticket);

/* *done = 1 once the request's outputs are complete in device memory (the
 * scheduler has seen its last launch finish); *latency_s (may be NULL) is
 * then completion - arrival in seconds (host clock), else -1.
 * Errors: VFS_E_INVALID (unknown ticket), VFS_E_DEVICE (the request failed). */
vfs_status vfs_server_poll(vfs_server* server, unsigned long long ticket, int* done, double* latency_s);

/* Admission and completion times of a request, seconds after its arrival
 * (-1 if not yet). */
vfs_status vfs_server_times(vfs_server* server, unsigned long long ticket, double* admit_s, double* done_s);

/* Block until every submitted request is done, or timeout_s passes
 * (VFS_E_DEVICE). */
vfs_status vfs_server_wait_all(vfs_server* server, double timeout_s);

vfs_status vfs_server_stats(vfs_server* server, vfs_server_counters* out);

/* Finish the work in flight, stop the scheduler and free the server's
 * device memory. */
void vfs_server_destroy(vfs_server* server);

/* Message of the calling thread's last error ("" if none). */
const char* vfs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VFS_H */
