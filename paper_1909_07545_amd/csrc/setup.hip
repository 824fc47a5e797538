// Once-per-calibration set-up in double precision: calibration field
// (Sec. IV-A) and, per pyramid level, the trajectory field (Sec. III-B,
// Eqs. (6)-(7)), the circular mask (Sec. IV-B), the epipole guard and the
// per-pixel flag byte used by every later step.
#include "vfs_internal.h"

namespace vfs {

namespace {

// Calibration field: a point of the unit sphere seen at x by camera 0 is
// seen by camera 1 at pi1(R r0(x)); c(x) = pi1(R r0) - pi0(r0) (zero
// translation, so the surface depth does not matter).
__global__ void calibration_kernel(RigGeom g, float2* calib, int pitch)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= g.cam0.width || i >= g.cam0.height) return;
    double r0[3], X1[3], x0[2], x1[2];
    cam_ray(g.cam0, j, i, r0);
    for (int a = 0; a < 3; ++a) X1[a] = g.R[3 * a] * r0[0] + g.R[3 * a + 1] * r0[1] + g.R[3 * a + 2] * r0[2];
    float2 c = make_float2(0.f, 0.f);
    if (cam_pixel(g.cam0, r0, x0) && cam_pixel(g.cam1, X1, x1))
        c = make_float2(float(x1[0] - x0[0]), float(x1[1] - x0[1]));
    calib[(size_t)i * pitch + j] = c;
}

// Mask of camera 0 at a level-0 pixel: r_d(x) <= r_d(FOV/2).
__device__ inline bool mask0_at(const RigGeom& g, int I, int J)
{
    const double mx = (J - g.cam0.cx) / g.cam0.fx, my = (I - g.cam0.cy) / g.cam0.fy;
    return sqrt(mx * mx + my * my) <= g.rmax0;
}

// The direction seen at level-0 pixel (J, I) lies inside camera 1's field of view.
__device__ inline bool seen_by_cam1(const RigGeom& g, int I, int J)
{
    double r0[3], X1[3], x0[2], x1[2];
    cam_ray(g.cam0, J, I, r0);
    for (int a = 0; a < 3; ++a) X1[a] = g.R[3 * a] * r0[0] + g.R[3 * a + 1] * r0[1] + g.R[3 * a + 2] * r0[2];
    if (!cam_pixel(g.cam0, r0, x0) || !cam_pixel(g.cam1, X1, x1)) return false;
    return atan2(sqrt(X1[0] * X1[0] + X1[1] * X1[1]), X1[2]) <= g.half1;
}

// Level-l pixel (j, i) -> level-0 pixel of its nearest-neighbour sample.
__device__ inline int nn0(int v, int l) { return l > 0 ? (v << l) + (1 << (l - 1)) : v; }

__global__ void level_fields_kernel(RigGeom g, int l, float2* gamma, uint8_t* flags, int pitch)
{
    const Cam cl = cam_level(g.cam0, l);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= cl.width || i >= cl.height) return;

    // trajectory tangent: flow of the unit-sphere point under a vanishing
    // translation eps t'/|t'|, normalised
    double r0[3], X1[3], x0[2], x1[2];
    cam_ray(cl, j, i, r0);
    for (int a = 0; a < 3; ++a) X1[a] = r0[a] + g.eps * g.tdir[a];
    const double ct = r0[0] * g.tdir[0] + r0[1] * g.tdir[1] + r0[2] * g.tdir[2];
    const bool epi = fabs(ct) > g.cos_guard;
    float2 gm = make_float2(0.f, 0.f);
    if (!epi && cam_pixel(cl, r0, x0) && cam_pixel(cl, X1, x1)) {
        const double gx = x1[0] - x0[0], gy = x1[1] - x0[1];
        const double n = sqrt(gx * gx + gy * gy);
        if (n > 0.0) gm = make_float2(float(gx / n), float(gy / n));
    }
    gamma[(size_t)i * pitch + j] = gm;

    // masks (nearest-neighbour scaled from level 0) and data-term switch
    const int I = nn0(i, l), J = nn0(j, l);
    const bool m = mask0_at(g, I, J);
    const bool mr = (j + 1 < cl.width) && mask0_at(g, I, nn0(j + 1, l));
    const bool md = (i + 1 < cl.height) && mask0_at(g, nn0(i + 1, l), J);
    const bool d = m && seen_by_cam1(g, I, J) && !epi;
    uint8_t f = 0;
    if (m) f |= F_MASK;
    if (m && mr) f |= F_MX;
    if (m && md) f |= F_MY;
    if (d) f |= F_DATA;
    if (epi) f |= F_EPI;
    flags[(size_t)i * pitch + j] = f;
}

}  // namespace

void launch_calibration(const RigGeom& g, float2* calib, int pitch, hipStream_t s)
{
    dim3 blk(64), grd((g.cam0.width + 63) / 64, g.cam0.height);
    hipLaunchKernelGGL(calibration_kernel, grd, blk, 0, s, g, calib, pitch);
}

void launch_level_fields(const RigGeom& g, int level, float2* gamma, uint8_t* flags, int pitch, hipStream_t s)
{
    const int W = g.cam0.width >> level, H = g.cam0.height >> level;
    dim3 blk(64), grd((W + 63) / 64, H);
    hipLaunchKernelGGL(level_fields_kernel, grd, blk, 0, s, g, level, gamma, flags, pitch);
}

}  // namespace vfs
