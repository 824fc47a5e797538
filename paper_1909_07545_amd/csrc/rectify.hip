// Resampling between a camera and a rotated virtual pinhole view: the
// rectification of a conventional pipeline, which the paper compares against
// (Sec. V-A: the same energy run on rectified images), and the way back, to
// show a rectified result on the original image.  Geometry in double
// precision (the camera models of the set-up), samples bilinear in float.
#include "vfs_internal.h"

namespace vfs {

namespace {

__device__ inline int clamp_i(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Positions this close (pixels) outside a plane still count as inside: the
// border pixels of a view land there by rounding (the taps are clamped).
constexpr double kEdge = 1e-6;

__device__ inline bool inside(double x, double y, int W, int H)
{
    return x >= -kEdge && x <= W - 1.0 + kEdge && y >= -kEdge && y <= H - 1.0 + kEdge;
}

// Bilinear sample at an absolute position, taps clamped to the plane.
__device__ inline float sample(const float* I, size_t pitch, int W, int H, double x, double y)
{
    const double fx0 = floor(x), fy0 = floor(y);
    const float ax = float(x - fx0), ay = float(y - fy0);
    const int x0 = int(fx0), y0 = int(fy0);
    const int xa = clamp_i(x0, 0, W - 1), xb = clamp_i(x0 + 1, 0, W - 1);
    const int ya = clamp_i(y0, 0, H - 1), yb = clamp_i(y0 + 1, 0, H - 1);
    const float* ra = I + (size_t)ya * pitch;
    const float* rb = I + (size_t)yb * pitch;
    return (1.f - ax) * (1.f - ay) * ra[xa] + ax * (1.f - ay) * ra[xb] + (1.f - ax) * ay * rb[xa] + ax * ay * rb[xb];
}

// One virtual pixel per thread: its ray in the camera frame is Rv^T applied
// to ((x - cx) / fx, (y - cy) / fy, 1); it samples the camera image where
// the camera sees that ray, if that is inside the camera's circular mask.
__global__ void rectify_kernel(RectifyGeom g, const float* src, size_t src_pitch, float* dst, size_t dst_pitch,
                               uint8_t* valid)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= g.pin.width || i >= g.pin.height) return;
    const double v[3] = {(j - g.pin.cx) / g.pin.fx, (i - g.pin.cy) / g.pin.fy, 1.0};
    double X[3], x[2];
    for (int a = 0; a < 3; ++a) X[a] = g.Rv[a] * v[0] + g.Rv[3 + a] * v[1] + g.Rv[6 + a] * v[2];
    float out = 0.f;
    uint8_t ok = 0;
    if (cam_pixel(g.cam, X, x)) {
        const double mx = (x[0] - g.cam.cx) / g.cam.fx, my = (x[1] - g.cam.cy) / g.cam.fy;
        const bool in_view = atan2(sqrt(X[0] * X[0] + X[1] * X[1]), X[2]) <= g.half;
        if (in_view && sqrt(mx * mx + my * my) <= g.rmax && inside(x[0], x[1], g.cam.width, g.cam.height)) {
            out = sample(src, src_pitch, g.cam.width, g.cam.height, x[0], x[1]);
            ok = 1;
        }
    }
    dst[(size_t)i * dst_pitch + j] = out;
    if (valid) valid[(size_t)i * dst_pitch + j] = ok;
}

// One camera pixel per thread, inside the camera's mask: its ray rotated
// into the virtual view; if it lands inside the view with all four bilinear
// taps valid, the field sampled there.
__global__ void unrectify_kernel(RectifyGeom g, const float* field, const uint8_t* field_valid, size_t field_pitch,
                                 float* dst, size_t dst_pitch, uint8_t* valid)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= g.cam.width || i >= g.cam.height) return;
    float out = 0.f;
    uint8_t ok = 0;
    const double mx = (j - g.cam.cx) / g.cam.fx, my = (i - g.cam.cy) / g.cam.fy;
    if (sqrt(mx * mx + my * my) <= g.rmax) {
        double r[3], V[3];
        cam_ray(g.cam, j, i, r);
        for (int a = 0; a < 3; ++a) V[a] = g.Rv[3 * a] * r[0] + g.Rv[3 * a + 1] * r[1] + g.Rv[3 * a + 2] * r[2];
        if (V[2] > 0.0) {
            const double px = g.pin.cx + g.pin.fx * V[0] / V[2], py = g.pin.cy + g.pin.fy * V[1] / V[2];
            const int Wp = g.pin.width, Hp = g.pin.height;
            if (inside(px, py, Wp, Hp)) {
                bool taps = true;
                if (field_valid) {
                    const int x0 = int(floor(px)), y0 = int(floor(py));
                    const int xa = clamp_i(x0, 0, Wp - 1), xb = clamp_i(x0 + 1, 0, Wp - 1);
                    const int ya = clamp_i(y0, 0, Hp - 1), yb = clamp_i(y0 + 1, 0, Hp - 1);
                    taps = field_valid[(size_t)ya * field_pitch + xa] && field_valid[(size_t)ya * field_pitch + xb] &&
                           field_valid[(size_t)yb * field_pitch + xa] && field_valid[(size_t)yb * field_pitch + xb];
                }
                if (taps) {
                    out = sample(field, field_pitch, Wp, Hp, px, py);
                    ok = 1;
                }
            }
        }
    }
    dst[(size_t)i * dst_pitch + j] = out;
    if (valid) valid[(size_t)i * dst_pitch + j] = ok;
}

}  // namespace

void launch_rectify(const RectifyGeom& g, const float* src, size_t src_pitch, float* dst, size_t dst_pitch,
                    uint8_t* valid, hipStream_t s)
{
    const dim3 grid((g.pin.width + 63) / 64, g.pin.height);
    hipLaunchKernelGGL(rectify_kernel, grid, dim3(64), 0, s, g, src, src_pitch, dst, dst_pitch, valid);
}

void launch_unrectify(const RectifyGeom& g, const float* field, const uint8_t* field_valid, size_t field_pitch,
                      float* dst, size_t dst_pitch, uint8_t* valid, hipStream_t s)
{
    const dim3 grid((g.cam.width + 63) / 64, g.cam.height);
    hipLaunchKernelGGL(unrectify_kernel, grid, dim3(64), 0, s, g, field, field_valid, field_pitch, dst, dst_pitch,
                       valid);
}

}  // namespace vfs
