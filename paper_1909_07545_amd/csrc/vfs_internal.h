// Internal declarations of the gfx950 library: camera model (double
// precision, used by the once-per-calibration set-up and the triangulation),
// interpolation helpers, per-pixel flag bits, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vfs {

// ----------------------------------------------------------------- flags
enum : uint8_t {
    F_MASK = 1u,    // inside the circular field-of-view mask of the level
    F_MX = 2u,      // mask at P and at P + x (forward difference in x is on)
    F_MY = 4u,      // mask at P and at P + y
    F_DATA = 8u,    // data term on: mask, camera-1 view after pre-rotation, no epipole
    F_EPI = 16u,    // within the epipole guard
};

constexpr int kMaxLevels = 12;
constexpr int kMaxBatch = 32;

// ----------------------------------------------------------------- camera
// Kannala-Brandt radial map r_d(theta) = theta + k1 theta^3 + k2 theta^5 +
// k3 theta^7 + k4 theta^9; equidistant is k = 0, pinhole r_d = tan(theta).
struct Cam {
    int model;          // 0 pinhole, 1 equidistant, 2 Kannala-Brandt
    int width, height;
    double fx, fy, cx, cy;
    double k[4];
    double th_lim;      // the radial map is inverted on [0, th_lim] and saturates beyond
};

__host__ __device__ inline double cam_rd(const Cam& c, double th)
{
    if (c.model == 0) return tan(th);
    if (c.model == 1) return th;
    const double t2 = th * th;
    return th * (1.0 + t2 * (c.k[0] + t2 * (c.k[1] + t2 * (c.k[2] + t2 * c.k[3]))));
}

__host__ __device__ inline double cam_drd(const Cam& c, double th)
{
    if (c.model == 0) { const double cs = cos(th); return 1.0 / (cs * cs); }
    if (c.model == 1) return 1.0;
    const double t2 = th * th;
    return 1.0 + t2 * (3.0 * c.k[0] + t2 * (5.0 * c.k[1] + t2 * (7.0 * c.k[2] + t2 * 9.0 * c.k[3])));
}

// Inverse of the radial map: bracketed Newton on [0, th_lim].
__host__ __device__ inline double cam_theta(const Cam& c, double rd)
{
    if (!(rd > 0.0)) return 0.0;
    if (c.model == 0) return atan(rd);
    if (c.model == 1) return rd < c.th_lim ? rd : c.th_lim;
    if (rd >= cam_rd(c, c.th_lim)) return c.th_lim;
    double lo = 0.0, hi = c.th_lim, th = rd < c.th_lim ? rd : 0.5 * c.th_lim;
    for (int it = 0; it < 200; ++it) {
        const double f = cam_rd(c, th) - rd;
        if (f == 0.0) return th;
        if (f > 0.0) hi = th; else lo = th;
        double nt = th - f / cam_drd(c, th);
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        if (fabs(nt - th) < 1e-15) return nt;
        th = nt;
    }
    return th;
}

// pi^-1: pixel (px, py) -> unit ray.
__host__ __device__ inline void cam_ray(const Cam& c, double px, double py, double r[3])
{
    const double mx = (px - c.cx) / c.fx, my = (py - c.cy) / c.fy;
    if (c.model == 0) {
        const double n = sqrt(mx * mx + my * my + 1.0);
        r[0] = mx / n; r[1] = my / n; r[2] = 1.0 / n;
        return;
    }
    const double rd = sqrt(mx * mx + my * my);
    const double th = cam_theta(c, rd);
    if (rd > 0.0) {
        const double s = sin(th) / rd;
        r[0] = s * mx; r[1] = s * my; r[2] = cos(th);
    } else {
        r[0] = 0.0; r[1] = 0.0; r[2] = 1.0;
    }
}

// pi: point -> pixel; false if it has no image (pinhole, behind the camera).
__host__ __device__ inline bool cam_pixel(const Cam& c, const double X[3], double x[2])
{
    if (c.model == 0) {
        if (!(X[2] > 0.0)) return false;
        x[0] = c.cx + c.fx * X[0] / X[2];
        x[1] = c.cy + c.fy * X[1] / X[2];
        return true;
    }
    const double rho = sqrt(X[0] * X[0] + X[1] * X[1]);
    const double rd = cam_rd(c, atan2(rho, X[2]));
    if (rho > 0.0) {
        x[0] = c.cx + c.fx * rd * X[0] / rho;
        x[1] = c.cy + c.fy * rd * X[1] / rho;
    } else {
        x[0] = c.cx;
        x[1] = c.cy;
    }
    return true;
}

// Level-l camera of the pyramid (scale 1/2 per level, pixel centres).
__host__ __device__ inline Cam cam_level(const Cam& c, int l)
{
    Cam o = c;
    const double s = 1.0 / double(1 << l);
    o.fx = c.fx * s; o.fy = c.fy * s;
    o.cx = (c.cx + 0.5) * s - 0.5; o.cy = (c.cy + 0.5) * s - 0.5;
    o.width = c.width >> l; o.height = c.height >> l;
    return o;
}

// ----------------------------------------------------------------- rig geometry (device side)
struct RigGeom {
    Cam cam0, cam1;
    double R[9];        // X1 = R X0 + t
    double tdir[3];     // t' / |t'| with t' = R^T t
    double C[3];        // pre-rotated camera-1 centre, -t'
    double rmax0;       // radial limit of camera 0's mask, r_d(FOV0 / 2)
    double half1;       // FOV1 / 2 (radians)
    double cos_guard;   // cos of the epipole guard angle
    double eps;         // step along t' of the trajectory-field construction
};

// ----------------------------------------------------------------- compact storage
// The dual variables (p, q) and the tensor pack (t11, t12, t22, I_u) are
// stored as 32-bit floats (ST_F32), IEEE half (ST_F16) or bfloat16
// (ST_BF16); every update is computed in FP32.
enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

__device__ inline uint16_t f32_to_h(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ inline float h_to_f32(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
// bfloat16 by round-to-nearest-even of the upper half of the FP32 bits
__device__ inline uint16_t f32_to_bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <int S> __device__ inline uint16_t enc16(float x) { return S == ST_F16 ? f32_to_h(x) : f32_to_bf(x); }
template <int S> __device__ inline float dec16(uint16_t b) { return S == ST_F16 ? h_to_f32(b) : bf_to_f32(b); }

// The value a float takes once stored.
template <int S> __device__ inline float as_stored(float x)
{
    if constexpr (S == ST_F32) return x;
    else return dec16<S>(enc16<S>(x));
}

template <int S> __device__ inline float2 ld2(const void* base, size_t i)
{
    if constexpr (S == ST_F32) {
        return static_cast<const float2*>(base)[i];
    } else {
        const uint32_t v = static_cast<const uint32_t*>(base)[i];
        return make_float2(dec16<S>(uint16_t(v & 0xffffu)), dec16<S>(uint16_t(v >> 16)));
    }
}

template <int S> __device__ inline float4 ld4(const void* base, size_t i)
{
    if constexpr (S == ST_F32) {
        return static_cast<const float4*>(base)[i];
    } else {
        const uint2 v = static_cast<const uint2*>(base)[i];
        return make_float4(dec16<S>(uint16_t(v.x & 0xffffu)), dec16<S>(uint16_t(v.x >> 16)),
                           dec16<S>(uint16_t(v.y & 0xffffu)), dec16<S>(uint16_t(v.y >> 16)));
    }
}

template <int S> __device__ inline void st2(void* base, size_t i, float2 f)
{
    if constexpr (S == ST_F32) {
        static_cast<float2*>(base)[i] = f;
    } else {
        static_cast<uint32_t*>(base)[i] = uint32_t(enc16<S>(f.x)) | (uint32_t(enc16<S>(f.y)) << 16);
    }
}

template <int S> __device__ inline void st4(void* base, size_t i, float4 f)
{
    if constexpr (S == ST_F32) {
        static_cast<float4*>(base)[i] = f;
    } else {
        static_cast<uint2*>(base)[i] = make_uint2(uint32_t(enc16<S>(f.x)) | (uint32_t(enc16<S>(f.y)) << 16),
                                                  uint32_t(enc16<S>(f.z)) | (uint32_t(enc16<S>(f.w)) << 16));
    }
}

// ----------------------------------------------------------------- launchers
// Set-up (double precision).
void launch_calibration(const RigGeom& g, float2* calib, int pitch, hipStream_t s);
void launch_level_fields(const RigGeom& g, int level, float2* gamma, uint8_t* flags, int pitch,
                         hipStream_t s);

// Per-pair image steps (batched over pairs b < n with element strides).
struct PairPtrs {
    const float* in[kMaxBatch];
    int in_pitch;       // elements
};
void launch_prerotate(const PairPtrs& I1, int n, int W, int H, const float2* calib, int cpitch,
                      float* out, int opitch, long long ostride, hipStream_t s);
void launch_downsample(int n, int Wc, int Hc, const float* const* fine, int fpitch, long long fstride,
                       float* coarse, int cpitch, long long cstride, hipStream_t s);
void launch_tensor(int n, int W, int H, const float* const* J0, int jpitch, long long jstride,
                   const uint8_t* flags, int fpitch, const float* betas, const float* etas,
                   void* tpack, int tpitch, long long tstride, int storage, hipStream_t s);
void launch_linearise(int n, int W, int H, int pitch, long long stride, const float* const* J0,
                      int j0pitch, long long j0stride, const float* J1, long long j1stride,
                      const float2* gamma, const uint8_t* flags, float* u, float* u_w, float2* w,
                      float2* gamma_w, void* tpack, float* rho, int clip, int clip_only, float du_max,
                      int storage, hipStream_t s);
void launch_upsample(int n, int Wc, int Hc, int cpitch, long long cstride, const uint8_t* flags_c,
                     int fcpitch, const float* u_c, const float2* w_c, int fpitch, long long fstride,
                     float* u_f, float2* w_f, float2* v_f, void* p_f, void* q_f, int storage, hipStream_t s);
void launch_zero_state(int n, int W, int H, int pitch, long long stride, float* u, float2* w, float2* v,
                       void* p, void* q, int storage, hipStream_t s);
void launch_triangulate(int n, const RigGeom& g, int W, int H, int pitch, long long stride,
                        const float* u, const float2* w, const uint8_t* flags, int fpitch,
                        float* const* u_out, float* const* w_out, float* const* depth_out,
                        float* const* z_out, uint8_t* const* valid_out, int opitch, hipStream_t s);

// Primal-dual iteration (Eq. (11)).
enum PdMode { PD_DUAL_FIRST = 0, PD_FUSED = 1, PD_PRIMAL_LAST = 2, PD_FUSED2 = 3 };
struct PdArgs {
    int W, H, pitch;            // level size, element pitch of every plane
    long long stride;           // elements between pairs
    int n;                      // pairs
    const float* u_in; const float2* v_in; const void* p_in; const void* q_in;
    float* u_out; float2* v_out; void* p_out; void* q_out;
    const void* tpack;          // (t11, t12, t22, I_u)
    const float* rho;           // rho_c
    const uint8_t* flags;       // shared by all pairs (rig field)
    float alpha0, alpha1, lambda;
    float tau_scale, sigma_scale, theta;     // iteration k (PD_FUSED2: the first of its two)
    float tau_scale2, sigma_scale2, theta2;  // PD_FUSED2: iteration k + 1
    int mode;                   // PdMode
    int tgv;                    // 1: TGV-L1 (Eq. (10)); 0: TV-L1 (v = 0, no q)
    int storage;                // Storage of p, q and the tensor pack
};
void launch_pd(const PdArgs& a, hipStream_t s);

}  // namespace vfs
