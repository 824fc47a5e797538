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
// Widest image row in pixels: the primal-dual kernels address a row through a
// buffer resource with 32-bit byte offsets and record counts (16 bytes per
// pixel at most).
constexpr int kMaxWidth = 1 << 20;

// ----------------------------------------------------------------- camera
// Radially symmetric models: a ray at angle theta from the axis lands at
// normalised radius r_d(theta).
//   Kannala-Brandt: r_d = theta + k1 theta^3 + k2 theta^5 + k3 theta^7 +
//     k4 theta^9 (equidistant is k = 0; pinhole r_d = tan(theta)).
//   Unified (xi = k[0]): projection from the centre of a unit sphere moved
//     by xi along the axis, r_d = sin / (xi + cos).
//   Enhanced unified (alpha = k[0], beta = k[1]):
//     r_d = sin / (alpha sqrt(beta sin^2 + cos^2) + (1 - alpha) cos).
// The unified models invert in closed form; Kannala-Brandt by Newton.
struct Cam {
    int model;          // 0 pinhole, 1 equidistant, 2 Kannala-Brandt, 3 unified, 4 enhanced unified
    int width, height;
    double fx, fy, cx, cy;
    double k[4];
    double th_lim;      // the radial map is inverted on [0, th_lim] and saturates beyond
};

// Denominator of the unified models' radial map.
__host__ __device__ inline double cam_uden(const Cam& c, double th)
{
    const double s = sin(th), co = cos(th);
    if (c.model == 3) return c.k[0] + co;
    return c.k[0] * sqrt(c.k[1] * s * s + co * co) + (1.0 - c.k[0]) * co;
}

__host__ __device__ inline double cam_rd(const Cam& c, double th)
{
    if (c.model == 0) return tan(th);
    if (c.model == 1) return th;
    if (c.model >= 3) return sin(th) / cam_uden(c, th);
    const double t2 = th * th;
    return th * (1.0 + t2 * (c.k[0] + t2 * (c.k[1] + t2 * (c.k[2] + t2 * c.k[3]))));
}

__host__ __device__ inline double cam_drd(const Cam& c, double th)
{
    if (c.model == 0) { const double cs = cos(th); return 1.0 / (cs * cs); }
    if (c.model == 1) return 1.0;
    if (c.model >= 3) {
        const double s = sin(th), co = cos(th), D = cam_uden(c, th);
        double dD = -s;
        if (c.model == 4) {
            const double g = sqrt(c.k[1] * s * s + co * co);
            dD = c.k[0] * (c.k[1] - 1.0) * s * co / g - (1.0 - c.k[0]) * s;
        }
        return (co * D - s * dD) / (D * D);
    }
    const double t2 = th * th;
    return 1.0 + t2 * (3.0 * c.k[0] + t2 * (5.0 * c.k[1] + t2 * (7.0 * c.k[2] + t2 * 9.0 * c.k[3])));
}

// Inverse of the radial map: closed form for the unified models (the angle
// of their back-projected ray), bracketed Newton on [0, th_lim] otherwise.
__host__ __device__ inline double cam_theta(const Cam& c, double rd)
{
    if (!(rd > 0.0)) return 0.0;
    if (c.model == 0) return atan(rd);
    if (c.model == 1) return rd < c.th_lim ? rd : c.th_lim;
    if (rd >= cam_rd(c, c.th_lim)) return c.th_lim;
    if (c.model == 3) {
        // back-projected ray (lambda m, lambda - xi), lambda = (xi + sqrt(1 + (1 - xi^2) r^2)) / (1 + r^2)
        const double xi = c.k[0], r2 = rd * rd;
        const double disc = 1.0 + (1.0 - xi * xi) * r2;
        const double lam = (xi + sqrt(disc > 0.0 ? disc : 0.0)) / (1.0 + r2);
        return atan2(lam * rd, lam - xi);
    }
    if (c.model == 4) {
        // back-projected ray (m, m_z), m_z = (1 - beta alpha^2 r^2) / (alpha sqrt(1 - (2 alpha - 1) beta r^2) + 1 - alpha)
        const double a = c.k[0], b = c.k[1], r2 = rd * rd;
        const double disc = 1.0 - (2.0 * a - 1.0) * b * r2;
        const double mz = (1.0 - b * a * a * r2) / (a * sqrt(disc > 0.0 ? disc : 0.0) + 1.0 - a);
        return atan2(rd, mz);
    }
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
// Radial table of camera 0 for the per-pair back-projection in single
// precision: entry k holds r_d(theta_k) and dtheta r_d'(theta_k) at theta_k =
// k dtheta, dtheta = th_lim / kRadial, computed in double precision once per
// rig; the inverse of r_d is the cubic Hermite interpolant of these values
// inverted by Newton steps.
constexpr int kRadial = 4096;

// Camera 0 and the baseline in single precision, for the triangulation.
struct TriGeom {
    int model;
    float fx, fy, cx, cy;
    float th_lim, dtheta;
    float C[3];                 // -t'
    const float2* radial;       // kRadial + 1 entries (device; not used by pinhole / equidistant)
};

struct RigGeom {
    Cam cam0, cam1;
    double R[9];        // X1 = R X0 + t
    double tdir[3];     // t' / |t'| with t' = R^T t
    double C[3];        // pre-rotated camera-1 centre, -t'
    double rmax0;       // radial limit of camera 0's mask, r_d(FOV0 / 2)
    double half1;       // FOV1 / 2 (radians)
    double cos_guard;   // cos of the epipole guard angle
    double eps;         // step along t' of the trajectory-field construction
    TriGeom tri;
};

// A camera and a virtual pinhole view rotated against it (X_v = Rv X_cam).
struct RectifyGeom {
    Cam cam;            // the real camera (any model)
    Cam pin;            // the virtual view (pinhole model)
    double Rv[9];       // row-major
    double rmax;        // radial limit of the camera's mask, r_d(FOV / 2)
    double half;        // FOV / 2 (radians)
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

// ----------------------------------------------------------------- per-pair descriptors
// Sizes of the pyramid levels and the element offset of each level inside a
// level-stacked plane (levels stored one after the other, each with its own
// pitch, a multiple of 64 elements).
struct Geometry {
    int L;
    int W[kMaxLevels], H[kMaxLevels], pitch[kMaxLevels];
    long long off[kMaxLevels];
};

// One pair's descriptor, read by every batched kernel from device memory.
// Level-stacked arrays hold every level (level l at off[l]); single-level
// arrays hold the level in use with that level's pitch.  Element sizes of p,
// q and tpack follow the storage mode (FP32: 8, 16, 16 bytes; 16-bit: 4, 8, 8).
struct Slot {
    const float* I0;            // level-0 images (caller memory), pitch in_pitch
    const float* I1;
    int in_pitch;
    int out_pitch;
    float* u_out;               // outputs (caller memory, may be NULL), pitch out_pitch
    float* w_out;               // interleaved (x, y)
    float* depth_out;
    float* z_out;
    uint8_t* valid_out;
    const float2* gamma[kMaxLevels];    // rig fields of every level (level pitch)
    const uint8_t* flags[kMaxLevels];
    const float2* calib;        // level-0 pre-rotation map
    const RigGeom* geom;
    float* J0;                  // level-stacked pyramids (J0 level 0: copy of I0)
    float* J1;
    float* u[2];                // level-stacked state, double-buffered
    float2* v[2];
    void* p[2];
    void* q[2];
    float2* w;                  // level-stacked, single
    float* uw;                  // single-level
    float2* gw;
    void* tpack;
    float* rho;
    float* R0;                  // single-level data-term images of the level (rank transform
    float* R1;                  // or gradient magnitude; brightness data term: NULL)
    float beta, eta;
};

// Per-tick control of one pair of a serving tick (written between graph
// replays; entry z of a tick's launches covers slot `slot` of the bucket).
// ops: the stages of the tick the slot takes part in; level: the level of
// the tick's warp step; warp: its index in the level; flip: parity of the
// slot's double-buffered state relative to the launch's (bit 0 u/v, bit 1
// p/q).
enum : uint8_t {
    OP_START = 1u,      // pre-rotation, pyramids, zero state at the coarsest level
    OP_NEWLEVEL = 2u,   // close level+1 (final accumulate) and transfer to level
    OP_TENSOR = 4u,     // tensor of level
    OP_WARP = 8u,       // linearise + K primal-dual iterations at level
    OP_FINISH = 16u,    // final accumulate at level 0 and triangulation
    OP_ALL = 0xffu,
};
struct Ctrl {
    int8_t level;
    uint8_t ops;
    uint8_t flip;
    uint8_t slot;
    int32_t warp;
};

// Which pairs a launch covers and at which level.  tick = 0: pairs 0..n-1, all
// at level lev, parity (iu, ip).  tick = 1 (serving): entry z covers slot
// ctrl[z].slot, which takes part if ctrl[z].ops & op, at level lev if lev >= 0
// else ctrl[z].level + dl, with parity (iu, ip) ^ ctrl[z].flip.  The grid
// covers the level-gl size.
struct Launch {
    const Slot* slots;
    const Ctrl* ctrl;
    int n;
    int tick;
    int lev, dl;
    int gl;
    unsigned op;
    int iu, ip;
    Geometry g;
};

struct Pick {
    int l;
    unsigned flip;
    int warp;
    int slot;       // the pair's descriptor: lc.slots[slot]
};

__device__ inline bool pick(const Launch& lc, int z, Pick& pk)
{
    if (z >= lc.n) return false;
    if (!lc.tick) {
        pk.l = lc.lev;
        pk.flip = 0u;
        pk.warp = -1;
        pk.slot = z;
        return true;
    }
    const Ctrl c = lc.ctrl[z];
    if (!(c.ops & lc.op)) return false;
    pk.l = lc.lev >= 0 ? lc.lev : c.level + lc.dl;
    pk.flip = c.flip;
    pk.warp = c.warp;
    pk.slot = c.slot;
    return pk.l >= 0 && pk.l < lc.g.L;
}

// ----------------------------------------------------------------- launchers
// Set-up (double precision).
void launch_calibration(const RigGeom& g, float2* calib, int pitch, hipStream_t s);
void launch_level_fields(const RigGeom& g, int level, float2* gamma, uint8_t* flags, int pitch,
                         hipStream_t s);

// Descriptor writes (stream-ordered, graph-safe: kernels, not memsets).
void launch_write_slot(const Slot& sl, Slot* dst, hipStream_t s);
struct CtrlBlock { Ctrl c[kMaxBatch]; };
void launch_write_ctrl(const CtrlBlock& cb, int n, Ctrl* dst, hipStream_t s);

// Batched image steps; every launch takes a Launch (which pairs, which level).
void launch_prerotate(const Launch& lc, hipStream_t s);                      // J1[0], J0[0] of level 0
void launch_downsample(const Launch& lc, hipStream_t s);                     // J0, J1 level lev from lev - 1
void launch_tensor(const Launch& lc, int storage, hipStream_t s);
void launch_linearise(const Launch& lc, int clip, int clip_only, float du_max, int xform, int storage,
                      hipStream_t s);
// Rank transform (radius 2) of the level's J0, J1 into R0, R1.
constexpr int kRankRadius = 2;
void launch_transform(const Launch& lc, int kind, hipStream_t s);   // kind: vfs_data_term (1, 2)
void launch_upsample(const Launch& lc, int tgv, int storage, hipStream_t s);  // level + 1 -> level
void launch_zero_state(const Launch& lc, int tgv, int storage, hipStream_t s);
void launch_triangulate(const Launch& lc, hipStream_t s);                    // level 0
void launch_rectify(const RectifyGeom& g, const float* src, size_t src_pitch, float* dst, size_t dst_pitch,
                    uint8_t* valid, hipStream_t s);
void launch_unrectify(const RectifyGeom& g, const float* field, const uint8_t* field_valid, size_t field_pitch,
                      float* dst, size_t dst_pitch, uint8_t* valid, hipStream_t s);

// Primal-dual iteration (Eq. (11)).
// PD_FIRST2 / 3 / 4: a pass of N = 2, 3, 4 iterations whose first iteration is
// the dual half alone (PD_DUAL_FIRST followed by N - 1 iterations).
enum PdMode {
    PD_DUAL_FIRST = 0, PD_FUSED = 1, PD_PRIMAL_LAST = 2, PD_FUSED2 = 3, PD_FUSED3 = 4, PD_FUSED4 = 5, PD_FIRST3 = 6,
    PD_FIRST4 = 7, PD_FIRST2 = 8
};
struct PdArgs {
    Launch lc;                  // parity (lc.iu, lc.ip): the state read; the other copy is written
    float alpha0, alpha1, lambda;
    float tau_scale, sigma_scale, theta;     // PD_DUAL_FIRST, PD_FUSED, PD_PRIMAL_LAST: iteration k
    float tau_n[4], sigma_n[4], theta_n[4];  // PD_FUSED2 / 3 / 4, PD_FIRST2 / 3 / 4: iterations k .. k + N - 1
    int mode;                   // PdMode
    int tgv;                    // 1: TGV-L1 (Eq. (10)); 0: TV-L1 (v = 0, no q)
    int storage;                // Storage of p, q and the tensor pack
    int pass;                   // iterations per pass of the multi-iteration launches (2, 3, 4)
    int nt_stores;              // set per launch: the multi-iteration pass writes its state non-temporally
};
void launch_pd(const PdArgs& a, hipStream_t s);
// Queries the occupancy the primal-dual launches are sized by, for the
// current device (once; call before a graph capture of primal-dual work).
void prepare_pd();

// Linearised energy of Eq. (10) per pair of a launch (fixed-order FP64
// reduction): partial needs energy_partials(lc) doubles, out lc.n doubles.
struct EnergyConsts {
    float lambda, alpha0, alpha1;
    int tgv, storage;
};
size_t energy_partials(const Launch& lc);
void launch_energy(const Launch& lc, const EnergyConsts& k, double* partial, double* out, hipStream_t s);
// Sum, max and count of |a - b| over the mask bit of `mask` (all pixels if
// NULL): partial needs 3 * diff_partials(W, H) doubles, out3 3 doubles.
size_t diff_partials(int W, int H);
void launch_diff_stats(int W, int H, int pitch, const float* a, const float* b, const uint8_t* mask,
                       double* partial, double* out3, hipStream_t s);

}  // namespace vfs
