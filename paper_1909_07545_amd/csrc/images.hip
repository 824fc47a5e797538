// Per-pair image steps, batched over the pairs of a solve: pre-rotation
// (Sec. IV-A), pyramid (Sec. IV-B), tensor (Eq. (12)), warping and
// linearisation with the clip of the previous warp (Eqs. (3), (5), (8)-(9),
// Sec. III-B, Algorithm 1), coarse-to-fine transfer (Sec. IV-B) and
// triangulation (Sec. III-D).
//
// Sample points are kept as an integer pixel plus a small float offset
// (the warp vector), so that sub-pixel fractions keep float precision at any
// image size.
#include "vfs_internal.h"

namespace vfs {

namespace {

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bilinear sample of I at (bx + dx, by + dy), taps clamped to the image.
__device__ inline float bilinear(const float* I, int pitch, int W, int H, int bx, int by, float dx, float dy)
{
    const float fx = floorf(dx), fy = floorf(dy);
    const float ax = dx - fx, ay = dy - fy;
    const int x0 = bx + int(fx), y0 = by + int(fy);
    const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    const int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    const float* ra = I + (size_t)ya * pitch;
    const float* rb = I + (size_t)yb * pitch;
    return (1.f - ax) * (1.f - ay) * ra[xa] + ax * (1.f - ay) * ra[xb] + (1.f - ax) * ay * rb[xa] + ax * ay * rb[xb];
}

// Keys cubic convolution weights (a = -1/2) at fraction t of the taps -1, 0, 1, 2.
__device__ inline void keys(float t, float w[4])
{
    const float t2 = t * t, t3 = t2 * t;
    w[0] = -0.5f * t3 + t2 - 0.5f * t;
    w[1] = 1.5f * t3 - 2.5f * t2 + 1.f;
    w[2] = -1.5f * t3 + 2.f * t2 + 0.5f * t;
    w[3] = 0.5f * t3 - 0.5f * t2;
}

// Bicubic sample of a float2 field at (bx + dx, by + dy), taps clamped.
__device__ inline float2 bicubic2(const float2* g, int pitch, int W, int H, int bx, int by, float dx, float dy)
{
    const float fx = floorf(dx), fy = floorf(dy);
    float wx[4], wy[4];
    keys(dx - fx, wx);
    keys(dy - fy, wy);
    const int x0 = bx + int(fx), y0 = by + int(fy);
    int xs[4];
    for (int a = 0; a < 4; ++a) xs[a] = clampi(x0 - 1 + a, 0, W - 1);
    float sx = 0.f, sy = 0.f;
    for (int b = 0; b < 4; ++b) {
        const float2* row = g + (size_t)clampi(y0 - 1 + b, 0, H - 1) * pitch;
        float rx = 0.f, ry = 0.f;
        for (int a = 0; a < 4; ++a) {
            const float2 v = row[xs[a]];
            rx += wx[a] * v.x;
            ry += wx[a] * v.y;
        }
        sx += wy[b] * rx;
        sy += wy[b] * ry;
    }
    return make_float2(sx, sy);
}

__global__ void prerotate_kernel(PairPtrs I1, int W, int H, const float2* calib, int cpitch, float* out,
                                 int opitch, long long ostride)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= W) return;
    const float2 c = calib[(size_t)i * cpitch + j];
    out[b * ostride + (size_t)i * opitch + j] = bilinear(I1.in[b], I1.in_pitch, W, H, j, i, c.x, c.y);
}

struct FinePtrs { const float* p[kMaxBatch]; };

__global__ void downsample_kernel(int Wc, int Hc, FinePtrs fine, int fpitch, long long fstride, float* coarse,
                                  int cpitch, long long cstride)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= Wc) return;
    const float* f = fine.p[b] + (fstride ? b * fstride : 0);
    const float* r0 = f + (size_t)(2 * i) * fpitch + 2 * j;
    const float* r1 = r0 + fpitch;
    coarse[b * cstride + (size_t)i * cpitch + j] = 0.25f * (r0[0] + r0[1] + r1[0] + r1[1]);
}

__device__ inline bool in_mask(const uint8_t* flags, int fpitch, int W, int H, int i, int j)
{
    return i >= 0 && i < H && j >= 0 && j < W && (flags[(size_t)i * fpitch + j] & F_MASK);
}

struct Params2 { float beta[kMaxBatch]; float eta[kMaxBatch]; };

template <int S>
__global__ void tensor_kernel(int W, int H, FinePtrs J0, int jpitch, long long jstride, const uint8_t* flags,
                              int fpitch, Params2 be, void* tpack, int tpitch, long long tstride)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= W) return;
    float4 t = make_float4(1.f, 0.f, 1.f, 0.f);
    if (in_mask(flags, fpitch, W, H, i, j)) {
        const float* J = J0.p[b] + (jstride ? b * jstride : 0);
        const float* r = J + (size_t)i * jpitch;
        const float c = r[j];
        float gx = 0.f, gy = 0.f;
        const bool l = in_mask(flags, fpitch, W, H, i, j - 1), rr = in_mask(flags, fpitch, W, H, i, j + 1);
        if (l && rr) gx = 0.5f * (r[j + 1] - r[j - 1]);
        else if (rr) gx = r[j + 1] - c;
        else if (l) gx = c - r[j - 1];
        const bool u = in_mask(flags, fpitch, W, H, i - 1, j), d = in_mask(flags, fpitch, W, H, i + 1, j);
        if (u && d) gy = 0.5f * (r[j + jpitch] - r[j - jpitch]);
        else if (d) gy = r[j + jpitch] - c;
        else if (u) gy = c - r[j - jpitch];
        const float g = sqrtf(gx * gx + gy * gy);
        if (!(g < 1e-12f)) {
            const float nx = gx / g, ny = gy / g;
            const float e = expf(-be.beta[b] * powf(g, be.eta[b]));
            t = make_float4(e * nx * nx + ny * ny, (e - 1.f) * nx * ny, e * ny * ny + nx * nx, 0.f);
        }
    }
    st4<S>(tpack, b * tstride + (size_t)i * tpitch + j, t);
}

template <int S>
__global__ void linearise_kernel(int W, int H, int pitch, long long stride, FinePtrs J0, int j0pitch,
                                 long long j0stride, const float* J1, long long j1stride, const float2* gamma,
                                 const uint8_t* flags, float* u, float* u_w, float2* w, float2* gamma_w,
                                 void* tpack, float* rho, int clip, int clip_only, float du_max)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= W) return;
    const size_t o = b * stride + (size_t)i * pitch + j;
    float uu = u[o];
    float2 ww = w[o];
    if (clip) {
        // Sec. III-C / Algorithm 1: clip the increment of the finished warp, accumulate
        float du = uu - u_w[o];
        du = fminf(fmaxf(du, -du_max), du_max);
        uu = u_w[o] + du;
        const float2 gw = gamma_w[o];
        ww.x += du * gw.x;
        ww.y += du * gw.y;
        u[o] = uu;
        w[o] = ww;
    }
    if (clip_only) return;
    u_w[o] = uu;
    // tangent at the warped point (bicubic sample of the trajectory field, renormalised)
    float2 g = bicubic2(gamma, pitch, W, H, j, i, ww.x, ww.y);
    const float n = sqrtf(g.x * g.x + g.y * g.y);
    if (n > 0.f) { g.x /= n; g.y /= n; } else { g.x = 0.f; g.y = 0.f; }
    gamma_w[o] = g;
    float Iu = 0.f, rc = 0.f;
    if (flags[(size_t)i * pitch + j] & F_DATA) {
        const float* J1b = J1 + b * j1stride;
        const float i1 = bilinear(J1b, pitch, W, H, j, i, ww.x, ww.y);
        const float i1s = bilinear(J1b, pitch, W, H, j, i, ww.x + g.x, ww.y + g.y);
        const float* J0b = J0.p[b] + (j0stride ? b * j0stride : 0);
        // rho_c is formed from I_u as stored, so that rho_c + u I_u is exact at u = u_w
        Iu = as_stored<S>(i1s - i1);
        rc = i1 - J0b[(size_t)i * j0pitch + j] - uu * Iu;
    }
    if constexpr (S == ST_F32) {
        static_cast<float4*>(tpack)[o].w = Iu;
    } else {
        float4 t = ld4<S>(tpack, o);
        t.w = Iu;
        st4<S>(tpack, o, t);
    }
    rho[o] = rc;
}

template <int S>
__global__ void upsample_kernel(int Wc, int Hc, int cpitch, long long cstride, const uint8_t* flags_c, int fcpitch,
                                const float* u_c, const float2* w_c, int fpitch, long long fstride, float* u_f,
                                float2* w_f, float2* v_f, void* p_f, void* q_f)
{
    const int Wf = 2 * Wc;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= Wf) return;
    const float x = 0.5f * j - 0.25f, y = 0.5f * i - 0.25f;
    const float fx0 = floorf(x), fy0 = floorf(y), ax = x - fx0, ay = y - fy0;
    const int x0 = int(fx0), y0 = int(fy0);
    float sw = 0.f, su = 0.f, s1 = 0.f, s2 = 0.f;
    for (int bb = 0; bb < 2; ++bb) {
        const int yy = clampi(y0 + bb, 0, Hc - 1);
        const float wy = bb ? ay : 1.f - ay;
        for (int aa = 0; aa < 2; ++aa) {
            const int xx = clampi(x0 + aa, 0, Wc - 1);
            if (!(flags_c[(size_t)yy * fcpitch + xx] & F_MASK)) continue;
            const float wt = (aa ? ax : 1.f - ax) * wy;
            const size_t co = b * cstride + (size_t)yy * cpitch + xx;
            sw += wt;
            su += wt * u_c[co];
            s1 += wt * w_c[co].x;
            s2 += wt * w_c[co].y;
        }
    }
    const size_t fo = b * fstride + (size_t)i * fpitch + j;
    if (sw > 0.f) {
        u_f[fo] = 2.f * su / sw;
        w_f[fo] = make_float2(2.f * s1 / sw, 2.f * s2 / sw);
    } else {
        u_f[fo] = 0.f;
        w_f[fo] = make_float2(0.f, 0.f);
    }
    if (v_f) v_f[fo] = make_float2(0.f, 0.f);
    if (p_f) st2<S>(p_f, fo, make_float2(0.f, 0.f));
    if (q_f) st4<S>(q_f, fo, make_float4(0.f, 0.f, 0.f, 0.f));
}

template <int S>
__global__ void zero_state_kernel(int W, int pitch, long long stride, float* u, float2* w, float2* v, void* p,
                                  void* q)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= W) return;
    const size_t o = b * stride + (size_t)i * pitch + j;
    u[o] = 0.f;
    w[o] = make_float2(0.f, 0.f);
    if (v) v[o] = make_float2(0.f, 0.f);
    st2<S>(p, o, make_float2(0.f, 0.f));
    if (q) st4<S>(q, o, make_float4(0.f, 0.f, 0.f, 0.f));
}

struct OutPtrs {
    float* u[kMaxBatch];
    float* w[kMaxBatch];
    float* depth[kMaxBatch];
    float* z[kMaxBatch];
    uint8_t* valid[kMaxBatch];
};

// Closest approach of the rays a = pi0^-1(x) from the origin and
// b = pi0^-1(x + w) from C = -t', in double precision.
__global__ void triangulate_kernel(RigGeom g, int W, int H, int pitch, long long stride, const float* u,
                                   const float2* w, const uint8_t* flags, int fpitch, OutPtrs out, int opitch)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (j >= W) return;
    const size_t o = b * stride + (size_t)i * pitch + j;
    const size_t oo = (size_t)i * opitch + j;
    const float2 ww = w[o];
    if (out.u[b]) out.u[b][oo] = u[o];
    if (out.w[b]) { out.w[b][2 * oo] = ww.x; out.w[b][2 * oo + 1] = ww.y; }
    double a[3], bb[3];
    cam_ray(g.cam0, j, i, a);
    cam_ray(g.cam0, double(j) + double(ww.x), double(i) + double(ww.y), bb);
    const double ab = a[0] * bb[0] + a[1] * bb[1] + a[2] * bb[2];
    const double aC = a[0] * g.C[0] + a[1] * g.C[1] + a[2] * g.C[2];
    const double bC = bb[0] * g.C[0] + bb[1] * g.C[1] + bb[2] * g.C[2];
    const double den = 1.0 - ab * ab;
    float depth = __builtin_inff(), z = __builtin_inff();
    uint8_t ok = 0;
    if (den > 1e-12 && (flags[(size_t)i * fpitch + j] & F_DATA)) {
        const double d0 = (aC - ab * bC) / den, d1 = (ab * aC - bC) / den;
        if (d0 > 0.0 && d1 > 0.0) {
            depth = float(d0);
            z = float(d0 * a[2]);
            ok = 1;
        }
    }
    if (out.depth[b]) out.depth[b][oo] = depth;
    if (out.z[b]) out.z[b][oo] = z;
    if (out.valid[b]) out.valid[b][oo] = ok;
}

inline dim3 grid_for(int W, int H, int n) { return dim3((W + 63) / 64, H, n); }

}  // namespace

void launch_prerotate(const PairPtrs& I1, int n, int W, int H, const float2* calib, int cpitch, float* out,
                      int opitch, long long ostride, hipStream_t s)
{
    hipLaunchKernelGGL(prerotate_kernel, grid_for(W, H, n), dim3(64), 0, s, I1, W, H, calib, cpitch, out, opitch,
                       ostride);
}

void launch_downsample(int n, int Wc, int Hc, const float* const* fine, int fpitch, long long fstride, float* coarse,
                       int cpitch, long long cstride, hipStream_t s)
{
    FinePtrs f;
    for (int b = 0; b < n; ++b) f.p[b] = fine[b];
    hipLaunchKernelGGL(downsample_kernel, grid_for(Wc, Hc, n), dim3(64), 0, s, Wc, Hc, f, fpitch, fstride, coarse,
                       cpitch, cstride);
}

#define VFS_BY_STORAGE(storage, call)                   \
    do {                                                \
        if ((storage) == ST_F16) { constexpr int S = ST_F16; call; }         \
        else if ((storage) == ST_BF16) { constexpr int S = ST_BF16; call; }  \
        else { constexpr int S = ST_F32; call; }                             \
    } while (0)

void launch_tensor(int n, int W, int H, const float* const* J0, int jpitch, long long jstride, const uint8_t* flags,
                   int fpitch, const float* betas, const float* etas, void* tpack, int tpitch, long long tstride,
                   int storage, hipStream_t s)
{
    FinePtrs f;
    Params2 be;
    for (int b = 0; b < n; ++b) {
        f.p[b] = J0[b];
        be.beta[b] = betas[b];
        be.eta[b] = etas[b];
    }
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(tensor_kernel<S>, grid_for(W, H, n), dim3(64), 0, s, W, H, f, jpitch,
                                               jstride, flags, fpitch, be, tpack, tpitch, tstride));
}

void launch_linearise(int n, int W, int H, int pitch, long long stride, const float* const* J0, int j0pitch,
                      long long j0stride, const float* J1, long long j1stride, const float2* gamma,
                      const uint8_t* flags, float* u, float* u_w, float2* w, float2* gamma_w, void* tpack,
                      float* rho, int clip, int clip_only, float du_max, int storage, hipStream_t s)
{
    FinePtrs f;
    for (int b = 0; b < n; ++b) f.p[b] = J0[b];
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(linearise_kernel<S>, grid_for(W, H, n), dim3(64), 0, s, W, H, pitch,
                                               stride, f, j0pitch, j0stride, J1, j1stride, gamma, flags, u, u_w, w,
                                               gamma_w, tpack, rho, clip, clip_only, du_max));
}

void launch_upsample(int n, int Wc, int Hc, int cpitch, long long cstride, const uint8_t* flags_c, int fcpitch,
                     const float* u_c, const float2* w_c, int fpitch, long long fstride, float* u_f, float2* w_f,
                     float2* v_f, void* p_f, void* q_f, int storage, hipStream_t s)
{
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(upsample_kernel<S>, grid_for(2 * Wc, 2 * Hc, n), dim3(64), 0, s, Wc,
                                               Hc, cpitch, cstride, flags_c, fcpitch, u_c, w_c, fpitch, fstride, u_f,
                                               w_f, v_f, p_f, q_f));
}

void launch_zero_state(int n, int W, int H, int pitch, long long stride, float* u, float2* w, float2* v, void* p,
                       void* q, int storage, hipStream_t s)
{
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(zero_state_kernel<S>, grid_for(W, H, n), dim3(64), 0, s, W, pitch,
                                               stride, u, w, v, p, q));
}

void launch_triangulate(int n, const RigGeom& g, int W, int H, int pitch, long long stride, const float* u,
                        const float2* w, const uint8_t* flags, int fpitch, float* const* u_out, float* const* w_out,
                        float* const* depth_out, float* const* z_out, uint8_t* const* valid_out, int opitch,
                        hipStream_t s)
{
    OutPtrs o;
    for (int b = 0; b < n; ++b) {
        o.u[b] = u_out ? u_out[b] : nullptr;
        o.w[b] = w_out ? w_out[b] : nullptr;
        o.depth[b] = depth_out ? depth_out[b] : nullptr;
        o.z[b] = z_out ? z_out[b] : nullptr;
        o.valid[b] = valid_out ? valid_out[b] : nullptr;
    }
    hipLaunchKernelGGL(triangulate_kernel, grid_for(W, H, n), dim3(64), 0, s, g, W, H, pitch, stride, u, w, flags,
                       fpitch, o, opitch);
}

}  // namespace vfs
