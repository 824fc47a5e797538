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

__device__ inline bool in_mask(const uint8_t* flags, int fpitch, int W, int H, int i, int j)
{
    return i >= 0 && i < H && j >= 0 && j < W && (flags[(size_t)i * fpitch + j] & F_MASK);
}

// Pixel (j, i) of pair z handled by this thread at the pair's level pk.l;
// false if the pair is not in the launch or the pixel lies outside its level.
__device__ inline bool pixel_of(const Launch& lc, Pick& pk, int& j, int& i)
{
    if (!pick(lc, blockIdx.z, pk)) return false;
    j = blockIdx.x * blockDim.x + threadIdx.x;
    i = blockIdx.y;
    return j < lc.g.W[pk.l] && i < lc.g.H[pk.l];
}

__device__ inline int par_u(const Launch& lc, const Pick& pk) { return (lc.iu ^ int(pk.flip)) & 1; }
__device__ inline int par_p(const Launch& lc, const Pick& pk) { return (lc.ip ^ int(pk.flip >> 1)) & 1; }

// Level 0 of both pyramids: J1 = I1 pre-rotated (Sec. IV-A), J0 = I0.
__global__ void prerotate_kernel(Launch lc)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int W = lc.g.W[0], H = lc.g.H[0], pitch = lc.g.pitch[0];
    const size_t o = (size_t)i * pitch + j;
    const float2 c = sl.calib[o];
    sl.J1[o] = bilinear(sl.I1, sl.in_pitch, W, H, j, i, c.x, c.y);
    sl.J0[o] = sl.I0[(size_t)i * sl.in_pitch + j];
}

// Level l of both pyramids from level l - 1 (2x2 box filter).
__global__ void downsample_kernel(Launch lc)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int l = pk.l;
    const int fp = lc.g.pitch[l - 1];
    const size_t fo = lc.g.off[l - 1] + (size_t)(2 * i) * fp + 2 * j;
    const size_t co = lc.g.off[l] + (size_t)i * lc.g.pitch[l] + j;
    const float* a = sl.J0 + fo;
    const float* b = sl.J1 + fo;
    sl.J0[co] = 0.25f * (a[0] + a[1] + a[fp] + a[fp + 1]);
    sl.J1[co] = 0.25f * (b[0] + b[1] + b[fp] + b[fp + 1]);
}

template <int S>
__global__ void tensor_kernel(Launch lc)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int l = pk.l, W = lc.g.W[l], H = lc.g.H[l], pitch = lc.g.pitch[l];
    const uint8_t* flags = sl.flags[l];
    float4 t = make_float4(1.f, 0.f, 1.f, 0.f);
    if (in_mask(flags, pitch, W, H, i, j)) {
        const float* r = sl.J0 + lc.g.off[l] + (size_t)i * pitch;
        const float c = r[j];
        float gx = 0.f, gy = 0.f;
        const bool lf = in_mask(flags, pitch, W, H, i, j - 1), rt = in_mask(flags, pitch, W, H, i, j + 1);
        if (lf && rt) gx = 0.5f * (r[j + 1] - r[j - 1]);
        else if (rt) gx = r[j + 1] - c;
        else if (lf) gx = c - r[j - 1];
        const bool up = in_mask(flags, pitch, W, H, i - 1, j), dn = in_mask(flags, pitch, W, H, i + 1, j);
        if (up && dn) gy = 0.5f * (r[j + pitch] - r[j - pitch]);
        else if (dn) gy = r[j + pitch] - c;
        else if (up) gy = c - r[j - pitch];
        const float g = sqrtf(gx * gx + gy * gy);
        if (!(g < 1e-12f)) {
            const float nx = gx / g, ny = gy / g;
            const float e = expf(-sl.beta * powf(g, sl.eta));
            t = make_float4(e * nx * nx + ny * ny, (e - 1.f) * nx * ny, e * ny * ny + nx * nx, 0.f);
        }
    }
    st4<S>(sl.tpack, (size_t)i * pitch + j, t);
}

// clip < 0: clip when the slot's warp index is > 0 (serving ticks).  rank:
// the data term compares the level's rank transforms R0, R1 instead of the
// images themselves (the tensor keeps the intensities).
template <int S>
__global__ void linearise_kernel(Launch lc, int clip, int clip_only, float du_max, int xform)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int l = pk.l, W = lc.g.W[l], H = lc.g.H[l], pitch = lc.g.pitch[l];
    const long long off = lc.g.off[l];
    const size_t o = (size_t)i * pitch + j;       // single-level planes
    const size_t os = off + o;                    // level-stacked planes
    float* u = sl.u[par_u(lc, pk)];
    const bool do_clip = clip < 0 ? pk.warp > 0 : clip != 0;
    float uu = u[os];
    float2 ww = sl.w[os];
    if (do_clip) {
        // Sec. III-C / Algorithm 1: clip the increment of the finished warp, accumulate
        float du = uu - sl.uw[o];
        du = fminf(fmaxf(du, -du_max), du_max);
        uu = sl.uw[o] + du;
        const float2 gw = sl.gw[o];
        ww.x += du * gw.x;
        ww.y += du * gw.y;
        u[os] = uu;
        sl.w[os] = ww;
    }
    if (clip_only) return;
    sl.uw[o] = uu;
    // Tangent at the warped point: the bicubic sample of the trajectory field
    // over max(|sample|, 1/2).  Samples shorter than 1/2 only occur where the
    // taps reach an epipole (the field turns through every direction around
    // it); scaling them by 2 instead of to unit length keeps gamma_w a
    // continuous function of the warped point there.
    float2 g = bicubic2(sl.gamma[l], pitch, W, H, j, i, ww.x, ww.y);
    const float n = fmaxf(sqrtf(g.x * g.x + g.y * g.y), 0.5f);
    g.x /= n;
    g.y /= n;
    sl.gw[o] = g;
    float Iu = 0.f, rc = 0.f;
    if (sl.flags[l][o] & F_DATA) {
        const float* J1 = xform ? sl.R1 : sl.J1 + off;
        const float i0 = xform ? sl.R0[o] : sl.J0[os];
        const float i1 = bilinear(J1, pitch, W, H, j, i, ww.x, ww.y);
        const float i1s = bilinear(J1, pitch, W, H, j, i, ww.x + g.x, ww.y + g.y);
        // rho_c is formed from I_u as stored, so that rho_c + u I_u is exact at u = u_w
        Iu = as_stored<S>(i1s - i1);
        rc = i1 - i0 - uu * Iu;
    }
    if constexpr (S == ST_F32) {
        static_cast<float4*>(sl.tpack)[o].w = Iu;
    } else {
        float4 t = ld4<S>(sl.tpack, o);
        t.w = Iu;
        st4<S>(sl.tpack, o, t);
    }
    sl.rho[o] = rc;
}

// The data term's images of a level (into R0, R1):
//  KIND 1, rank transform (a census variant): the share of the 5x5 neighbours
//    strictly darker than the pixel; counts are exact, so the result is that
//    of any correct implementation on the same float inputs;
//  KIND 2, gradient magnitude: sqrt(Ix^2 + Iy^2), central differences
//    (I(x+1) - I(x-1)) / 2.
// Neighbours outside the level are taken at the nearest edge pixel.
template <int KIND>
__global__ void transform_kernel(Launch lc)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int l = pk.l, W = lc.g.W[l], H = lc.g.H[l], pitch = lc.g.pitch[l];
    const long long off = lc.g.off[l];
    const float* img[2] = {sl.J0 + off, sl.J1 + off};
    float* out[2] = {sl.R0, sl.R1};
    for (int k = 0; k < 2; ++k) {
        const float* I = img[k];
        if constexpr (KIND == 1) {
            constexpr int r = kRankRadius;
            constexpr float norm = 1.f / float((2 * r + 1) * (2 * r + 1) - 1);
            const float c = I[(size_t)i * pitch + j];
            int count = 0;
            for (int di = -r; di <= r; ++di) {
                const float* row = I + (size_t)clampi(i + di, 0, H - 1) * pitch;
                for (int dj = -r; dj <= r; ++dj)
                    if (di || dj) count += row[clampi(j + dj, 0, W - 1)] < c;
            }
            out[k][(size_t)i * pitch + j] = float(count) * norm;
        } else {
            const float* row = I + (size_t)i * pitch;
            const float gx = 0.5f * (row[clampi(j + 1, 0, W - 1)] - row[clampi(j - 1, 0, W - 1)]);
            const float gy = 0.5f * (I[(size_t)clampi(i + 1, 0, H - 1) * pitch + j] -
                                     I[(size_t)clampi(i - 1, 0, H - 1) * pitch + j]);
            out[k][(size_t)i * pitch + j] = sqrtf(gx * gx + gy * gy);
        }
    }
}

// Level l + 1 -> level l (Sec. IV-B): u doubled, w doubled (bilinear over the
// coarse mask); v, p, q restart at zero.  Same parity in and out.
template <int S>
__global__ void upsample_kernel(Launch lc, int tgv)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int l = pk.l, lc1 = l + 1;
    const int Wc = lc.g.W[lc1], Hc = lc.g.H[lc1], cp = lc.g.pitch[lc1];
    const uint8_t* flags_c = sl.flags[lc1];
    const int pu = par_u(lc, pk), pp = par_p(lc, pk);
    const float* u_c = sl.u[pu] + lc.g.off[lc1];
    const float2* w_c = sl.w + lc.g.off[lc1];
    const float x = 0.5f * j - 0.25f, y = 0.5f * i - 0.25f;
    const float fx0 = floorf(x), fy0 = floorf(y), ax = x - fx0, ay = y - fy0;
    const int x0 = int(fx0), y0 = int(fy0);
    float sw = 0.f, su = 0.f, s1 = 0.f, s2 = 0.f;
    for (int bb = 0; bb < 2; ++bb) {
        const int yy = clampi(y0 + bb, 0, Hc - 1);
        const float wy = bb ? ay : 1.f - ay;
        for (int aa = 0; aa < 2; ++aa) {
            const int xx = clampi(x0 + aa, 0, Wc - 1);
            const size_t co = (size_t)yy * cp + xx;
            if (!(flags_c[co] & F_MASK)) continue;
            const float wt = (aa ? ax : 1.f - ax) * wy;
            sw += wt;
            su += wt * u_c[co];
            s1 += wt * w_c[co].x;
            s2 += wt * w_c[co].y;
        }
    }
    const size_t fo = lc.g.off[l] + (size_t)i * lc.g.pitch[l] + j;
    if (sw > 0.f) {
        sl.u[pu][fo] = 2.f * su / sw;
        sl.w[fo] = make_float2(2.f * s1 / sw, 2.f * s2 / sw);
    } else {
        sl.u[pu][fo] = 0.f;
        sl.w[fo] = make_float2(0.f, 0.f);
    }
    if (sl.p[pp]) st2<S>(sl.p[pp], fo, make_float2(0.f, 0.f));
    if (tgv) {
        sl.v[pu][fo] = make_float2(0.f, 0.f);
        st4<S>(sl.q[pp], fo, make_float4(0.f, 0.f, 0.f, 0.f));
    }
}

template <int S>
__global__ void zero_state_kernel(Launch lc, int tgv)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const int pu = par_u(lc, pk), pp = par_p(lc, pk);
    const size_t o = lc.g.off[pk.l] + (size_t)i * lc.g.pitch[pk.l] + j;
    sl.u[pu][o] = 0.f;
    sl.w[o] = make_float2(0.f, 0.f);
    st2<S>(sl.p[pp], o, make_float2(0.f, 0.f));
    if (tgv) {
        sl.v[pu][o] = make_float2(0.f, 0.f);
        st4<S>(sl.q[pp], o, make_float4(0.f, 0.f, 0.f, 0.f));
    }
}

// Polar angle of a ray of camera 0 at normalised radius rd (single
// precision): equidistant in closed form, the other radially symmetric
// models from the rig's radial table -- the interval of rd by bisection,
// then two Newton steps on the cubic Hermite interpolant of r_d there --
// saturating at the model's limit like the set-up's inverse.
__device__ inline float theta32(const TriGeom& t, float rd)
{
    if (t.model == 1) return fminf(rd, t.th_lim);
    const float2* R = t.radial;
    if (!(rd > 0.f)) return 0.f;
    if (rd >= R[kRadial].x) return t.th_lim;
    int lo = 0, hi = kRadial;             // R[lo].x <= rd < R[hi].x
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (R[mid].x <= rd) lo = mid;
        else hi = mid;
    }
    // the interpolant as r_d = a.x + s (m + s (c2 + s c3)), s in [0, 1]: the
    // residual is formed from the small differences rd - a.x and b.x - a.x
    // (exact in float), not from values of the size of r_d
    const float2 a = R[lo], b = R[hi];
    const float dr = b.x - a.x, e = rd - a.x;
    const float c2 = 3.f * dr - 2.f * a.y - b.y, c3 = a.y + b.y - 2.f * dr;
    float s = e / dr;
    for (int it = 0; it < 2; ++it) {
        const float h = s * (a.y + s * (c2 + s * c3)) - e;
        const float dh = a.y + s * (2.f * c2 + 3.f * s * c3);
        s = fminf(fmaxf(s - h / dh, 0.f), 1.f);
    }
    return (float(lo) + s) * t.dtheta;
}

// Unit ray of camera 0 at normalised coordinates (mx, my) = (x - c) / f.
__device__ inline float3 ray32(const TriGeom& t, float mx, float my)
{
    if (t.model == 0) {
        const float n = rsqrtf(mx * mx + my * my + 1.f);
        return make_float3(mx * n, my * n, n);
    }
    const float rd = sqrtf(mx * mx + my * my);
    if (!(rd > 0.f)) return make_float3(0.f, 0.f, 1.f);
    float sn, cs;
    sincosf(theta32(t, rd), &sn, &cs);
    const float k = sn / rd;
    return make_float3(k * mx, k * my, cs);
}

__device__ inline float3 cross3(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Closest approach of the rays a = pi0^-1(x) from the origin and
// b = pi0^-1(x + w) from C = -t' (level 0), in single precision: with
// n = a x b, the ranges along a and b are d0 = ((C x b) . n) / |n|^2 and
// d1 = ((C x a) . n) / |n|^2 (the cross products avoid the cancellation of
// 1 - (a . b)^2 for nearly parallel rays).
__global__ void triangulate_kernel(Launch lc)
{
    Pick pk;
    int j, i;
    if (!pixel_of(lc, pk, j, i)) return;
    const Slot& sl = lc.slots[pk.slot];
    const TriGeom& g = sl.geom->tri;
    const size_t o = (size_t)i * lc.g.pitch[0] + j;
    const size_t oo = (size_t)i * sl.out_pitch + j;
    const float2 ww = sl.w[o];
    if (sl.u_out) sl.u_out[oo] = sl.u[par_u(lc, pk)][o];
    if (sl.w_out) { sl.w_out[2 * oo] = ww.x; sl.w_out[2 * oo + 1] = ww.y; }
    const float px = float(j) - g.cx, py = float(i) - g.cy;
    const float3 a = ray32(g, px / g.fx, py / g.fy);
    const float3 b = ray32(g, (px + ww.x) / g.fx, (py + ww.y) / g.fy);
    const float3 C = make_float3(g.C[0], g.C[1], g.C[2]);
    const float3 n = cross3(a, b);
    const float den = dot3(n, n);
    float depth = __builtin_inff(), z = __builtin_inff();
    uint8_t ok = 0;
    if (den > 1e-12f && (sl.flags[0][o] & F_DATA)) {
        const float d0 = dot3(cross3(C, b), n) / den, d1 = dot3(cross3(C, a), n) / den;
        if (d0 > 0.f && d1 > 0.f) {
            depth = d0;
            z = d0 * a.z;
            ok = 1;
        }
    }
    if (sl.depth_out) sl.depth_out[oo] = depth;
    if (sl.z_out) sl.z_out[oo] = z;
    if (sl.valid_out) sl.valid_out[oo] = ok;
}

// Descriptor writes: one thread, every store a vector-memory store.
__global__ void write_slot_kernel(Slot sl, Slot* dst)
{
    if (threadIdx.x == 0) *dst = sl;
}

__global__ void write_ctrl_kernel(CtrlBlock cb, int n, Ctrl* dst)
{
    const int z = threadIdx.x;
    if (z < n) dst[z] = cb.c[z];
}

inline dim3 grid_for(const Launch& lc) { return dim3((lc.g.W[lc.gl] + 63) / 64, lc.g.H[lc.gl], lc.n); }

}  // namespace

void launch_write_slot(const Slot& sl, Slot* dst, hipStream_t s)
{
    hipLaunchKernelGGL(write_slot_kernel, dim3(1), dim3(64), 0, s, sl, dst);
}

void launch_write_ctrl(const CtrlBlock& cb, int n, Ctrl* dst, hipStream_t s)
{
    hipLaunchKernelGGL(write_ctrl_kernel, dim3(1), dim3(kMaxBatch), 0, s, cb, n, dst);
}

void launch_prerotate(const Launch& lc, hipStream_t s)
{
    hipLaunchKernelGGL(prerotate_kernel, grid_for(lc), dim3(64), 0, s, lc);
}

void launch_downsample(const Launch& lc, hipStream_t s)
{
    hipLaunchKernelGGL(downsample_kernel, grid_for(lc), dim3(64), 0, s, lc);
}

#define VFS_BY_STORAGE(storage, call)                   \
    do {                                                \
        if ((storage) == ST_F16) { constexpr int S = ST_F16; call; }         \
        else if ((storage) == ST_BF16) { constexpr int S = ST_BF16; call; }  \
        else { constexpr int S = ST_F32; call; }                             \
    } while (0)

void launch_tensor(const Launch& lc, int storage, hipStream_t s)
{
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(tensor_kernel<S>, grid_for(lc), dim3(64), 0, s, lc));
}

void launch_linearise(const Launch& lc, int clip, int clip_only, float du_max, int xform, int storage,
                      hipStream_t s)
{
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(linearise_kernel<S>, grid_for(lc), dim3(64), 0, s, lc, clip,
                                               clip_only, du_max, xform));
}

void launch_transform(const Launch& lc, int kind, hipStream_t s)
{
    if (kind == 1) hipLaunchKernelGGL(transform_kernel<1>, grid_for(lc), dim3(64), 0, s, lc);
    else hipLaunchKernelGGL(transform_kernel<2>, grid_for(lc), dim3(64), 0, s, lc);
}

void launch_upsample(const Launch& lc, int tgv, int storage, hipStream_t s)
{
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(upsample_kernel<S>, grid_for(lc), dim3(64), 0, s, lc, tgv));
}

void launch_zero_state(const Launch& lc, int tgv, int storage, hipStream_t s)
{
    VFS_BY_STORAGE(storage, hipLaunchKernelGGL(zero_state_kernel<S>, grid_for(lc), dim3(64), 0, s, lc, tgv));
}

void launch_triangulate(const Launch& lc, hipStream_t s)
{
    hipLaunchKernelGGL(triangulate_kernel, grid_for(lc), dim3(64), 0, s, lc);
}

}  // namespace vfs
