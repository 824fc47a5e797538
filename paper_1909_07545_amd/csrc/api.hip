// C ABI (include/vfs.h): rig set-up, whole-method solves, step entry points,
// level-0 primal-dual timing.  Host code only enqueues work; the solve never
// waits on the device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <utility>
#include <vector>

#include "../../include/vfs.h"
#include "vfs_internal.h"

using namespace vfs;

namespace {

thread_local char g_err[512] = "";

vfs_status fail(vfs_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_OK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail(VFS_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr double kPi = 3.14159265358979323846;

int round_pitch(int w) { return (w + 63) / 64 * 64; }

// Largest angle of the grid i*pi/4096 up to which the radial map increases.
double theta_limit(const vfs_camera& c)
{
    if (c.model == VFS_PINHOLE) return 0.5 * kPi * (1.0 - 1e-9);
    if (c.model == VFS_EQUIDISTANT) return kPi;
    Cam t{};
    t.model = 2;
    for (int a = 0; a < 4; ++a) t.k[a] = c.k[a];
    for (int i = 1; i <= 4096; ++i)
        if (!(cam_drd(t, kPi * i / 4096.0) > 0.0)) return kPi * (i - 1) / 4096.0;
    return kPi;
}

vfs_status check_camera(const vfs_camera* c, const char* name)
{
    if (!c) return fail(VFS_E_INVALID, "%s is NULL", name);
    if (c->width <= 0 || c->height <= 0 || !(c->fx > 0.0) || !(c->fy > 0.0))
        return fail(VFS_E_INVALID, "%s: bad size or focal length", name);
    if (c->model < VFS_PINHOLE || c->model > VFS_KANNALA_BRANDT) return fail(VFS_E_INVALID, "%s: bad model", name);
    const double half = 0.5 * c->fov_deg * kPi / 180.0;
    if (!(half > 0.0)) return fail(VFS_E_INVALID, "%s: field of view must be positive", name);
    if (c->model == VFS_PINHOLE && !(half < 0.5 * kPi))
        return fail(VFS_E_MODEL, "%s: pinhole field of view must be below 180 degrees", name);
    if (half > kPi) return fail(VFS_E_MODEL, "%s: field of view above 360 degrees", name);
    if (c->model == VFS_KANNALA_BRANDT && theta_limit(*c) < half)
        return fail(VFS_E_MODEL, "%s: radial map not increasing up to half the field of view", name);
    return VFS_OK;
}

Cam to_cam(const vfs_camera& c)
{
    Cam o{};
    o.model = c.model;
    o.width = c.width;
    o.height = c.height;
    o.fx = c.fx; o.fy = c.fy; o.cx = c.cx; o.cy = c.cy;
    for (int a = 0; a < 4; ++a) o.k[a] = c.model == VFS_KANNALA_BRANDT ? c.k[a] : 0.0;
    o.th_lim = theta_limit(c);
    return o;
}

struct Level {
    int W, H, pitch;
    size_t plane;       // pitch * H
};

}  // namespace

struct vfs_rig {
    RigGeom geom;
    int L = 0;
    Level lv[kMaxLevels];
    float2* gamma[kMaxLevels] = {};
    uint8_t* flags[kMaxLevels] = {};
    float2* calib = nullptr;
    int device = 0;

    // workspace for up to `cap` pairs
    int cap = 0;
    void* ws = nullptr;
    size_t n0 = 0;              // elements of a level-0 plane
    size_t sj0 = 0, sj1 = 0;    // floats per pair of the J0 (levels >= 1) and J1 pyramids
    size_t off0[kMaxLevels] = {}, off1[kMaxLevels] = {};
    float* J0 = nullptr;
    float* J1 = nullptr;
    float* u[2] = {};
    float* uw = nullptr;
    float2* w[2] = {};
    float2* v[2] = {};
    void* p[2] = {};            // float2 / 2 x 16-bit per pixel, by storage
    void* q[2] = {};            // float4 / 4 x 16-bit
    void* tpack = nullptr;      // float4 / 4 x 16-bit
    float* rho = nullptr;
    float2* gw = nullptr;

    // level-0 primal-dual timing
    bool profile = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    long long launches = 0;
    double ms = 0.0;
    hipStream_t last_stream = nullptr;

    ~vfs_rig()
    {
        for (int l = 0; l < kMaxLevels; ++l) {
            if (gamma[l]) (void)hipFree(gamma[l]);
            if (flags[l]) (void)hipFree(flags[l]);
        }
        if (calib) (void)hipFree(calib);
        if (ws) (void)hipFree(ws);
        for (auto& e : events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};

namespace {

vfs_status ensure_workspace(vfs_rig* r, int n)
{
    if (n <= r->cap) return VFS_OK;
    if (r->ws) {
        HIP_OK(hipFree(r->ws));
        r->ws = nullptr;
        r->cap = 0;
    }
    const Level& l0 = r->lv[0];
    r->n0 = l0.plane;
    size_t sj0 = 0, sj1 = 0;
    for (int l = 0; l < r->L; ++l) {
        r->off1[l] = sj1;
        sj1 += r->lv[l].plane;
        r->off0[l] = sj0;
        if (l > 0) sj0 += r->lv[l].plane;
    }
    r->sj0 = sj0;
    r->sj1 = sj1;
    // float counts per pair: J0 (levels >= 1), J1, u x2, uw, w x2 (2), v x2 (2), p x2 (2),
    // q x2 (4), tpack (4), rho, gw (2)
    const size_t per = sj0 + sj1 + r->n0 * (2 + 1 + 4 + 4 + 4 + 8 + 4 + 1 + 2);
    const size_t bytes = per * sizeof(float) * size_t(n) + 4096;
    void* m = nullptr;
    if (hipMalloc(&m, bytes) != hipSuccess)
        return fail(VFS_E_NOMEM, "workspace of %zu bytes for %d pairs", bytes, n);
    r->ws = m;
    r->cap = n;
    float* f = static_cast<float*>(m);
    size_t at = 0;
    auto take = [&](size_t floats_per_pair) {
        float* ptr = f + at;
        at += floats_per_pair * size_t(n);
        return ptr;
    };
    r->J0 = take(sj0);
    r->J1 = take(sj1);
    r->u[0] = take(r->n0);
    r->u[1] = take(r->n0);
    r->uw = take(r->n0);
    r->w[0] = reinterpret_cast<float2*>(take(2 * r->n0));
    r->w[1] = reinterpret_cast<float2*>(take(2 * r->n0));
    r->v[0] = reinterpret_cast<float2*>(take(2 * r->n0));
    r->v[1] = reinterpret_cast<float2*>(take(2 * r->n0));
    r->p[0] = take(2 * r->n0);
    r->p[1] = take(2 * r->n0);
    r->q[0] = take(4 * r->n0);
    r->q[1] = take(4 * r->n0);
    r->tpack = take(4 * r->n0);
    r->rho = take(r->n0);
    r->gw = reinterpret_cast<float2*>(take(2 * r->n0));
    return VFS_OK;
}

// Scalar schedule of the over-relaxation (theta) and the step factors.
struct Sched {
    std::vector<float> s, theta;
};

Sched schedule(const vfs_params& p)
{
    Sched sc;
    sc.s.resize(p.iters + 1);
    sc.theta.resize(p.iters + 1);
    double s = 1.0;
    for (int k = 0; k <= p.iters; ++k) {
        double th = 1.0;
        if (p.theta_gamma > 0.0) th = 1.0 / sqrt(1.0 + 2.0 * p.theta_gamma * s);
        sc.s[k] = float(s);
        sc.theta[k] = float(th);
        s = th * s;
    }
    return sc;
}

vfs_status check_params(const vfs_params* p)
{
    if (!p) return fail(VFS_E_INVALID, "params is NULL");
    if (p->levels < 1 || p->levels > kMaxLevels) return fail(VFS_E_INVALID, "levels must be in [1, %d]", kMaxLevels);
    if (p->warps < 0 || p->iters < 0) return fail(VFS_E_INVALID, "warps and iters must be >= 0");
    if (p->reg != VFS_TGV && p->reg != VFS_TV) return fail(VFS_E_INVALID, "bad regulariser");
    if (p->storage != VFS_F32 && p->storage != VFS_F16 && p->storage != VFS_BF16)
        return fail(VFS_E_INVALID, "unsupported storage");
    if (!(p->alpha0 > 0.0) || !(p->alpha1 > 0.0) || !(p->lambda >= 0.0) || !(p->du_max > 0.0) ||
        !(p->theta_gamma >= 0.0) || !(p->beta >= 0.0) || !(p->eta > 0.0))
        return fail(VFS_E_INVALID, "bad solver constants");
    return VFS_OK;
}

// K primal-dual iterations from a warp start on the state index pair (iu, ip);
// the indices are updated to those holding the result.  Returns the number of
// two-iteration launches, which ev0 / ev1 (if given) bracket.
int run_pd(PdArgs base, const Sched& sc, int K, float* const* u, float2* const* v, void* const* p,
           void* const* q, int& iu, int& ip, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (K <= 0) return 0;
    auto bind = [&](PdArgs& a) {
        a.u_in = u[iu]; a.v_in = v ? v[iu] : nullptr; a.p_in = p[ip]; a.q_in = q ? q[ip] : nullptr;
        a.u_out = u[1 - iu]; a.v_out = v ? v[1 - iu] : nullptr;
        a.p_out = p[1 - ip]; a.q_out = q ? q[1 - ip] : nullptr;
    };
    PdArgs a = base;
    a.mode = PD_DUAL_FIRST;
    a.tau_scale = 1.f;
    a.sigma_scale = 1.f / sc.s[0];
    a.theta = 1.f;
    bind(a);
    launch_pd(a, s);
    ip = 1 - ip;
    // iterations 1 .. K-1: an odd one alone, then pairs in one pass each
    int k = 1;
    if ((K - 1) % 2) {
        a.mode = PD_FUSED;
        a.tau_scale = sc.s[k - 1];
        a.theta = sc.theta[k - 1];
        a.sigma_scale = 1.f / sc.s[k];
        bind(a);
        launch_pd(a, s);
        iu = 1 - iu;
        ip = 1 - ip;
        ++k;
    }
    if (ev0) (void)hipEventRecord(ev0, s);
    int pairs = 0;
    for (; k + 1 <= K - 1; k += 2, ++pairs) {
        a.mode = PD_FUSED2;
        a.tau_scale = sc.s[k - 1];
        a.theta = sc.theta[k - 1];
        a.sigma_scale = 1.f / sc.s[k];
        a.tau_scale2 = sc.s[k];
        a.theta2 = sc.theta[k];
        a.sigma_scale2 = 1.f / sc.s[k + 1];
        bind(a);
        launch_pd(a, s);
        iu = 1 - iu;
        ip = 1 - ip;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    a.mode = PD_PRIMAL_LAST;
    a.tau_scale = sc.s[K - 1];
    a.sigma_scale = 1.f;
    a.theta = 1.f;
    bind(a);
    launch_pd(a, s);
    iu = 1 - iu;
    return pairs;
}

}  // namespace

extern "C" {

const char* vfs_last_error(void) { return g_err; }

vfs_status vfs_params_default(vfs_params* out)
{
    if (!out) return fail(VFS_E_INVALID, "out is NULL");
    out->levels = 5;
    out->warps = 10;
    out->iters = 100;
    out->reg = VFS_TGV;
    out->lambda = 50.0;
    out->alpha0 = 17.0;
    out->alpha1 = 1.2;
    out->beta = 9.0;
    out->eta = 0.85;
    out->du_max = 0.2;
    out->theta_gamma = 0.0;
    out->storage = VFS_F32;
    return VFS_OK;
}

vfs_status vfs_rig_create(const vfs_camera* cam0, const vfs_camera* cam1, const double R[9], const double t[3],
                          int levels, void* hip_stream, vfs_rig** out)
{
    g_err[0] = 0;
    if (!out) return fail(VFS_E_INVALID, "out is NULL");
    *out = nullptr;
    vfs_status st = check_camera(cam0, "cam0");
    if (st) return st;
    st = check_camera(cam1, "cam1");
    if (st) return st;
    if (!R || !t) return fail(VFS_E_INVALID, "R or t is NULL");
    if (cam0->width != cam1->width || cam0->height != cam1->height)
        return fail(VFS_E_INVALID, "cameras must have the same image size");
    if (levels < 1 || levels > kMaxLevels) return fail(VFS_E_INVALID, "levels must be in [1, %d]", kMaxLevels);
    const int div = 1 << (levels - 1);
    if (cam0->width % div || cam0->height % div)
        return fail(VFS_E_INVALID, "image size %dx%d not divisible by 2^(levels-1) = %d", cam0->width, cam0->height, div);
    for (int a = 0; a < 9; ++a)
        if (!isfinite(R[a])) return fail(VFS_E_INVALID, "R is not finite");
    double tp[3];
    for (int a = 0; a < 3; ++a) tp[a] = R[a] * t[0] + R[3 + a] * t[1] + R[6 + a] * t[2];
    const double tn = sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
    if (!isfinite(tn)) return fail(VFS_E_INVALID, "t is not finite");
    if (!(tn > 0.0)) return fail(VFS_E_DEGENERATE, "zero baseline: the trajectory field is undefined");

    vfs_rig* r = new (std::nothrow) vfs_rig();
    if (!r) return fail(VFS_E_NOMEM, "host allocation");
    RigGeom& g = r->geom;
    g.cam0 = to_cam(*cam0);
    g.cam1 = to_cam(*cam1);
    for (int a = 0; a < 9; ++a) g.R[a] = R[a];
    for (int a = 0; a < 3; ++a) {
        g.tdir[a] = tp[a] / tn;
        g.C[a] = -tp[a];
    }
    g.rmax0 = cam_rd(g.cam0, 0.5 * cam0->fov_deg * kPi / 180.0);
    g.half1 = 0.5 * cam1->fov_deg * kPi / 180.0;
    g.cos_guard = cos(2.0 * kPi / 180.0);
    g.eps = 1e-6;
    r->L = levels;
    for (int l = 0; l < levels; ++l) {
        Level& lv = r->lv[l];
        lv.W = cam0->width >> l;
        lv.H = cam0->height >> l;
        lv.pitch = round_pitch(lv.W);
        lv.plane = size_t(lv.pitch) * lv.H;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto cleanup = [&](vfs_status e) { delete r; return e; };
    if (hipGetDevice(&r->device) != hipSuccess) return cleanup(fail(VFS_E_DEVICE, "hipGetDevice failed"));
    for (int l = 0; l < levels; ++l) {
        const Level& lv = r->lv[l];
        if (hipMalloc(&r->gamma[l], lv.plane * sizeof(float2)) != hipSuccess ||
            hipMalloc(&r->flags[l], lv.plane) != hipSuccess)
            return cleanup(fail(VFS_E_NOMEM, "rig fields"));
        if (hipMemsetAsync(r->gamma[l], 0, lv.plane * sizeof(float2), s) != hipSuccess ||
            hipMemsetAsync(r->flags[l], 0, lv.plane, s) != hipSuccess)
            return cleanup(fail(VFS_E_DEVICE, "clearing rig fields"));
        launch_level_fields(g, l, r->gamma[l], r->flags[l], lv.pitch, s);
    }
    if (hipMalloc(&r->calib, r->lv[0].plane * sizeof(float2)) != hipSuccess)
        return cleanup(fail(VFS_E_NOMEM, "calibration field"));
    launch_calibration(g, r->calib, r->lv[0].pitch, s);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return cleanup(fail(VFS_E_DEVICE, "rig set-up kernels failed"));
    *out = r;
    return VFS_OK;
}

void vfs_rig_destroy(vfs_rig* rig) { delete rig; }

vfs_status vfs_rig_field(const vfs_rig* r, int level, int which, void* dst, size_t pitch_bytes, void* hip_stream)
{
    g_err[0] = 0;
    if (!r || !dst) return fail(VFS_E_INVALID, "NULL argument");
    if (level < 0 || level >= r->L) return fail(VFS_E_INVALID, "level out of range");
    if (which < 0 || which > 2 || (which == 1 && level != 0)) return fail(VFS_E_INVALID, "bad field");
    const Level& lv = r->lv[level];
    const size_t esz = which == 2 ? 1 : sizeof(float2);
    if (pitch_bytes < esz * lv.W) return fail(VFS_E_INVALID, "pitch too small");
    const void* src = which == 0 ? (const void*)r->gamma[level] : which == 1 ? (const void*)r->calib
                                                                            : (const void*)r->flags[level];
    HIP_OK(hipMemcpy2DAsync(dst, pitch_bytes, src, esz * lv.pitch, esz * lv.W, lv.H, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(hip_stream)));
    return VFS_OK;
}

vfs_status vfs_solve_batch(vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                           float* const* u_out, float* const* w_out, float* const* depth_out, float* const* z_out,
                           uint8_t* const* valid_out, const vfs_params* params, const double* betas,
                           const double* etas, void* hip_stream)
{
    g_err[0] = 0;
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    if (n < 1 || n > kMaxBatch) return fail(VFS_E_INVALID, "n must be in [1, %d]", kMaxBatch);
    vfs_status st = check_params(params);
    if (st) return st;
    if (params->levels != r->L) return fail(VFS_E_INVALID, "params->levels (%d) differs from the rig's (%d)",
                                            params->levels, r->L);
    const Level& l0 = r->lv[0];
    if (pitch_bytes % sizeof(float) || pitch_bytes < sizeof(float) * l0.W)
        return fail(VFS_E_INVALID, "bad pitch");
    if (!I0 || !I1 || !u_out || !w_out || !depth_out) return fail(VFS_E_INVALID, "NULL array argument");
    for (int b = 0; b < n; ++b) {
        if (!I0[b] || !I1[b] || !u_out[b] || !w_out[b] || !depth_out[b])
            return fail(VFS_E_INVALID, "NULL buffer for pair %d", b);
        if ((betas && !(betas[b] >= 0.0)) || (etas && !(etas[b] > 0.0)))
            return fail(VFS_E_INVALID, "bad tensor parameters for pair %d", b);
    }
    st = ensure_workspace(r, n);
    if (st) return st;

    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    r->last_stream = s;
    const int ip_caller = int(pitch_bytes / sizeof(float));
    const long long N0 = (long long)r->n0;
    const int L = r->L;
    const bool tgv = params->reg == VFS_TGV;

    // A1: pre-rotation of I1 (Sec. IV-A) into level 0 of the J1 pyramid
    PairPtrs in1;
    in1.in_pitch = ip_caller;
    for (int b = 0; b < n; ++b) in1.in[b] = I1[b];
    launch_prerotate(in1, n, l0.W, l0.H, r->calib, l0.pitch, r->J1 + r->off1[0], l0.pitch, (long long)r->sj1, s);

    // A2: pyramids (Sec. IV-B); level 0 of J0 is the caller's image
    const float* j0[kMaxLevels][kMaxBatch];
    int j0pitch[kMaxLevels];
    for (int b = 0; b < n; ++b) j0[0][b] = I0[b];
    j0pitch[0] = ip_caller;
    for (int l = 1; l < L; ++l) {
        const Level& lv = r->lv[l];
        for (int b = 0; b < n; ++b) j0[l][b] = r->J0 + b * r->sj0 + r->off0[l];
        j0pitch[l] = lv.pitch;
        launch_downsample(n, lv.W, lv.H, j0[l - 1], j0pitch[l - 1], 0, r->J0 + r->off0[l], lv.pitch,
                          (long long)r->sj0, s);
        const float* f1[kMaxBatch];
        for (int b = 0; b < n; ++b) f1[b] = r->J1 + b * r->sj1 + r->off1[l - 1];
        launch_downsample(n, lv.W, lv.H, f1, r->lv[l - 1].pitch, 0, r->J1 + r->off1[l], lv.pitch,
                          (long long)r->sj1, s);
    }

    float bet[kMaxBatch], et[kMaxBatch];
    for (int b = 0; b < n; ++b) {
        bet[b] = float(betas ? betas[b] : params->beta);
        et[b] = float(etas ? etas[b] : params->eta);
    }
    const Sched sc = schedule(*params);
    int iu = 0, ip = 0, iw = 0;

    for (int l = L - 1; l >= 0; --l) {
        const Level& lv = r->lv[l];
        // A3: tensor of the level (Eq. (12))
        launch_tensor(n, lv.W, lv.H, j0[l], j0pitch[l], 0, r->flags[l], lv.pitch, bet, et, r->tpack, lv.pitch, N0,
                      params->storage, s);
        // A7: state of the level: zero at the coarsest, else transferred from level l+1
        if (l == L - 1) {
            launch_zero_state(n, lv.W, lv.H, lv.pitch, N0, r->u[iu], r->w[iw], tgv ? r->v[iu] : nullptr, r->p[ip],
                              tgv ? r->q[ip] : nullptr, params->storage, s);
        } else {
            const Level& lc = r->lv[l + 1];
            launch_upsample(n, lc.W, lc.H, lc.pitch, N0, r->flags[l + 1], lc.pitch, r->u[iu], r->w[iw], lv.pitch, N0,
                            r->u[1 - iu], r->w[1 - iw], tgv ? r->v[1 - iu] : nullptr, r->p[ip],
                            tgv ? r->q[ip] : nullptr, params->storage, s);
            iu = 1 - iu;
            iw = 1 - iw;
        }
        PdArgs pa{};
        pa.W = lv.W;
        pa.H = lv.H;
        pa.pitch = lv.pitch;
        pa.stride = N0;
        pa.n = n;
        pa.tpack = r->tpack;
        pa.rho = r->rho;
        pa.flags = r->flags[l];
        pa.alpha0 = float(params->alpha0);
        pa.alpha1 = float(params->alpha1);
        pa.lambda = float(params->lambda);
        pa.tgv = tgv ? 1 : 0;
        pa.storage = params->storage;
        const float* J1l = r->J1 + r->off1[l];
        for (int wv = 0; wv <= params->warps; ++wv) {
            // A4 (+A6 of the previous warp): clip, accumulate, linearise
            const bool last = wv == params->warps;
            if (last && wv == 0) break;
            launch_linearise(n, lv.W, lv.H, lv.pitch, N0, j0[l], j0pitch[l], 0, J1l, (long long)r->sj1, r->gamma[l],
                             r->flags[l], r->u[iu], r->uw, r->w[iw], r->gw, r->tpack, r->rho, wv > 0 ? 1 : 0,
                             last ? 1 : 0, float(params->du_max), params->storage, s);
            if (last) break;
            // A5: K primal-dual iterations (Eq. (11))
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (r->profile && l == 0 && params->iters >= 3) {
                if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                    return fail(VFS_E_DEVICE, "hipEventCreate");
                r->events.emplace_back(e0, e1);
            }
            const int np = run_pd(pa, sc, params->iters, r->u, tgv ? r->v : nullptr, r->p, tgv ? r->q : nullptr, iu,
                                  ip, s, e0, e1);
            if (e0) r->launches += np;
        }
    }
    // A8: triangulation and outputs
    launch_triangulate(n, r->geom, l0.W, l0.H, l0.pitch, N0, r->u[iu], r->w[iw], r->flags[0], l0.pitch, u_out, w_out,
                       depth_out, z_out, valid_out, ip_caller, s);
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_solve(vfs_rig* rig, const float* I0, const float* I1, size_t pitch_bytes, float* u_out, float* w_out,
                     float* depth_out, float* z_out, uint8_t* valid_out, const vfs_params* params, void* hip_stream)
{
    return vfs_solve_batch(rig, 1, &I0, &I1, pitch_bytes, &u_out, &w_out, &depth_out, z_out ? &z_out : nullptr,
                           valid_out ? &valid_out : nullptr, params, nullptr, nullptr, hip_stream);
}

// ---------------------------------------------------------------- step entry points

vfs_status vfs_step_tensor(int W, int H, size_t pitch, const float* J0, const uint8_t* flags, double beta, double eta,
                           float* tpack, void* hip_stream)
{
    g_err[0] = 0;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !J0 || !flags || !tpack || !(beta >= 0.0) || !(eta > 0.0))
        return fail(VFS_E_INVALID, "bad argument");
    const float* j[1] = {J0};
    const float b = float(beta), e = float(eta);
    launch_tensor(1, W, H, j, int(pitch), 0, flags, int(pitch), &b, &e, tpack, int(pitch), 0, ST_F32,
                  static_cast<hipStream_t>(hip_stream));
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_step_linearise(int W, int H, size_t pitch, const float* J0, const float* J1, const float* gamma,
                              const uint8_t* flags, float* u, float* u_w, float* w, float* gamma_w, float* tpack,
                              float* rho, int clip, int clip_only, double du_max, void* hip_stream)
{
    g_err[0] = 0;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !J0 || !J1 || !gamma || !flags || !u || !u_w || !w || !gamma_w ||
        !tpack || !rho || !(du_max > 0.0))
        return fail(VFS_E_INVALID, "bad argument");
    const float* j[1] = {J0};
    launch_linearise(1, W, H, int(pitch), 0, j, int(pitch), 0, J1, 0, reinterpret_cast<const float2*>(gamma), flags, u,
                     u_w, reinterpret_cast<float2*>(w), reinterpret_cast<float2*>(gamma_w), tpack, rho, clip ? 1 : 0,
                     clip_only ? 1 : 0, float(du_max), ST_F32, static_cast<hipStream_t>(hip_stream));
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_step_pd(int W, int H, size_t pitch, const float* tpack, const float* rho, const uint8_t* flags, float* u,
                       float* v, float* p, float* q, float* su, float* sv, float* sp, float* sq,
                       const vfs_params* params, int iters, void* hip_stream)
{
    g_err[0] = 0;
    vfs_status st = check_params(params);
    if (st) return st;
    const bool tgv = params->reg == VFS_TGV;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !tpack || !rho || !flags || !u || !p || !su || !sp || iters < 0 ||
        (tgv && (!v || !q || !sv || !sq)))
        return fail(VFS_E_INVALID, "bad argument");
    if (iters == 0) return VFS_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs_params pp = *params;
    pp.iters = iters;
    const Sched sc = schedule(pp);
    PdArgs a{};
    a.W = W; a.H = H; a.pitch = int(pitch); a.stride = 0; a.n = 1;
    a.tpack = tpack;
    a.storage = ST_F32;
    a.rho = rho;
    a.flags = flags;
    a.alpha0 = float(params->alpha0);
    a.alpha1 = float(params->alpha1);
    a.lambda = float(params->lambda);
    a.tgv = tgv ? 1 : 0;
    float* U[2] = {u, su};
    float2* V[2] = {reinterpret_cast<float2*>(v), reinterpret_cast<float2*>(sv)};
    void* P[2] = {p, sp};
    void* Q[2] = {q, sq};
    int iu = 0, ip = 0;
    run_pd(a, sc, iters, U, tgv ? V : nullptr, P, tgv ? Q : nullptr, iu, ip, s, nullptr, nullptr);
    const size_t plane = pitch * size_t(H);
    if (iu) {
        HIP_OK(hipMemcpyAsync(u, su, plane * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (tgv) HIP_OK(hipMemcpyAsync(v, sv, plane * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    if (ip) {
        HIP_OK(hipMemcpyAsync(p, sp, plane * sizeof(float2), hipMemcpyDeviceToDevice, s));
        if (tgv) HIP_OK(hipMemcpyAsync(q, sq, plane * sizeof(float4), hipMemcpyDeviceToDevice, s));
    }
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_step_upsample(int Wc, int Hc, size_t pitch_c, const uint8_t* flags_c, const float* u_c, const float* w_c,
                             size_t pitch_f, float* u_f, float* w_f, void* hip_stream)
{
    g_err[0] = 0;
    if (Wc <= 0 || Hc <= 0 || pitch_c < size_t(Wc) || pitch_f < size_t(2 * Wc) || !flags_c || !u_c || !w_c || !u_f ||
        !w_f)
        return fail(VFS_E_INVALID, "bad argument");
    launch_upsample(1, Wc, Hc, int(pitch_c), 0, flags_c, int(pitch_c), u_c, reinterpret_cast<const float2*>(w_c),
                    int(pitch_f), 0, u_f, reinterpret_cast<float2*>(w_f), nullptr, nullptr, nullptr, ST_F32,
                    static_cast<hipStream_t>(hip_stream));
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_step_triangulate(const vfs_rig* r, size_t pitch, const float* w, float* depth, float* z, uint8_t* valid,
                                void* hip_stream)
{
    g_err[0] = 0;
    if (!r || !w || !depth) return fail(VFS_E_INVALID, "NULL argument");
    const Level& l0 = r->lv[0];
    if (pitch < size_t(l0.W)) return fail(VFS_E_INVALID, "pitch too small");
    // reads u only to copy it to u_out, which is not requested here
    float* dz[1] = {depth};
    float* zz[1] = {z};
    uint8_t* vv[1] = {valid};
    launch_triangulate(1, r->geom, l0.W, l0.H, int(pitch), 0, nullptr, reinterpret_cast<const float2*>(w),
                       r->flags[0], l0.pitch, nullptr, nullptr, dz, z ? zz : nullptr, valid ? vv : nullptr,
                       int(pitch), static_cast<hipStream_t>(hip_stream));
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_profile_enable(vfs_rig* r, int enable)
{
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    r->profile = enable != 0;
    return VFS_OK;
}

vfs_status vfs_profile_read(vfs_rig* r, double* ms, long long* launches, int reset)
{
    g_err[0] = 0;
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    if (!r->events.empty()) {
        HIP_OK(hipStreamSynchronize(r->last_stream));
        for (auto& e : r->events) {
            float t = 0.f;
            HIP_OK(hipEventElapsedTime(&t, e.first, e.second));
            r->ms += t;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        r->events.clear();
    }
    if (ms) *ms = r->ms;
    if (launches) *launches = r->launches;
    if (reset) {
        r->ms = 0.0;
        r->launches = 0;
    }
    return VFS_OK;
}

}  // extern "C"
