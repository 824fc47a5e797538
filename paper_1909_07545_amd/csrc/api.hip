// C ABI (include/vfs.h): rig set-up, whole-method solves, step entry points,
// level-0 primal-dual timing.  Host code only enqueues work; the solve never
// waits on the device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "runtime.h"

using namespace vfs;

namespace vfs {

thread_local char g_err[512] = "";

vfs_status fail(vfs_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace vfs

#define HIP_OK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail(VFS_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr double kPi = 3.14159265358979323846;

// Largest angle of the grid i*pi/4096 up to which the radial map is defined
// (unified models: positive denominator) and increases.
double theta_limit(const vfs_camera& c)
{
    if (c.model == VFS_PINHOLE) return 0.5 * kPi * (1.0 - 1e-9);
    if (c.model == VFS_EQUIDISTANT) return kPi;
    Cam t{};
    t.model = c.model;
    for (int a = 0; a < 4; ++a) t.k[a] = c.k[a];
    for (int i = 1; i <= 4096; ++i) {
        const double th = kPi * i / 4096.0;
        if (t.model >= VFS_UNIFIED && !(cam_uden(t, th) > 0.0)) return kPi * (i - 1) / 4096.0;
        if (!(cam_drd(t, th) > 0.0)) return kPi * (i - 1) / 4096.0;
    }
    return kPi;
}

vfs_status check_camera(const vfs_camera* c, const char* name)
{
    if (!c) return fail(VFS_E_INVALID, "%s is NULL", name);
    if (c->width <= 0 || c->height <= 0 || !(c->fx > 0.0) || !(c->fy > 0.0))
        return fail(VFS_E_INVALID, "%s: bad size or focal length", name);
    if (c->width > kMaxWidth) return fail(VFS_E_INVALID, "%s: width above %d", name, kMaxWidth);
    if (c->model < VFS_PINHOLE || c->model > VFS_ENHANCED_UNIFIED) return fail(VFS_E_INVALID, "%s: bad model", name);
    if (c->model == VFS_UNIFIED && !(c->k[0] >= 0.0)) return fail(VFS_E_INVALID, "%s: unified model needs xi >= 0", name);
    if (c->model == VFS_ENHANCED_UNIFIED && !(c->k[0] >= 0.0 && c->k[0] <= 1.0 && c->k[1] > 0.0))
        return fail(VFS_E_INVALID, "%s: enhanced unified model needs 0 <= alpha <= 1, beta > 0", name);
    const double half = 0.5 * c->fov_deg * kPi / 180.0;
    if (!(half > 0.0)) return fail(VFS_E_INVALID, "%s: field of view must be positive", name);
    if (c->model == VFS_PINHOLE && !(half < 0.5 * kPi))
        return fail(VFS_E_MODEL, "%s: pinhole field of view must be below 180 degrees", name);
    if (half > kPi) return fail(VFS_E_MODEL, "%s: field of view above 360 degrees", name);
    if (c->model >= VFS_KANNALA_BRANDT && theta_limit(*c) < half)
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
    for (int a = 0; a < 4; ++a) o.k[a] = c.model >= VFS_KANNALA_BRANDT ? c.k[a] : 0.0;
    o.th_lim = theta_limit(c);
    return o;
}

}  // namespace

vfs_rig::~vfs_rig()
{
    for (int l = 0; l < vfs::kMaxLevels; ++l) {
        if (gamma[l]) (void)hipFree(gamma[l]);
        if (flags[l]) (void)hipFree(flags[l]);
    }
    if (calib) (void)hipFree(calib);
    if (radial) (void)hipFree(radial);
    if (geom_dev) (void)hipFree(geom_dev);
    for (auto& e : events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto& gr : graphs) {
        (void)hipGraphExecDestroy(gr.exec);
        (void)hipGraphDestroy(gr.graph);
    }
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

namespace vfs {

Geometry make_geometry(int W, int H, int L)
{
    Geometry g{};
    g.L = L;
    long long off = 0;
    for (int l = 0; l < L; ++l) {
        g.W[l] = W >> l;
        g.H[l] = H >> l;
        g.pitch[l] = ((W >> l) + 63) / 64 * 64;
        g.off[l] = off;
        off += (long long)g.pitch[l] * g.H[l];
    }
    return g;
}

PairLayout make_layout(const Geometry& g, int storage, bool tgv, bool xform)
{
    PairLayout y{};
    y.storage = storage;
    y.tgv = tgv;
    y.xform = xform;
    const size_t st = stacked_elems(g), one = plane_elems(g, 0);
    const size_t e2 = storage == ST_F32 ? 8 : 4, e4 = storage == ST_F32 ? 16 : 8;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at += (bytes + 255) / 256 * 256;
        return o;
    };
    y.J0 = take(st * 4);
    y.J1 = take(st * 4);
    for (int k = 0; k < 2; ++k) y.u[k] = take(st * 4);
    for (int k = 0; k < 2; ++k) y.p[k] = take(st * e2);
    if (tgv) {
        for (int k = 0; k < 2; ++k) y.v[k] = take(st * 8);
        for (int k = 0; k < 2; ++k) y.q[k] = take(st * e4);
    }
    y.w = take(st * 8);
    y.uw = take(one * 4);
    y.gw = take(one * 8);
    y.tpack = take(one * e4);
    y.rho = take(one * 4);
    if (xform) {
        y.R0 = take(one * 4);
        y.R1 = take(one * 4);
    }
    y.bytes = at;
    return y;
}

void bind_state(Slot& sl, void* region, const PairLayout& y)
{
    char* m = static_cast<char*>(region);
    sl.J0 = reinterpret_cast<float*>(m + y.J0);
    sl.J1 = reinterpret_cast<float*>(m + y.J1);
    for (int k = 0; k < 2; ++k) {
        sl.u[k] = reinterpret_cast<float*>(m + y.u[k]);
        sl.p[k] = m + y.p[k];
        sl.v[k] = y.tgv ? reinterpret_cast<float2*>(m + y.v[k]) : nullptr;
        sl.q[k] = y.tgv ? static_cast<void*>(m + y.q[k]) : nullptr;
    }
    sl.w = reinterpret_cast<float2*>(m + y.w);
    sl.uw = reinterpret_cast<float*>(m + y.uw);
    sl.gw = reinterpret_cast<float2*>(m + y.gw);
    sl.tpack = m + y.tpack;
    sl.rho = reinterpret_cast<float*>(m + y.rho);
    sl.R0 = y.xform ? reinterpret_cast<float*>(m + y.R0) : nullptr;
    sl.R1 = y.xform ? reinterpret_cast<float*>(m + y.R1) : nullptr;
}

void bind_rig(Slot& sl, const vfs_rig* r)
{
    for (int l = 0; l < kMaxLevels; ++l) {
        sl.gamma[l] = l < r->g.L ? r->gamma[l] : nullptr;
        sl.flags[l] = l < r->g.L ? r->flags[l] : nullptr;
    }
    sl.calib = r->calib;
    sl.geom = r->geom_dev;
}

void Workspace::release()
{
    if (mem) (void)hipFree(mem);
    if (slots) (void)hipFree(slots);
    mem = nullptr;
    slots = nullptr;
    cap = 0;
}

vfs_status ensure_workspace(Workspace& ws, const Geometry& g, int n, int storage, bool tgv, bool xform)
{
    bool same = ws.mem && ws.cap >= n && ws.g.L == g.L && ws.lay.storage == storage && ws.lay.tgv == tgv &&
                ws.lay.xform == xform;
    for (int l = 0; same && l < g.L; ++l) same = ws.g.W[l] == g.W[l] && ws.g.H[l] == g.H[l];
    if (same) return VFS_OK;
    ws.release();
    ws.g = g;
    ws.lay = make_layout(g, storage, tgv, xform);
    const size_t bytes = ws.lay.bytes * size_t(n);
    void* m = nullptr;
    if (hipMalloc(&m, bytes) != hipSuccess) return fail(VFS_E_NOMEM, "workspace of %zu bytes for %d pairs", bytes, n);
    ws.mem = m;
    if (hipMalloc(&ws.slots, sizeof(Slot) * kMaxBatch) != hipSuccess) {
        ws.release();
        return fail(VFS_E_NOMEM, "slot descriptors");
    }
    ws.cap = n;
    return VFS_OK;
}

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
    if (p->pass_iters != 0 && (p->pass_iters < 2 || p->pass_iters > 4))
        return fail(VFS_E_INVALID, "pass_iters must be 0 (automatic) or 2, 3, 4");
    if (p->data_term < VFS_DATA_BRIGHTNESS || p->data_term > VFS_DATA_GRADIENT)
        return fail(VFS_E_INVALID, "unknown data term");
    if (!(p->alpha0 > 0.0) || !(p->alpha1 > 0.0) || !(p->lambda >= 0.0) || !(p->du_max > 0.0) ||
        !(p->theta_gamma >= 0.0) || !(p->beta >= 0.0) || !(p->eta > 0.0))
        return fail(VFS_E_INVALID, "bad solver constants");
    return VFS_OK;
}

// Iterations per pass of the dominant primal-dual launches for pairs whose
// level 0 is g's, in a storage mode, unless `requested` (2, 3 or 4) fixes it.
// Measured on MI355X, whole solves: four iterations per pass in FP32 from
// 2 M level-0 pixels (8 pairs of 2048x2048: 165.3 Gpix-iter/s against 134.6
// with three); three with 16-bit storage there (chosen at 171.6 against
// 162.6 with four, the 16-bit kernels spending more vector issue per
// iteration; since the first pass of a warp and the next-row prefetch, four
// measure 0.6 % faster, kept at three because the 16-bit accuracy figures
// were measured with it and a change of depth moves the points where the
// duals are rounded); and three
// on smaller pairs in both modes, where the launches are latency-bound and
// fewer of them per warp pays (1280x1024: 55.6 against 50.0 with two and 52.6
// with four; 640x480: 19.6 against 18.6 and 18.6; the serving study: 386
// against 364 pairs/s with two).  The choice depends on the pair's size and
// the storage only, not on how many pairs share a launch, so that a pair's
// result does not depend on its batch (16-bit storage rounds the duals at
// pass boundaries; in FP32 the pass depth changes no result).
int pd_pass_iters(const Geometry& g, int requested, int storage)
{
    if (requested >= 2 && requested <= 4) return requested;
    if ((long long)g.W[0] * g.H[0] < (2ll << 20)) return 3;
    return storage == VFS_F32 ? 4 : 3;
}

// Whether the K iterations of a warp start with a multi-iteration pass whose
// first iteration is the dual half alone (PD_FIRST2 / 3 / 4) rather than with
// a PD_DUAL_FIRST launch: whenever K >= NP.
static bool first_pass(int K, int NP) { return NP >= 2 && K >= NP; }

void pd_parity(int K, int NP, int& pu, int& pp)
{
    pu = pp = 0;
    if (K <= 0) return;
    const bool fp = first_pass(K, NP);
    const int k0 = fp ? NP : 1;                      // the first iteration left after the start
    const int rem = (K - k0) % NP, passes = (K - k0) / NP;
    const int both = rem % 2 + rem / 2 + passes + (fp ? 1 : 0);  // launches that flip both copies
    pp = (both + (fp ? 0 : 1)) & 1;                  // plus PD_DUAL_FIRST (dual only)
    pu = (both + 1) & 1;                             // plus the last (primal only)
}

int run_pd(PdArgs base, const Sched& sc, int K, int& iu, int& ip, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    iu = base.lc.iu;
    ip = base.lc.ip;
    if (K <= 0) return 0;
    PdArgs a = base;
    auto go = [&]() {
        a.lc.iu = iu;
        a.lc.ip = ip;
        launch_pd(a, s);
    };
    const int NP = base.pass;
    int k = 1;
    if (first_pass(K, NP)) {
        // y^1 and iterations 1 .. NP-1 in one pass
        a.mode = NP == 2 ? PD_FIRST2 : NP == 3 ? PD_FIRST3 : PD_FIRST4;
        a.tau_n[0] = 1.f;
        a.theta_n[0] = 1.f;
        a.sigma_n[0] = 1.f / sc.s[0];
        for (int i = 1; i < NP; ++i) {
            a.tau_n[i] = sc.s[i - 1];
            a.theta_n[i] = sc.theta[i - 1];
            a.sigma_n[i] = 1.f / sc.s[i];
        }
        go();
        iu ^= 1;
        ip ^= 1;
        k = NP;
    } else {
        a.mode = PD_DUAL_FIRST;
        a.tau_scale = 1.f;
        a.sigma_scale = 1.f / sc.s[0];
        a.theta = 1.f;
        go();
        ip ^= 1;
    }
    // iterations k .. K-1: the remainder first (one alone, then a pair),
    // then passes of NP iterations each
    int rem = (K - k) % NP;
    if (rem % 2) {
        a.mode = PD_FUSED;
        a.tau_scale = sc.s[k - 1];
        a.theta = sc.theta[k - 1];
        a.sigma_scale = 1.f / sc.s[k];
        go();
        iu ^= 1;
        ip ^= 1;
        ++k;
        --rem;
    }
    for (; rem >= 2; rem -= 2, k += 2) {
        a.mode = PD_FUSED2;
        for (int i = 0; i < 2; ++i) {
            a.tau_n[i] = sc.s[k + i - 1];
            a.theta_n[i] = sc.theta[k + i - 1];
            a.sigma_n[i] = 1.f / sc.s[k + i];
        }
        go();
        iu ^= 1;
        ip ^= 1;
    }
    if (ev0) (void)hipEventRecord(ev0, s);
    int passes = 0;
    for (; k + NP - 1 <= K - 1; k += NP, ++passes) {
        a.mode = NP == 2 ? PD_FUSED2 : NP == 3 ? PD_FUSED3 : PD_FUSED4;
        for (int i = 0; i < NP; ++i) {
            a.tau_n[i] = sc.s[k + i - 1];
            a.theta_n[i] = sc.theta[k + i - 1];
            a.sigma_n[i] = 1.f / sc.s[k + i];
        }
        go();
        iu ^= 1;
        ip ^= 1;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    a.mode = PD_PRIMAL_LAST;
    a.tau_scale = sc.s[K - 1];
    a.sigma_scale = 1.f;
    a.theta = 1.f;
    go();
    iu ^= 1;
    return passes;
}

PdArgs pd_args(const Launch& lc, const vfs_params& params)
{
    PdArgs pa{};
    pa.lc = lc;
    pa.alpha0 = float(params.alpha0);
    pa.alpha1 = float(params.alpha1);
    pa.lambda = float(params.lambda);
    pa.tgv = params.reg == VFS_TGV ? 1 : 0;
    pa.storage = params.storage;
    pa.pass = pd_pass_iters(lc.g, params.pass_iters, params.storage);
    return pa;
}

// Whole method (Algorithm 1 in the pyramid of Sec. IV-B after the
// pre-rotation of Sec. IV-A, then the triangulation of Sec. III-D).
// Copies level l of one state plane of a probed pair to dst (level-stacked
// planes at the level's offset, single-level planes from their start).
static vfs_status probe_copy(void* dst, const Probe& pr, const Geometry& g, int l, size_t at, bool stacked,
                             size_t esz, hipStream_t s)
{
    if (!dst) return VFS_OK;
    const char* src = pr.region + at + (stacked ? size_t(g.off[l]) * esz : 0);
    if (hipMemcpy2DAsync(dst, pr.req.pitch * esz, src, size_t(g.pitch[l]) * esz, size_t(g.W[l]) * esz, g.H[l],
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(VFS_E_DEVICE, "probe copy failed");
    return VFS_OK;
}

vfs_status solve_slots(const Slot* slots, int n, const Geometry& g, const vfs_params& params, hipStream_t s,
                       vfs_rig* prof, const Probe* pr)
{
    const int L = g.L;
    const bool tgv = params.reg == VFS_TGV;
    const int st = params.storage;
    const int xform = params.data_term;   // 0: the intensities themselves
    Launch lc{};
    lc.slots = slots;
    lc.n = n;
    lc.g = g;
    auto at = [&](int l) {
        lc.lev = l;
        lc.gl = l;
    };
    // A1, A2: level 0 of the pyramids (pre-rotation), then levels 1 .. L-1
    at(0);
    launch_prerotate(lc, s);
    for (int l = 1; l < L; ++l) {
        at(l);
        launch_downsample(lc, s);
    }
    const Sched sc = schedule(params);
    for (int l = L - 1; l >= 0; --l) {
        at(l);
        // A3: tensor of the level (Eq. (12)); A7: state of the level
        launch_tensor(lc, st, s);
        if (xform) launch_transform(lc, xform, s);
        if (l == L - 1) launch_zero_state(lc, tgv ? 1 : 0, st, s);
        else launch_upsample(lc, tgv ? 1 : 0, st, s);
        for (int wv = 0; wv <= params.warps; ++wv) {
            // A4 (+A6 of the previous warp): clip, accumulate, linearise
            const bool last = wv == params.warps;
            if (last && wv == 0) break;
            launch_linearise(lc, wv > 0 ? 1 : 0, last ? 1 : 0, float(params.du_max), xform != 0, st, s);
            if (pr && l == pr->req.level && wv == pr->req.warp) {
                // the warp's start: linearised, duals warm-started
                const PairLayout& y = pr->lay;
                const vfs_probe& q = pr->req;
                const size_t e2 = st == ST_F32 ? 8 : 4, e4 = st == ST_F32 ? 16 : 8;
                vfs_status e = VFS_OK;
                if (!e) e = probe_copy(q.J0, *pr, g, l, y.J0, true, 4, s);
                if (!e) e = probe_copy(q.J1, *pr, g, l, y.J1, true, 4, s);
                if (!e) e = probe_copy(q.u, *pr, g, l, y.u[lc.iu], true, 4, s);
                if (!e) e = probe_copy(q.w, *pr, g, l, y.w, true, 8, s);
                if (!e && tgv) e = probe_copy(q.v, *pr, g, l, y.v[lc.iu], true, 8, s);
                if (!e) e = probe_copy(q.p, *pr, g, l, y.p[lc.ip], true, e2, s);
                if (!e && tgv) e = probe_copy(q.q, *pr, g, l, y.q[lc.ip], true, e4, s);
                if (!e) e = probe_copy(q.tpack, *pr, g, l, y.tpack, false, e4, s);
                if (!e) e = probe_copy(q.rho, *pr, g, l, y.rho, false, 4, s);
                if (!e) e = probe_copy(q.gw, *pr, g, l, y.gw, false, 8, s);
                if (e) return e;
            }
            if (pr && l == pr->req.level && wv == pr->req.warp + 1) {
                // the warp's end: clipped and accumulated (by this launch)
                vfs_status e = probe_copy(pr->req.u_next, *pr, g, l, pr->lay.u[lc.iu], true, 4, s);
                if (!e) e = probe_copy(pr->req.w_next, *pr, g, l, pr->lay.w, true, 8, s);
                if (!e && hipGetLastError() != hipSuccess) e = fail(VFS_E_DEVICE, "kernel launch failed");
                return e;
            }
            if (last) break;
            // A5: K primal-dual iterations (Eq. (11))
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (prof && prof->profile && l == 0 && params.iters >= 3) {
                if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                    return fail(VFS_E_DEVICE, "hipEventCreate");
                prof->events.emplace_back(e0, e1);
            }
            int iu, ip;
            const int np = run_pd(pd_args(lc, params), sc, params.iters, iu, ip, s, e0, e1);
            lc.iu = iu;
            lc.ip = ip;
            if (e0) prof->launches += np;
            if (pr && l == pr->req.level && wv == pr->req.warp) {
                // after the iterations, before the clip
                const PairLayout& y = pr->lay;
                const vfs_probe& q = pr->req;
                const size_t e2 = st == ST_F32 ? 8 : 4, e4 = st == ST_F32 ? 16 : 8;
                vfs_status e = probe_copy(q.u_pd, *pr, g, l, y.u[iu], true, 4, s);
                if (!e && tgv) e = probe_copy(q.v_pd, *pr, g, l, y.v[iu], true, 8, s);
                if (!e) e = probe_copy(q.p_pd, *pr, g, l, y.p[ip], true, e2, s);
                if (!e && tgv) e = probe_copy(q.q_pd, *pr, g, l, y.q[ip], true, e4, s);
                if (e) return e;
            }
        }
    }
    // A8: triangulation and outputs
    at(0);
    launch_triangulate(lc, s);
    if (hipGetLastError() != hipSuccess) return fail(VFS_E_DEVICE, "kernel launch failed");
    return VFS_OK;
}

}  // namespace vfs

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
    out->pass_iters = 0;
    out->data_term = VFS_DATA_BRIGHTNESS;
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
    r->g = make_geometry(cam0->width, cam0->height, levels);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto cleanup = [&](vfs_status e) { delete r; return e; };
    if (hipGetDevice(&r->device) != hipSuccess) return cleanup(fail(VFS_E_DEVICE, "hipGetDevice failed"));
    prepare_pd();
    // camera 0 and the baseline in single precision for the triangulation,
    // with the radial table of its back-projection computed here in double
    // precision (once per rig)
    TriGeom& tg = g.tri;
    tg.model = g.cam0.model;
    tg.fx = float(g.cam0.fx);
    tg.fy = float(g.cam0.fy);
    tg.cx = float(g.cam0.cx);
    tg.cy = float(g.cam0.cy);
    tg.th_lim = float(g.cam0.th_lim);
    tg.dtheta = float(g.cam0.th_lim / kRadial);
    for (int a = 0; a < 3; ++a) tg.C[a] = float(g.C[a]);
    std::vector<float2> table(kRadial + 1);
    const double dth = g.cam0.th_lim / kRadial;
    for (int k = 0; k <= kRadial; ++k)
        table[k] = make_float2(float(cam_rd(g.cam0, k * dth)), float(dth * cam_drd(g.cam0, k * dth)));
    if (hipMalloc(&r->radial, table.size() * sizeof(float2)) != hipSuccess)
        return cleanup(fail(VFS_E_NOMEM, "radial table"));
    if (hipMemcpy(r->radial, table.data(), table.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(VFS_E_DEVICE, "copying the radial table"));
    tg.radial = r->radial;
    if (hipMalloc(&r->geom_dev, sizeof(RigGeom)) != hipSuccess) return cleanup(fail(VFS_E_NOMEM, "rig geometry"));
    if (hipMemcpyAsync(r->geom_dev, &g, sizeof(RigGeom), hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(fail(VFS_E_DEVICE, "copying rig geometry"));
    for (int l = 0; l < levels; ++l) {
        const size_t plane = plane_elems(r->g, l);
        if (hipMalloc(&r->gamma[l], plane * sizeof(float2)) != hipSuccess || hipMalloc(&r->flags[l], plane) != hipSuccess)
            return cleanup(fail(VFS_E_NOMEM, "rig fields"));
        if (hipMemsetAsync(r->gamma[l], 0, plane * sizeof(float2), s) != hipSuccess ||
            hipMemsetAsync(r->flags[l], 0, plane, s) != hipSuccess)
            return cleanup(fail(VFS_E_DEVICE, "clearing rig fields"));
        launch_level_fields(g, l, r->gamma[l], r->flags[l], r->g.pitch[l], s);
    }
    if (hipMalloc(&r->calib, plane_elems(r->g, 0) * sizeof(float2)) != hipSuccess)
        return cleanup(fail(VFS_E_NOMEM, "calibration field"));
    launch_calibration(g, r->calib, r->g.pitch[0], s);
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
    if (level < 0 || level >= r->g.L) return fail(VFS_E_INVALID, "level out of range");
    if (which < 0 || which > 2 || (which == 1 && level != 0)) return fail(VFS_E_INVALID, "bad field");
    const int W = r->g.W[level], H = r->g.H[level], pitch = r->g.pitch[level];
    const size_t esz = which == 2 ? 1 : sizeof(float2);
    if (pitch_bytes < esz * W) return fail(VFS_E_INVALID, "pitch too small");
    const void* src = which == 0 ? (const void*)r->gamma[level] : which == 1 ? (const void*)r->calib
                                                                            : (const void*)r->flags[level];
    HIP_OK(hipMemcpy2DAsync(dst, pitch_bytes, src, esz * pitch, esz * W, H, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(hip_stream)));
    return VFS_OK;
}

}  // extern "C"

namespace vfs {

vfs_status check_batch(const vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                       float* const* u_out, float* const* w_out, float* const* depth_out, const vfs_params* params,
                       const double* betas, const double* etas, bool outputs)
{
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    if (n < 1 || n > kMaxBatch) return fail(VFS_E_INVALID, "n must be in [1, %d]", kMaxBatch);
    vfs_status st = check_params(params);
    if (st) return st;
    if (params->levels != r->g.L)
        return fail(VFS_E_INVALID, "params->levels (%d) differs from the rig's (%d)", params->levels, r->g.L);
    const int W = r->g.W[0];
    if (pitch_bytes % sizeof(float) || pitch_bytes < sizeof(float) * W) return fail(VFS_E_INVALID, "bad pitch");
    if (!I0 || !I1 || (outputs && (!u_out || !w_out || !depth_out))) return fail(VFS_E_INVALID, "NULL array argument");
    for (int b = 0; b < n; ++b) {
        if (!I0[b] || !I1[b] || (outputs && (!u_out[b] || !w_out[b] || !depth_out[b])))
            return fail(VFS_E_INVALID, "NULL buffer for pair %d", b);
        if ((betas && !(betas[b] >= 0.0)) || (etas && !(etas[b] > 0.0)))
            return fail(VFS_E_INVALID, "bad tensor parameters for pair %d", b);
    }
    return VFS_OK;
}

void write_batch_slots(const vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                       float* const* u_out, float* const* w_out, float* const* depth_out, float* const* z_out,
                       uint8_t* const* valid_out, const vfs_params* params, const double* betas,
                       const double* etas, bool outputs, char* state, const PairLayout& lay, Slot* slots,
                       hipStream_t s)
{
    const int ip = int(pitch_bytes / sizeof(float));
    for (int b = 0; b < n; ++b) {
        Slot sl{};
        sl.I0 = I0[b];
        sl.I1 = I1[b];
        sl.in_pitch = ip;
        sl.out_pitch = ip;
        sl.u_out = outputs ? u_out[b] : nullptr;
        sl.w_out = outputs ? w_out[b] : nullptr;
        sl.depth_out = outputs ? depth_out[b] : nullptr;
        sl.z_out = outputs && z_out ? z_out[b] : nullptr;
        sl.valid_out = outputs && valid_out ? valid_out[b] : nullptr;
        bind_rig(sl, r);
        bind_state(sl, state + size_t(b) * lay.bytes, lay);
        sl.beta = float(betas ? betas[b] : params->beta);
        sl.eta = float(etas ? etas[b] : params->eta);
        launch_write_slot(sl, slots + b, s);
    }
}

}  // namespace vfs

namespace {

// Validates a batched solve's arguments, sizes the rig's workspace and
// writes the pairs' descriptors (outputs may be NULL arrays: a probe).
vfs_status prepare_batch(vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                         float* const* u_out, float* const* w_out, float* const* depth_out, float* const* z_out,
                         uint8_t* const* valid_out, const vfs_params* params, const double* betas,
                         const double* etas, bool outputs, hipStream_t s)
{
    vfs_status st = check_batch(r, n, I0, I1, pitch_bytes, u_out, w_out, depth_out, params, betas, etas, outputs);
    if (st) return st;
    st = ensure_workspace(r->ws, r->g, n, params->storage, params->reg == VFS_TGV,
                          params->data_term != VFS_DATA_BRIGHTNESS);
    if (st) return st;
    r->last_stream = s;
    write_batch_slots(r, n, I0, I1, pitch_bytes, u_out, w_out, depth_out, z_out, valid_out, params, betas, etas,
                      outputs, static_cast<char*>(r->ws.mem), r->ws.lay, r->ws.slots, s);
    r->pass_iters = pd_pass_iters(r->g, params->pass_iters, params->storage);
    return VFS_OK;
}

// Solver parameters that change a solve's launches (beta and eta travel in
// the pair descriptors).
bool same_launches(const vfs_params& a, const vfs_params& b)
{
    return a.levels == b.levels && a.warps == b.warps && a.iters == b.iters && a.reg == b.reg &&
           a.lambda == b.lambda && a.alpha0 == b.alpha0 && a.alpha1 == b.alpha1 && a.du_max == b.du_max &&
           a.theta_gamma == b.theta_gamma && a.storage == b.storage && a.pass_iters == b.pass_iters &&
           a.data_term == b.data_term;
}

constexpr size_t kMaxGraphs = 8;

void drop_graphs(vfs_rig* r)
{
    for (auto& gr : r->graphs) {
        (void)hipGraphExecDestroy(gr.exec);
        (void)hipGraphDestroy(gr.graph);
    }
    r->graphs.clear();
}

// The whole method on the rig's workspace as one graph launch on s: the
// launches of solve_slots are captured (on a stream of the rig's) the first
// time a launch configuration occurs and replayed after.  The pair
// descriptors, written on s before this, carry the images, outputs and
// tensor parameters, so one graph serves any inputs of that configuration.
vfs_status solve_graph(vfs_rig* r, int n, const vfs_params& p, hipStream_t s)
{
    vfs_rig::SolveGraph* hit = nullptr;
    for (auto& gr : r->graphs)
        if (gr.n == n && gr.mem == r->ws.mem && gr.slots == r->ws.slots && same_launches(gr.params, p)) hit = &gr;
    if (!hit) {
        if (r->graphs.size() >= kMaxGraphs) drop_graphs(r);
        if (!r->capture_stream && hipStreamCreateWithFlags(&r->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(VFS_E_DEVICE, "hipStreamCreate");
        vfs_rig::SolveGraph gr{};
        gr.params = p;
        gr.n = n;
        gr.mem = r->ws.mem;
        gr.slots = r->ws.slots;
        if (hipStreamBeginCapture(r->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(VFS_E_DEVICE, "hipStreamBeginCapture");
        const vfs_status st = solve_slots(r->ws.slots, n, r->g, p, r->capture_stream, nullptr);
        const hipError_t ec = hipStreamEndCapture(r->capture_stream, &gr.graph);
        if (st || ec != hipSuccess) {
            if (ec == hipSuccess) (void)hipGraphDestroy(gr.graph);
            return st ? st : fail(VFS_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        }
        if (hipGraphInstantiateWithFlags(&gr.exec, gr.graph, 0) != hipSuccess) {
            (void)hipGraphDestroy(gr.graph);
            return fail(VFS_E_DEVICE, "hipGraphInstantiate");
        }
        r->graphs.push_back(gr);
        hit = &r->graphs.back();
    }
    HIP_OK(hipGraphLaunch(hit->exec, s));
    return VFS_OK;
}

}  // namespace

extern "C" {

vfs_status vfs_rig_graphs(vfs_rig* r, int enable)
{
    g_err[0] = 0;
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    r->use_graphs = enable != 0;
    if (!r->use_graphs) drop_graphs(r);
    return VFS_OK;
}

vfs_status vfs_solve_batch(vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                           float* const* u_out, float* const* w_out, float* const* depth_out, float* const* z_out,
                           uint8_t* const* valid_out, const vfs_params* params, const double* betas,
                           const double* etas, void* hip_stream)
{
    g_err[0] = 0;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs_status st = prepare_batch(r, n, I0, I1, pitch_bytes, u_out, w_out, depth_out, z_out, valid_out, params,
                                  betas, etas, true, s);
    if (st) return st;
    if (r->use_graphs && !r->profile) return solve_graph(r, n, *params, s);
    return solve_slots(r->ws.slots, n, r->g, *params, s, r);
}

vfs_status vfs_solve_probe(vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                           const vfs_params* params, const double* betas, const double* etas, const vfs_probe* probe,
                           void* hip_stream)
{
    g_err[0] = 0;
    if (!r || !params || !probe) return fail(VFS_E_INVALID, "NULL argument");
    if (probe->level < 0 || probe->level >= r->g.L || probe->level >= params->levels)
        return fail(VFS_E_INVALID, "probe level out of range");
    if (probe->warp < 0 || probe->warp >= params->warps) return fail(VFS_E_INVALID, "probe warp out of range");
    if (probe->pair < 0 || probe->pair >= n) return fail(VFS_E_INVALID, "probe pair out of range");
    if (probe->pitch < size_t(r->g.W[probe->level])) return fail(VFS_E_INVALID, "probe pitch too small");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs_status st = prepare_batch(r, n, I0, I1, pitch_bytes, nullptr, nullptr, nullptr, nullptr, nullptr, params,
                                  betas, etas, false, s);
    if (st) return st;
    Probe pr{};
    pr.req = *probe;
    pr.lay = r->ws.lay;
    pr.region = static_cast<const char*>(r->ws.mem) + size_t(probe->pair) * r->ws.lay.bytes;
    st = solve_slots(r->ws.slots, n, r->g, *params, s, nullptr, &pr);
    if (st) return st;
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_solve(vfs_rig* rig, const float* I0, const float* I1, size_t pitch_bytes, float* u_out, float* w_out,
                     float* depth_out, float* z_out, uint8_t* valid_out, const vfs_params* params, void* hip_stream)
{
    return vfs_solve_batch(rig, 1, &I0, &I1, pitch_bytes, &u_out, &w_out, &depth_out, z_out ? &z_out : nullptr,
                           valid_out ? &valid_out : nullptr, params, nullptr, nullptr, hip_stream);
}

// ---------------------------------------------------------------- step entry points
// Test hooks: each builds a one-pair descriptor over the caller's planes (one
// level, the caller's pitch), runs the step and waits for it.

namespace {

struct OneSlot {
    Slot* dev = nullptr;
    ~OneSlot()
    {
        if (dev) (void)hipFree(dev);
    }
};

Geometry one_level(int W, int H, size_t pitch)
{
    Geometry g{};
    g.L = 1;
    g.W[0] = W;
    g.H[0] = H;
    g.pitch[0] = int(pitch);
    g.off[0] = 0;
    return g;
}

vfs_status run_one(OneSlot& os, const Slot& sl, hipStream_t s)
{
    HIP_OK(hipMalloc(&os.dev, sizeof(Slot)));
    launch_write_slot(sl, os.dev, s);
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

Launch one_launch(const OneSlot& os, const Geometry& g)
{
    Launch lc{};
    lc.slots = os.dev;
    lc.n = 1;
    lc.g = g;
    return lc;
}

}  // namespace

vfs_status vfs_step_tensor(int W, int H, size_t pitch, const float* J0, const uint8_t* flags, double beta, double eta,
                           float* tpack, void* hip_stream)
{
    g_err[0] = 0;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !J0 || !flags || !tpack || !(beta >= 0.0) || !(eta > 0.0))
        return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Slot sl{};
    sl.J0 = const_cast<float*>(J0);
    sl.flags[0] = flags;
    sl.beta = float(beta);
    sl.eta = float(eta);
    sl.tpack = tpack;
    OneSlot os;
    vfs_status st = run_one(os, sl, s);
    if (st) return st;
    launch_tensor(one_launch(os, one_level(W, H, pitch)), ST_F32, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_step_rank(int W, int H, size_t pitch, const float* I0, const float* I1, float* R0, float* R1,
                         void* hip_stream)
{
    g_err[0] = 0;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !I0 || !I1 || !R0 || !R1) return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Slot sl{};
    sl.J0 = const_cast<float*>(I0);
    sl.J1 = const_cast<float*>(I1);
    sl.R0 = R0;
    sl.R1 = R1;
    OneSlot os;
    vfs_status st = run_one(os, sl, s);
    if (st) return st;
    launch_transform(one_launch(os, one_level(W, H, pitch)), VFS_DATA_RANK, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_step_gradient(int W, int H, size_t pitch, const float* I0, const float* I1, float* G0, float* G1,
                             void* hip_stream)
{
    g_err[0] = 0;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !I0 || !I1 || !G0 || !G1) return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Slot sl{};
    sl.J0 = const_cast<float*>(I0);
    sl.J1 = const_cast<float*>(I1);
    sl.R0 = G0;
    sl.R1 = G1;
    OneSlot os;
    vfs_status st = run_one(os, sl, s);
    if (st) return st;
    launch_transform(one_launch(os, one_level(W, H, pitch)), VFS_DATA_GRADIENT, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
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
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Slot sl{};
    sl.J0 = const_cast<float*>(J0);
    sl.J1 = const_cast<float*>(J1);
    sl.gamma[0] = reinterpret_cast<const float2*>(gamma);
    sl.flags[0] = flags;
    sl.u[0] = u;
    sl.uw = u_w;
    sl.w = reinterpret_cast<float2*>(w);
    sl.gw = reinterpret_cast<float2*>(gamma_w);
    sl.tpack = tpack;
    sl.rho = rho;
    OneSlot os;
    vfs_status st = run_one(os, sl, s);
    if (st) return st;
    launch_linearise(one_launch(os, one_level(W, H, pitch)), clip ? 1 : 0, clip_only ? 1 : 0, float(du_max), 0,
                     ST_F32, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_step_pd(int W, int H, size_t pitch, const void* tpack, const float* rho, const uint8_t* flags, float* u,
                       float* v, void* p, void* q, float* su, float* sv, void* sp, void* sq,
                       const vfs_params* params, int iters, void* hip_stream)
{
    g_err[0] = 0;
    vfs_status st = check_params(params);
    if (st) return st;
    const bool tgv = params->reg == VFS_TGV;
    if (W <= 0 || H <= 0 || W > kMaxWidth || pitch < size_t(W) || !tpack || !rho || !flags || !u || !p || !su || !sp ||
        iters < 0 || (tgv && (!v || !q || !sv || !sq)))
        return fail(VFS_E_INVALID, "bad argument");
    if (iters == 0) return VFS_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs_params pp = *params;
    pp.iters = iters;
    const Sched sc = schedule(pp);
    Slot sl{};
    sl.tpack = const_cast<void*>(tpack);
    sl.rho = const_cast<float*>(rho);
    sl.flags[0] = flags;
    sl.u[0] = u;
    sl.u[1] = su;
    sl.v[0] = reinterpret_cast<float2*>(v);
    sl.v[1] = reinterpret_cast<float2*>(sv);
    sl.p[0] = p;
    sl.p[1] = sp;
    sl.q[0] = q;
    sl.q[1] = sq;
    OneSlot os;
    st = run_one(os, sl, s);
    if (st) return st;
    int iu, ip;
    run_pd(pd_args(one_launch(os, one_level(W, H, pitch)), pp), sc, iters, iu, ip, s, nullptr, nullptr);
    const size_t plane = pitch * size_t(H);
    const size_t e2 = pp.storage == VFS_F32 ? 8 : 4, e4 = pp.storage == VFS_F32 ? 16 : 8;
    if (iu) {
        HIP_OK(hipMemcpyAsync(u, su, plane * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (tgv) HIP_OK(hipMemcpyAsync(v, sv, plane * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    if (ip) {
        HIP_OK(hipMemcpyAsync(p, sp, plane * e2, hipMemcpyDeviceToDevice, s));
        if (tgv) HIP_OK(hipMemcpyAsync(q, sq, plane * e4, hipMemcpyDeviceToDevice, s));
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_step_upsample(int Wc, int Hc, size_t pitch_c, const uint8_t* flags_c, const float* u_c, const float* w_c,
                             size_t pitch_f, float* u_f, float* w_f, void* hip_stream)
{
    g_err[0] = 0;
    if (Wc <= 0 || Hc <= 0 || pitch_c < size_t(Wc) || pitch_f < size_t(2 * Wc) || !flags_c || !u_c || !w_c || !u_f ||
        !w_f)
        return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // two-level stack: fine plane (the caller's pitch) then the coarse one
    Geometry g{};
    g.L = 2;
    g.W[0] = 2 * Wc; g.H[0] = 2 * Hc; g.pitch[0] = int(pitch_f); g.off[0] = 0;
    g.W[1] = Wc; g.H[1] = Hc; g.pitch[1] = int(pitch_c); g.off[1] = (long long)pitch_f * 2 * Hc;
    const size_t elems = size_t(g.off[1]) + pitch_c * size_t(Hc);
    struct Bufs {
        float* u = nullptr;
        float2* w = nullptr;
        ~Bufs()
        {
            if (u) (void)hipFree(u);
            if (w) (void)hipFree(w);
        }
    } b;
    HIP_OK(hipMalloc(&b.u, elems * sizeof(float)));
    HIP_OK(hipMalloc(&b.w, elems * sizeof(float2)));
    HIP_OK(hipMemcpyAsync(b.u + g.off[1], u_c, pitch_c * Hc * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(b.w + g.off[1], w_c, pitch_c * Hc * sizeof(float2), hipMemcpyDeviceToDevice, s));
    Slot sl{};
    sl.flags[1] = flags_c;
    sl.u[0] = b.u;
    sl.w = b.w;
    OneSlot os;
    vfs_status st = run_one(os, sl, s);
    if (st) return st;
    Launch lc = one_launch(os, g);
    launch_upsample(lc, 0, ST_F32, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(u_f, b.u, pitch_f * 2 * Hc * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(w_f, b.w, pitch_f * 2 * Hc * sizeof(float2), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_step_triangulate(const vfs_rig* r, size_t pitch, const float* w, float* depth, float* z, uint8_t* valid,
                                void* hip_stream)
{
    g_err[0] = 0;
    if (!r || !w || !depth) return fail(VFS_E_INVALID, "NULL argument");
    const int W = r->g.W[0], H = r->g.H[0], rp = r->g.pitch[0];
    if (pitch < size_t(W)) return fail(VFS_E_INVALID, "pitch too small");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float2* ww = nullptr;
    HIP_OK(hipMalloc(&ww, size_t(rp) * H * sizeof(float2)));
    struct Free {
        void* p;
        ~Free() { (void)hipFree(p); }
    } fw{ww};
    HIP_OK(hipMemcpy2DAsync(ww, rp * sizeof(float2), w, pitch * sizeof(float2), W * sizeof(float2), H,
                            hipMemcpyDeviceToDevice, s));
    Slot sl{};
    bind_rig(sl, r);
    sl.w = ww;
    sl.out_pitch = int(pitch);
    sl.depth_out = depth;
    sl.z_out = z;
    sl.valid_out = valid;
    OneSlot os;
    vfs_status st = run_one(os, sl, s);
    if (st) return st;
    launch_triangulate(one_launch(os, r->g), s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

// ---------------------------------------------------------------- energy and difference statistics

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

EnergyConsts energy_consts(const vfs_params& p)
{
    EnergyConsts k{};
    k.lambda = float(p.lambda);
    k.alpha0 = float(p.alpha0);
    k.alpha1 = float(p.alpha1);
    k.tgv = p.reg == VFS_TGV ? 1 : 0;
    k.storage = ST_F32;
    return k;
}

}  // namespace

vfs_status vfs_step_energy(int W, int H, size_t pitch, const float* tpack, const float* rho, const uint8_t* flags,
                           const float* u, const float* v, const vfs_params* params, double* energy,
                           void* hip_stream)
{
    g_err[0] = 0;
    vfs_status st = check_params(params);
    if (st) return st;
    const bool tgv = params->reg == VFS_TGV;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !tpack || !rho || !flags || !u || (tgv && !v) || !energy)
        return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Slot sl{};
    sl.tpack = const_cast<float*>(tpack);
    sl.rho = const_cast<float*>(rho);
    sl.flags[0] = flags;
    sl.u[0] = const_cast<float*>(u);
    sl.v[0] = reinterpret_cast<float2*>(const_cast<float*>(v));
    OneSlot os;
    st = run_one(os, sl, s);
    if (st) return st;
    Launch lc = one_launch(os, one_level(W, H, pitch));
    DevBuf part;
    HIP_OK(hipMalloc(&part.p, (energy_partials(lc) + 1) * sizeof(double)));
    double* d = static_cast<double*>(part.p);
    launch_energy(lc, energy_consts(*params), d + 1, d, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(energy, d, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_step_pd_energy(int W, int H, size_t pitch, const float* tpack, const float* rho, const uint8_t* flags,
                              float* u, float* v, float* p, float* q, float* su, float* sv, float* sp, float* sq,
                              const vfs_params* params, int iters, double* energy, void* hip_stream)
{
    g_err[0] = 0;
    vfs_status st = check_params(params);
    if (st) return st;
    const bool tgv = params->reg == VFS_TGV;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !tpack || !rho || !flags || !u || !p || !su || !sp || iters < 1 ||
        !energy || (tgv && (!v || !q || !sv || !sq)))
        return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs_params pp = *params;
    pp.iters = iters;
    pp.storage = VFS_F32;
    const Sched sc = schedule(pp);
    Slot sl{};
    sl.tpack = const_cast<float*>(tpack);
    sl.rho = const_cast<float*>(rho);
    sl.flags[0] = flags;
    sl.u[0] = u;
    sl.u[1] = su;
    sl.v[0] = reinterpret_cast<float2*>(v);
    sl.v[1] = reinterpret_cast<float2*>(sv);
    sl.p[0] = p;
    sl.p[1] = sp;
    sl.q[0] = q;
    sl.q[1] = sq;
    OneSlot os;
    st = run_one(os, sl, s);
    if (st) return st;
    Launch lc = one_launch(os, one_level(W, H, pitch));
    const size_t np = energy_partials(lc);
    DevBuf buf;
    HIP_OK(hipMalloc(&buf.p, (np + iters + 1) * sizeof(double)));
    double* e = static_cast<double*>(buf.p);
    double* part = e + iters + 1;
    const EnergyConsts ek = energy_consts(pp);
    // the energy of x^0, then one iteration per launch with the energy of
    // each new primal iterate x^k (the memory holds (x^k, y^{k+1}) between
    // launches)
    int iu = 0, ip = 0;
    auto energy_at = [&](int k) {
        lc.iu = iu;
        launch_energy(lc, ek, part, e + k, s);
    };
    energy_at(0);
    PdArgs a = pd_args(lc, pp);
    a.mode = PD_DUAL_FIRST;
    a.tau_scale = 1.f;
    a.sigma_scale = 1.f / sc.s[0];
    a.theta = 1.f;
    a.lc.iu = iu;
    a.lc.ip = ip;
    launch_pd(a, s);
    ip ^= 1;
    for (int k = 1; k < iters; ++k) {
        a.mode = PD_FUSED;
        a.tau_scale = sc.s[k - 1];
        a.theta = sc.theta[k - 1];
        a.sigma_scale = 1.f / sc.s[k];
        a.lc.iu = iu;
        a.lc.ip = ip;
        launch_pd(a, s);
        iu ^= 1;
        ip ^= 1;
        energy_at(k);
    }
    a.mode = PD_PRIMAL_LAST;
    a.tau_scale = sc.s[iters - 1];
    a.sigma_scale = 1.f;
    a.theta = 1.f;
    a.lc.iu = iu;
    a.lc.ip = ip;
    launch_pd(a, s);
    iu ^= 1;
    energy_at(iters);
    HIP_OK(hipGetLastError());
    const size_t plane = pitch * size_t(H);
    if (iu) {
        HIP_OK(hipMemcpyAsync(u, su, plane * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (tgv) HIP_OK(hipMemcpyAsync(v, sv, plane * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    if (ip) {
        HIP_OK(hipMemcpyAsync(p, sp, plane * sizeof(float2), hipMemcpyDeviceToDevice, s));
        if (tgv) HIP_OK(hipMemcpyAsync(q, sq, plane * sizeof(float4), hipMemcpyDeviceToDevice, s));
    }
    HIP_OK(hipMemcpyAsync(energy, e, (iters + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return VFS_OK;
}

vfs_status vfs_diff_stats(int W, int H, size_t pitch, const float* a, const float* b, const uint8_t* flags,
                          double* mean_abs, double* max_abs, long long* count, void* hip_stream)
{
    g_err[0] = 0;
    if (W <= 0 || H <= 0 || pitch < size_t(W) || !a || !b) return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n = diff_partials(W, H);
    DevBuf buf;
    HIP_OK(hipMalloc(&buf.p, (3 * n + 3) * sizeof(double)));
    double* out = static_cast<double*>(buf.p);
    launch_diff_stats(W, H, int(pitch), a, b, flags, out + 3, out, s);
    HIP_OK(hipGetLastError());
    double h[3];
    HIP_OK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (count) *count = (long long)h[2];
    if (mean_abs) *mean_abs = h[2] > 0 ? h[0] / h[2] : 0.0;
    if (max_abs) *max_abs = h[1];
    return VFS_OK;
}

vfs_status vfs_profile_enable(vfs_rig* r, int enable)
{
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    r->profile = enable != 0;
    return VFS_OK;
}

vfs_status vfs_profile_read(vfs_rig* r, double* ms, long long* launches, int* iters_per_launch, int reset)
{
    g_err[0] = 0;
    if (!r) return fail(VFS_E_INVALID, "rig is NULL");
    if (iters_per_launch) *iters_per_launch = r->pass_iters;
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

vfs_status vfs_rectify_rotations(const double R[9], const double t[3], double Rv0[9], double Rv1[9], double* baseline)
{
    g_err[0] = 0;
    if (!R || !t || !Rv0 || !Rv1) return fail(VFS_E_INVALID, "bad argument");
    // baseline direction t' = R^T t in camera 0's frame, and the mean of the two optical axes
    double ex[3], a[3];
    for (int k = 0; k < 3; ++k) {
        ex[k] = R[k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2];
        a[k] = (k == 2 ? 1.0 : 0.0) + R[6 + k];
    }
    const double b = sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2]);
    if (!(b > 0.0)) return fail(VFS_E_INVALID, "zero translation");
    for (double& v : ex) v /= b;
    double ey[3] = {a[1] * ex[2] - a[2] * ex[1], a[2] * ex[0] - a[0] * ex[2], a[0] * ex[1] - a[1] * ex[0]};
    const double ny = sqrt(ey[0] * ey[0] + ey[1] * ey[1] + ey[2] * ey[2]);
    if (!(ny > 1e-9)) return fail(VFS_E_MODEL, "baseline along the viewing direction: no side-by-side view");
    for (double& v : ey) v /= ny;
    const double ez[3] = {ex[1] * ey[2] - ex[2] * ey[1], ex[2] * ey[0] - ex[0] * ey[2], ex[0] * ey[1] - ex[1] * ey[0]};
    for (int k = 0; k < 3; ++k) {
        Rv0[k] = ex[k];
        Rv0[3 + k] = ey[k];
        Rv0[6 + k] = ez[k];
    }
    // Rv1 = Rv0 R^T: camera 1's frame to the shared virtual orientation
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Rv1[3 * r + c] = Rv0[3 * r] * R[3 * c] + Rv0[3 * r + 1] * R[3 * c + 1] + Rv0[3 * r + 2] * R[3 * c + 2];
    if (baseline) *baseline = b;
    return VFS_OK;
}

namespace {

vfs_status rectify_geom(const vfs_camera* cam, const double Rv[9], const vfs_camera* pin, vfs::RectifyGeom& g)
{
    if (vfs_status st = check_camera(cam, "cam")) return st;
    if (vfs_status st = check_camera(pin, "pinhole")) return st;
    if (pin->model != VFS_PINHOLE) return fail(VFS_E_INVALID, "the virtual view must be a pinhole camera");
    if (!Rv) return fail(VFS_E_INVALID, "Rv is NULL");
    g.cam = to_cam(*cam);
    g.pin = to_cam(*pin);
    for (int k = 0; k < 9; ++k) g.Rv[k] = Rv[k];
    g.half = 0.5 * cam->fov_deg * kPi / 180.0;
    g.rmax = vfs::cam_rd(g.cam, g.half);
    return VFS_OK;
}

}  // namespace

vfs_status vfs_rectify(const vfs_camera* cam, const double Rv[9], const vfs_camera* pinhole, const float* src,
                       size_t src_pitch, float* dst, size_t dst_pitch, uint8_t* valid, void* hip_stream)
{
    g_err[0] = 0;
    vfs::RectifyGeom g{};
    if (vfs_status st = rectify_geom(cam, Rv, pinhole, g)) return st;
    if (!src || !dst || src_pitch < size_t(cam->width) || dst_pitch < size_t(pinhole->width))
        return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs::launch_rectify(g, src, src_pitch, dst, dst_pitch, valid, s);
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

vfs_status vfs_unrectify(const vfs_camera* cam, const double Rv[9], const vfs_camera* pinhole, const float* field,
                         const uint8_t* field_valid, size_t field_pitch, float* dst, size_t dst_pitch, uint8_t* valid,
                         void* hip_stream)
{
    g_err[0] = 0;
    vfs::RectifyGeom g{};
    if (vfs_status st = rectify_geom(cam, Rv, pinhole, g)) return st;
    if (!field || !dst || field_pitch < size_t(pinhole->width) || dst_pitch < size_t(cam->width))
        return fail(VFS_E_INVALID, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    vfs::launch_unrectify(g, field, field_valid, field_pitch, dst, dst_pitch, valid, s);
    HIP_OK(hipGetLastError());
    return VFS_OK;
}

}  // extern "C"
