// Serving loop: stereo pairs of any registered rig arrive one by one and are
// solved by the whole method of the direct solves, batched on the device.
//
// Continuous batching.  Requests are grouped by image size (bucket: size and
// level count).  A bucket has up to max_slots slots; each admitted request
// owns a slot and a region of the HBM pool for its solve state.  The bucket
// advances all its requests one warp step at a time: one "tick" is one
// replay of a captured graph that, for every slot, runs the stages that slot
// needs at its own level and warp (start: pre-rotation, pyramids, zero state;
// level change: final accumulate of the coarser level and transfer; tensor;
// warp: linearise + K primal-dual iterations; finish: final accumulate and
// triangulation).  Between replays the host writes the slot table (new
// requests) and the per-slot control words (level, warp, stage bits,
// parity); a request admitted while others are mid-solve joins at the next
// tick.  Buckets run on their own streams, so their ticks overlap.  Every
// request's arithmetic is the direct solve's, pixel by pixel, in the same
// order, so results do not depend on the mix.
//
// Admission is by HBM budget: the per-request state comes from one pool of
// the budget's size; a request waits until its bucket has a free slot and
// the pool has room (arrival order; a full bucket does not hold up other
// sizes, a request the pool cannot hold yet holds up those behind it).
//
// The plain mode is the baseline: one request at a time, first come first
// served, with the eager launches of the direct solve.
#include <math.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "runtime.h"

using namespace vfs;

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t)
{
    return std::chrono::duration<double>(t - t0).count();
}

// First-fit allocator over [0, size) with coalescing (offsets, 256-byte units).
class Pool {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
        peak_ = 0;
    }
    bool alloc(size_t bytes, size_t& off)
    {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            if (used_ > peak_) peak_ = used_;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) / 256 * 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

enum ReqState { Q_WAIT = 0, Q_RUN = 1, Q_DONE = 2, Q_FAIL = 3 };

struct Request {
    unsigned long long ticket = 0;
    vfs_rig* rig = nullptr;
    Slot io{};                  // images, outputs, rig fields, beta / eta (state bound at admission)
    Clock::time_point t_arrive, t_admit, t_done;
    std::atomic<int> state{Q_WAIT};
    size_t mem_off = 0, mem_bytes = 0;
};

struct SlotState {
    Request* req = nullptr;     // NULL: free
    bool started = false;
    bool draining = false;      // finish enqueued, waiting for its tick to complete
    int level = 0, warp = 0;
    unsigned flip = 0;
};

struct Tick {
    hipEvent_t ev = nullptr;
    std::vector<int> finishing;     // slots whose request completes with this tick
};

// Launch sizes of a bucket's ticks: a tick's launches cover its active slots
// (their control words come first), rounded up to one of these sizes.
constexpr int kTickSizes = 6;    // 1, 2, 4, 8, 16, 32 (at most the bucket's slots)

struct Bucket {
    Geometry g{};
    PairLayout lay{};
    int S = 0;
    Slot* slots_dev = nullptr;
    Ctrl* ctrl_dev = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // graphs are captured here, launched on `stream`
    int sizes[kTickSizes] = {};
    int nsizes = 0;
    // [gl][0]: warp step only, [gl][1]: every stage; gl: the finest level
    // among the tick's slots (the warp step's grids cover that level);
    // [k]: launch size sizes[k]
    hipGraph_t graph[kMaxLevels][2][kTickSizes] = {};
    hipGraphExec_t exec[kMaxLevels][2][kTickSizes] = {};
    int par_u = 0, par_p = 0;       // parity change of one tick's primal-dual launches
    std::vector<SlotState> slot;
    std::deque<Tick> inflight;
    std::vector<hipEvent_t> spare_events;
    long long ticks = 0, full_ticks = 0;
};

bool same_geometry(const Geometry& a, const Geometry& b)
{
    if (a.L != b.L) return false;
    for (int l = 0; l < a.L; ++l)
        if (a.W[l] != b.W[l] || a.H[l] != b.H[l]) return false;
    return true;
}

}  // namespace

struct vfs_server {
    vfs_server_config cfg{};
    vfs_params params{};
    Sched sched;
    int device = 0;
    void* pool_mem = nullptr;
    Pool pool;

    std::mutex mu;                      // guards incoming, requests, error
    std::condition_variable cv;
    std::deque<Request*> incoming;
    std::unordered_map<unsigned long long, std::unique_ptr<Request>> requests;
    unsigned long long next_ticket = 1;
    std::atomic<long long> outstanding{0};
    std::atomic<bool> stop{false};
    vfs_status error = VFS_OK;
    char error_msg[256] = "";

    // scheduler-thread state
    std::deque<Request*> waiting;       // arrival order
    std::vector<std::unique_ptr<Bucket>> buckets;
    // plain mode
    hipStream_t plain_stream = nullptr;
    std::vector<std::unique_ptr<Workspace>> plain_ws;
    hipEvent_t plain_ev = nullptr;
    Request* plain_cur = nullptr;

    long long active = 0;               // scheduler thread only
    // counters written by the scheduler thread and read by vfs_server_stats
    std::atomic<long long> ticks{0}, peak_active{0}, joins{0}, full_ticks{0};
    std::atomic<size_t> pool_peak{0};
    std::atomic<int> nbuckets{0};
    std::thread worker;

    ~vfs_server();
};

namespace {

void set_error(vfs_server* sv, vfs_status st, const char* what)
{
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->error == VFS_OK) {
        sv->error = st;
        snprintf(sv->error_msg, sizeof(sv->error_msg), "%s", what);
    }
}

// One tick of a bucket: the stages every slot may need, selected per slot
// by its control word (see the comment at the top of this file).  Without
// `full`, only the warp step (for ticks where no slot starts, changes level
// or finishes).  The warp step's grids cover level gl, the finest level
// among the tick's slots; the launches cover n control words.
void enqueue_tick(vfs_server* sv, Bucket& b, hipStream_t s, bool full, int gl, int n, int& par_u, int& par_p)
{
    const vfs_params& P = sv->params;
    const bool tgv = P.reg == VFS_TGV;
    const int st = P.storage;
    const int xform = P.data_term;   // 0: the intensities themselves
    const int L = b.g.L;
    Launch lc{};
    lc.slots = b.slots_dev;
    lc.ctrl = b.ctrl_dev;
    lc.n = n;
    lc.tick = 1;
    lc.g = b.g;
    lc.lev = -1;
    if (full) {
        // start: pyramids of the new requests
        lc.op = OP_START;
        lc.lev = 0;
        lc.gl = 0;
        launch_prerotate(lc, s);
        for (int l = 1; l < L; ++l) {
            lc.lev = l;
            lc.gl = l;
            launch_downsample(lc, s);
        }
        lc.lev = -1;
        if (L > 1) {
            // level change: close level + 1, transfer to level
            lc.op = OP_NEWLEVEL;
            lc.dl = 1;
            lc.gl = gl + 1 < L ? gl + 1 : L - 1;
            launch_linearise(lc, 1, 1, float(P.du_max), xform != 0, st, s);
            lc.dl = 0;
            lc.gl = gl;
            launch_upsample(lc, tgv ? 1 : 0, st, s);
        }
        lc.op = OP_START;
        lc.gl = L - 1;
        launch_zero_state(lc, tgv ? 1 : 0, st, s);
        lc.gl = gl;
        lc.op = OP_TENSOR;
        launch_tensor(lc, st, s);
        if (xform) launch_transform(lc, xform, s);
    }
    // warp step
    lc.gl = gl;
    lc.op = OP_WARP;
    launch_linearise(lc, -1, 0, float(P.du_max), xform != 0, st, s);
    int iu = 0, ip = 0;
    run_pd(pd_args(lc, P), sv->sched, P.iters, iu, ip, s, nullptr, nullptr);
    // finish
    if (full) {
        lc.iu = iu;
        lc.ip = ip;
        lc.op = OP_FINISH;
        lc.lev = 0;
        lc.gl = 0;
        launch_linearise(lc, 1, 1, float(P.du_max), xform != 0, st, s);
        launch_triangulate(lc, s);
    }
    par_u = iu;
    par_p = ip;
}

vfs_status make_bucket(vfs_server* sv, const Geometry& g, Bucket*& out)
{
    auto b = std::make_unique<Bucket>();
    b->g = g;
    b->lay = make_layout(g, sv->params.storage, sv->params.reg == VFS_TGV, sv->params.data_term != VFS_DATA_BRIGHTNESS);
    b->S = sv->cfg.max_slots;
    b->slot.resize(b->S);
    for (int k = 1; b->nsizes < kTickSizes; k *= 2) {
        b->sizes[b->nsizes++] = k < b->S ? k : b->S;
        if (k >= b->S) break;
    }
    if (hipMalloc(&b->slots_dev, sizeof(Slot) * b->S) != hipSuccess ||
        hipMalloc(&b->ctrl_dev, sizeof(Ctrl) * kMaxBatch) != hipSuccess)
        return fail(VFS_E_NOMEM, "bucket tables");
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
        return fail(VFS_E_DEVICE, "hipStreamCreate");
    // every slot starts inactive
    CtrlBlock cb{};
    launch_write_ctrl(cb, kMaxBatch, b->ctrl_dev, b->stream);
    // parity change of one tick (the launch sequence of every tick, any size)
    pd_parity(sv->params.iters, pd_pass_iters(b->g, sv->params.pass_iters, sv->params.storage), b->par_u, b->par_p);
    if (sv->cfg.use_graphs) {
        prepare_pd();
        for (int gl = 0; gl < g.L; ++gl)
            for (int full = 0; full < 2; ++full)
                for (int k = 0; k < b->nsizes; ++k) {
                    int pu, pp;
                    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
                        return fail(VFS_E_DEVICE, "hipStreamBeginCapture");
                    enqueue_tick(sv, *b, b->capture, full != 0, gl, b->sizes[k], pu, pp);
                    if (hipStreamEndCapture(b->capture, &b->graph[gl][full][k]) != hipSuccess)
                        return fail(VFS_E_DEVICE, "hipStreamEndCapture");
                    if (hipGraphInstantiateWithFlags(&b->exec[gl][full][k], b->graph[gl][full][k], 0) != hipSuccess)
                        return fail(VFS_E_DEVICE, "hipGraphInstantiate");
                }
    }
    if (hipGetLastError() != hipSuccess) return fail(VFS_E_DEVICE, "bucket set-up launch failed");
    out = b.get();
    sv->buckets.push_back(std::move(b));
    sv->nbuckets.store(int(sv->buckets.size()));
    return VFS_OK;
}

Bucket* find_bucket(vfs_server* sv, const Geometry& g)
{
    for (auto& b : sv->buckets)
        if (same_geometry(b->g, g)) return b.get();
    return nullptr;
}

void bucket_destroy(Bucket& b)
{
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    for (auto& t : b.inflight) (void)hipEventDestroy(t.ev);
    for (auto e : b.spare_events) (void)hipEventDestroy(e);
    for (int l = 0; l < kMaxLevels; ++l)
        for (int f = 0; f < 2; ++f)
            for (int k = 0; k < kTickSizes; ++k) {
                if (b.exec[l][f][k]) (void)hipGraphExecDestroy(b.exec[l][f][k]);
                if (b.graph[l][f][k]) (void)hipGraphDestroy(b.graph[l][f][k]);
            }
    if (b.slots_dev) (void)hipFree(b.slots_dev);
    if (b.ctrl_dev) (void)hipFree(b.ctrl_dev);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    if (b.capture) (void)hipStreamDestroy(b.capture);
}

void finish_request(vfs_server* sv, Request* r, int state)
{
    r->t_done = Clock::now();
    r->state.store(state);
    {
        // under the lock: a vfs_server_wait_all that has just seen requests
        // outstanding is then already waiting when the notification comes
        // (a decrement between its check and its wait would otherwise leave
        // it asleep until its time-out)
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->outstanding.fetch_sub(1);
    }
    sv->cv.notify_all();
}

// Retire the completed ticks of a bucket; returns whether any completed.
bool retire(vfs_server* sv, Bucket& b)
{
    bool any = false;
    while (!b.inflight.empty()) {
        const hipError_t q = hipEventQuery(b.inflight.front().ev);
        if (q == hipErrorNotReady) break;
        Tick t = b.inflight.front();
        b.inflight.pop_front();
        any = true;
        const int state = q == hipSuccess ? Q_DONE : Q_FAIL;
        if (q != hipSuccess) set_error(sv, VFS_E_DEVICE, "device error in a serving tick");
        for (int z : t.finishing) {
            SlotState& ss = b.slot[z];
            Request* r = ss.req;
            sv->pool.release(r->mem_off, r->mem_bytes);
            ss = SlotState{};
            --sv->active;
            finish_request(sv, r, state);
        }
        b.spare_events.push_back(t.ev);
    }
    return any;
}

// Admit waiting requests in arrival order.  A request whose bucket has no
// free slot is passed over (other sizes go ahead); the first request the
// pool cannot hold stops admission, so that a stream of small requests cannot
// starve a large one.
bool admit(vfs_server* sv)
{
    bool any = false;
    for (auto it = sv->waiting.begin(); it != sv->waiting.end();) {
        Request* r = *it;
        Bucket* b = find_bucket(sv, r->rig->g);
        if (!b) {
            vfs_status st = make_bucket(sv, r->rig->g, b);
            if (st) {
                set_error(sv, st, "creating a bucket failed");
                it = sv->waiting.erase(it);
                finish_request(sv, r, Q_FAIL);
                continue;
            }
        }
        int z = -1;
        for (int k = 0; k < b->S; ++k)
            if (!b->slot[k].req) {
                z = k;
                break;
            }
        if (z < 0) {
            ++it;
            continue;
        }
        size_t off = 0;
        if (!sv->pool.alloc(b->lay.bytes, off)) break;
        sv->pool_peak.store(sv->pool.peak());
        it = sv->waiting.erase(it);
        r->mem_off = off;
        r->mem_bytes = b->lay.bytes;
        r->t_admit = Clock::now();
        r->state.store(Q_RUN);
        Slot sl = r->io;
        bind_state(sl, static_cast<char*>(sv->pool_mem) + off, b->lay);
        launch_write_slot(sl, b->slots_dev + z, b->stream);
        for (const SlotState& o : b->slot)
            if (o.req && o.started && !o.draining) {
                ++sv->joins;
                break;
            }
        SlotState& ss = b->slot[z];
        ss = SlotState{};
        ss.req = r;
        ++sv->active;
        if (sv->active > sv->peak_active.load()) sv->peak_active.store(sv->active);
        any = true;
    }
    return any;
}

// Compose and enqueue the next tick of a bucket; false if it has no work.
bool launch_tick(vfs_server* sv, Bucket& b)
{
    const int L = b.g.L, N = sv->params.warps;
    CtrlBlock cb{};
    Tick t;
    bool work = false, full = false;
    int gl = L - 1, n = 0;
    for (int z = 0; z < b.S; ++z) {
        SlotState& ss = b.slot[z];
        if (!ss.req || ss.draining) continue;
        // the active slots' control words come first: the tick's launches cover only them
        Ctrl& c = cb.c[n++];
        c.slot = uint8_t(z);
        uint8_t ops;
        if (!ss.started) {
            ss.started = true;
            ss.level = L - 1;
            ss.warp = 0;
            ss.flip = 0;
            ops = OP_START | OP_TENSOR | OP_WARP;
        } else {
            ss.flip ^= unsigned(b.par_u) | (unsigned(b.par_p) << 1);
            if (ss.warp + 1 < N) {
                ++ss.warp;
                ops = OP_WARP;
            } else {
                --ss.level;
                ss.warp = 0;
                ops = OP_NEWLEVEL | OP_TENSOR | OP_WARP;
            }
        }
        if (ss.level == 0 && ss.warp == N - 1) {
            ops |= OP_FINISH;
            ss.draining = true;
            t.finishing.push_back(z);
        }
        c.level = int8_t(ss.level);
        c.warp = ss.warp;
        c.ops = ops;
        full |= ops != OP_WARP;
        if (ss.level < gl) gl = ss.level;
        c.flip = uint8_t(ss.flip);
        work = true;
    }
    if (!work) return false;
    int k = 0;
    while (b.sizes[k] < n) ++k;         // launch size: the smallest one that covers the active slots
    launch_write_ctrl(cb, b.sizes[k], b.ctrl_dev, b.stream);
    if (sv->cfg.use_graphs) {
        if (hipGraphLaunch(b.exec[gl][full ? 1 : 0][k], b.stream) != hipSuccess)
            set_error(sv, VFS_E_DEVICE, "hipGraphLaunch failed");
    } else {
        int pu, pp;
        enqueue_tick(sv, b, b.stream, full, gl, b.sizes[k], pu, pp);
    }
    if (full) {
        ++b.full_ticks;
        ++sv->full_ticks;
    }
    if (!b.spare_events.empty()) {
        t.ev = b.spare_events.back();
        b.spare_events.pop_back();
    } else if (hipEventCreateWithFlags(&t.ev, hipEventDisableTiming) != hipSuccess) {
        set_error(sv, VFS_E_DEVICE, "hipEventCreate failed");
        return false;
    }
    (void)hipEventRecord(t.ev, b.stream);
    if (hipGetLastError() != hipSuccess) set_error(sv, VFS_E_DEVICE, "tick launch failed");
    b.inflight.push_back(std::move(t));
    ++b.ticks;
    ++sv->ticks;
    return true;
}

// Plain mode: one request at a time, in arrival order, eager launches.
bool plain_step(vfs_server* sv)
{
    if (sv->plain_cur) {
        const hipError_t q = hipEventQuery(sv->plain_ev);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) set_error(sv, VFS_E_DEVICE, "device error in a plain solve");
        Request* r = sv->plain_cur;
        sv->plain_cur = nullptr;
        --sv->active;
        finish_request(sv, r, q == hipSuccess ? Q_DONE : Q_FAIL);
    }
    if (sv->waiting.empty()) return false;
    Request* r = sv->waiting.front();
    sv->waiting.pop_front();
    Workspace* ws = nullptr;
    for (auto& w : sv->plain_ws)
        if (same_geometry(w->g, r->rig->g)) ws = w.get();
    if (!ws) {
        sv->plain_ws.push_back(std::make_unique<Workspace>());
        ws = sv->plain_ws.back().get();
    }
    const bool tgv = sv->params.reg == VFS_TGV, xform = sv->params.data_term != VFS_DATA_BRIGHTNESS;
    vfs_status st = VFS_OK;
    if (make_layout(r->rig->g, sv->params.storage, tgv, xform).bytes > sv->cfg.hbm_budget_bytes)
        st = fail(VFS_E_BUDGET, "request exceeds the HBM budget");
    // sizes the workspace on every request (nothing to do once it fits): a
    // failed allocation leaves it empty, and the next request of this size
    // allocates again or fails in turn, never runs on an empty workspace
    if (!st) st = ensure_workspace(*ws, r->rig->g, 1, sv->params.storage, tgv, xform);
    if (!st && (!ws->mem || !ws->slots)) st = fail(VFS_E_NOMEM, "plain workspace");
    if (st) {
        set_error(sv, st, "plain workspace");
        finish_request(sv, r, Q_FAIL);
        return true;
    }
    r->t_admit = Clock::now();
    r->state.store(Q_RUN);
    ++sv->active;
    if (sv->active > sv->peak_active.load()) sv->peak_active.store(sv->active);
    Slot sl = r->io;
    bind_state(sl, ws->mem, ws->lay);
    launch_write_slot(sl, ws->slots, sv->plain_stream);
    vfs_params p = sv->params;
    p.levels = r->rig->g.L;
    st = solve_slots(ws->slots, 1, r->rig->g, p, sv->plain_stream, nullptr);
    if (st) set_error(sv, st, "plain solve launch failed");
    (void)hipEventRecord(sv->plain_ev, sv->plain_stream);
    sv->plain_cur = r;
    ++sv->ticks;
    return true;
}

void scheduler(vfs_server* sv)
{
    (void)hipSetDevice(sv->device);
    const bool plain = sv->cfg.mode == VFS_SERVE_PLAIN;
    const int depth = 2;    // ticks enqueued ahead per bucket
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            bool idle = sv->incoming.empty() && sv->waiting.empty() && sv->active == 0 && !sv->plain_cur;
            if (idle) {
                if (sv->stop.load()) break;
                sv->cv.wait_for(lk, std::chrono::milliseconds(50));
            }
            while (!sv->incoming.empty()) {
                sv->waiting.push_back(sv->incoming.front());
                sv->incoming.pop_front();
            }
        }
        bool progress = false;
        if (plain) {
            progress = plain_step(sv);
        } else {
            for (auto& b : sv->buckets) progress |= retire(sv, *b);
            progress |= admit(sv);
            for (auto& b : sv->buckets)
                if (int(b->inflight.size()) < depth) progress |= launch_tick(sv, *b);
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

vfs_server::~vfs_server()
{
    stop.store(true);
    cv.notify_all();
    if (worker.joinable()) worker.join();
    for (auto& b : buckets) bucket_destroy(*b);
    if (plain_stream) {
        (void)hipStreamSynchronize(plain_stream);
        (void)hipStreamDestroy(plain_stream);
    }
    if (plain_ev) (void)hipEventDestroy(plain_ev);
    plain_ws.clear();
    if (pool_mem) (void)hipFree(pool_mem);
}

extern "C" {

vfs_status vfs_server_config_default(vfs_server_config* out)
{
    if (!out) return fail(VFS_E_INVALID, "out is NULL");
    out->mode = VFS_SERVE_BATCHED;
    out->hbm_budget_bytes = size_t(1) << 30;
    out->max_slots = 16;
    out->use_graphs = 1;
    return VFS_OK;
}

vfs_status vfs_server_create(const vfs_server_config* cfg, const vfs_params* params, vfs_server** out)
{
    if (!out) return fail(VFS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(VFS_E_INVALID, "cfg is NULL");
    vfs_status st = check_params(params);
    if (st) return st;
    if (params->warps < 1 || params->iters < 1) return fail(VFS_E_INVALID, "serving needs warps >= 1 and iters >= 1");
    if (cfg->mode != VFS_SERVE_BATCHED && cfg->mode != VFS_SERVE_PLAIN) return fail(VFS_E_INVALID, "bad mode");
    if (cfg->max_slots < 1 || cfg->max_slots > kMaxBatch)
        return fail(VFS_E_INVALID, "max_slots must be in [1, %d]", kMaxBatch);
    if (cfg->hbm_budget_bytes < 256) return fail(VFS_E_INVALID, "HBM budget too small");
    std::unique_ptr<vfs_server> sv(new (std::nothrow) vfs_server());
    if (!sv) return fail(VFS_E_NOMEM, "host allocation");
    sv->cfg = *cfg;
    sv->params = *params;
    sv->sched = schedule(*params);
    if (hipGetDevice(&sv->device) != hipSuccess) return fail(VFS_E_DEVICE, "hipGetDevice failed");
    if (cfg->mode == VFS_SERVE_BATCHED) {
        if (hipMalloc(&sv->pool_mem, cfg->hbm_budget_bytes) != hipSuccess)
            return fail(VFS_E_NOMEM, "HBM pool of %zu bytes", cfg->hbm_budget_bytes);
        sv->pool.reset(cfg->hbm_budget_bytes);
    } else {
        if (hipStreamCreateWithFlags(&sv->plain_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sv->plain_ev, hipEventDisableTiming) != hipSuccess)
            return fail(VFS_E_DEVICE, "stream / event creation");
    }
    vfs_server* raw = sv.get();
    raw->worker = std::thread(scheduler, raw);
    *out = sv.release();
    return VFS_OK;
}

vfs_status vfs_server_request_bytes(const vfs_server* sv, const vfs_rig* rig, size_t* bytes)
{
    if (!sv || !rig || !bytes) return fail(VFS_E_INVALID, "NULL argument");
    const vfs_params& P = sv->params;
    *bytes = make_layout(rig->g, P.storage, P.reg == VFS_TGV, P.data_term != VFS_DATA_BRIGHTNESS).bytes;
    return VFS_OK;
}

vfs_status vfs_server_submit(vfs_server* sv, vfs_rig* rig, const float* I0, const float* I1, size_t pitch_bytes,
                             float* u_out, float* w_out, float* depth_out, float* z_out, uint8_t* valid_out,
                             double beta, double eta, unsigned long long* ticket)
{
    if (!sv || !rig || !ticket) return fail(VFS_E_INVALID, "NULL argument");
    *ticket = 0;
    if (!I0 || !I1 || !depth_out) return fail(VFS_E_INVALID, "NULL image or depth buffer");
    const int W = rig->g.W[0];
    if (pitch_bytes % sizeof(float) || pitch_bytes < sizeof(float) * W) return fail(VFS_E_INVALID, "bad pitch");
    if (!(beta >= 0.0) || !(eta > 0.0)) return fail(VFS_E_INVALID, "bad tensor parameters");
    const vfs_params& P = sv->params;
    const size_t need = make_layout(rig->g, P.storage, P.reg == VFS_TGV, P.data_term != VFS_DATA_BRIGHTNESS).bytes;
    if (sv->cfg.mode == VFS_SERVE_BATCHED && need > sv->cfg.hbm_budget_bytes)
        return fail(VFS_E_BUDGET, "one request needs %zu bytes, the HBM budget is %zu", need,
                    sv->cfg.hbm_budget_bytes);
    auto r = std::make_unique<Request>();
    r->rig = rig;
    Slot& sl = r->io;
    sl.I0 = I0;
    sl.I1 = I1;
    sl.in_pitch = int(pitch_bytes / sizeof(float));
    sl.out_pitch = sl.in_pitch;
    sl.u_out = u_out;
    sl.w_out = w_out;
    sl.depth_out = depth_out;
    sl.z_out = z_out;
    sl.valid_out = valid_out;
    bind_rig(sl, rig);
    sl.beta = float(beta);
    sl.eta = float(eta);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->error) return fail(sv->error, "server failed earlier: %s", sv->error_msg);
        r->ticket = sv->next_ticket++;
        r->t_arrive = Clock::now();
        *ticket = r->ticket;
        sv->incoming.push_back(r.get());
        sv->requests.emplace(r->ticket, std::move(r));
        sv->outstanding.fetch_add(1);
    }
    sv->cv.notify_all();
    return VFS_OK;
}

vfs_status vfs_server_poll(vfs_server* sv, unsigned long long ticket, int* done, double* latency_s)
{
    if (!sv || !done) return fail(VFS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return fail(VFS_E_INVALID, "unknown ticket %llu", ticket);
    const Request& r = *it->second;
    const int st = r.state.load();
    if (st == Q_FAIL) return fail(sv->error ? sv->error : VFS_E_DEVICE, "request failed: %s", sv->error_msg);
    *done = st == Q_DONE;
    if (latency_s) *latency_s = *done ? seconds_since(r.t_arrive, r.t_done) : -1.0;
    return VFS_OK;
}

vfs_status vfs_server_times(vfs_server* sv, unsigned long long ticket, double* admit_s, double* done_s)
{
    if (!sv) return fail(VFS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return fail(VFS_E_INVALID, "unknown ticket %llu", ticket);
    const Request& r = *it->second;
    const int st = r.state.load();
    if (admit_s) *admit_s = st >= Q_RUN ? seconds_since(r.t_arrive, r.t_admit) : -1.0;
    if (done_s) *done_s = st == Q_DONE ? seconds_since(r.t_arrive, r.t_done) : -1.0;
    return VFS_OK;
}

vfs_status vfs_server_wait_all(vfs_server* sv, double timeout_s)
{
    if (!sv) return fail(VFS_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
    while (sv->outstanding.load() > 0) {
        if (sv->cv.wait_until(lk, until) == std::cv_status::timeout && sv->outstanding.load() > 0)
            return fail(VFS_E_DEVICE, "timed out with %lld requests outstanding", sv->outstanding.load());
    }
    if (sv->error) return fail(sv->error, "%s", sv->error_msg);
    return VFS_OK;
}

vfs_status vfs_server_stats(vfs_server* sv, vfs_server_counters* out)
{
    if (!sv || !out) return fail(VFS_E_INVALID, "NULL argument");
    // atomics written by the scheduler thread: no scheduler structure is read here
    out->ticks = sv->ticks.load();
    out->peak_active = sv->peak_active.load();
    out->pool_peak_bytes = sv->pool_peak.load();
    out->buckets = sv->nbuckets.load();
    out->joins = sv->joins.load();
    out->full_ticks = sv->full_ticks.load();
    return VFS_OK;
}

void vfs_server_destroy(vfs_server* sv) { delete sv; }

}  // extern "C"
