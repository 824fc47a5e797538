// Host runtime shared by the direct solves and the serving loop: rig
// (device-resident fields of one calibration and image size), per-pair state
// layout, workspace, the primal-dual launch schedule, and the batched solve.
#pragma once

#include <stdarg.h>
#include <stdio.h>

#include <utility>
#include <vector>

#include "../../include/vfs.h"
#include "vfs_internal.h"

namespace vfs {

vfs_status fail(vfs_status st, const char* fmt, ...);

// Level sizes of an image size and level count (pitch: multiple of 64
// elements), with the offsets of a level-stacked plane.
Geometry make_geometry(int W, int H, int L);
inline size_t plane_elems(const Geometry& g, int l) { return size_t(g.pitch[l]) * size_t(g.H[l]); }
inline size_t stacked_elems(const Geometry& g) { return size_t(g.off[g.L - 1]) + plane_elems(g, g.L - 1); }

// Byte offsets of one pair's solve state inside its region (256-byte aligned).
struct PairLayout {
    size_t J0, J1, u[2], v[2], p[2], q[2], w, uw, gw, tpack, rho, R0, R1;
    size_t bytes;
    int storage;
    bool tgv, xform;   // xform: the data term's image planes R0, R1
};
PairLayout make_layout(const Geometry& g, int storage, bool tgv, bool xform);
// Points the state fields of sl into region (device memory of lay.bytes).
void bind_state(Slot& sl, void* region, const PairLayout& lay);

// Per-pair state for up to `cap` pairs of one geometry (direct solves).
struct Workspace {
    int cap = 0;
    Geometry g{};
    PairLayout lay{};
    void* mem = nullptr;
    Slot* slots = nullptr;      // device descriptors, kMaxBatch entries

    Workspace() = default;
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    ~Workspace() { release(); }
    void release();
};
vfs_status ensure_workspace(Workspace& ws, const Geometry& g, int n, int storage, bool tgv, bool xform);

}  // namespace vfs

struct vfs_rig {
    vfs::RigGeom geom;
    vfs::RigGeom* geom_dev = nullptr;   // device copy (read by the triangulation)
    vfs::Geometry g{};
    float2* gamma[vfs::kMaxLevels] = {};
    uint8_t* flags[vfs::kMaxLevels] = {};
    float2* calib = nullptr;
    float2* radial = nullptr;           // camera 0's radial table (TriGeom)
    int device = 0;
    vfs::Workspace ws;                  // used by vfs_solve / vfs_solve_batch

    // captured direct solves: one HIP graph per launch configuration (batch
    // size, solver parameters, workspace), replayed by later solves
    struct SolveGraph {
        vfs_params params;
        int n;
        const void* mem;
        const vfs::Slot* slots;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<SolveGraph> graphs;
    hipStream_t capture_stream = nullptr;
    bool use_graphs = true;

    // level-0 primal-dual timing
    bool profile = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    long long launches = 0;
    int pass_iters = 2;                 // iterations per profiled launch (last solve)
    double ms = 0.0;
    hipStream_t last_stream = nullptr;

    ~vfs_rig();
};

namespace vfs {

vfs_status check_params(const vfs_params* p);

// Rig fields of r into sl.
void bind_rig(Slot& sl, const vfs_rig* r);

// Scalar schedule of the over-relaxation (theta) and the step factors.
struct Sched {
    std::vector<float> s, theta;
};
Sched schedule(const vfs_params& p);

// K primal-dual iterations from a warp start with the state parity
// (base.lc.iu, base.lc.ip); iu, ip receive the parity holding the result.
// Returns the number of multi-iteration passes (base.pass iterations each),
// which ev0 / ev1 (if given) bracket.
int run_pd(PdArgs base, const Sched& sc, int K, int& iu, int& ip, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
// Iterations per pass (2, 3 or 4) of the dominant primal-dual launches for
// pairs of level-0 geometry g in storage mode `storage` (independent of the
// batch), or `requested` if that is 2, 3 or 4.
int pd_pass_iters(const Geometry& g, int requested, int storage);
// Parity change of the state copies (u/v, p/q) over run_pd's K iterations
// with NP iterations per pass.
void pd_parity(int K, int NP, int& pu, int& pp);

// PdArgs of a launch with the solver constants of params.
PdArgs pd_args(const Launch& lc, const vfs_params& params);

// Validates the arguments of a batched solve of n pairs on rig r (outputs:
// whether u_out, w_out, depth_out are required).
vfs_status check_batch(const vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                       float* const* u_out, float* const* w_out, float* const* depth_out, const vfs_params* params,
                       const double* betas, const double* etas, bool outputs);
// Writes the descriptors of n pairs (state of pair b at state + b * lay.bytes)
// to slots (device), stream-ordered on s.
void write_batch_slots(const vfs_rig* r, int n, const float* const* I0, const float* const* I1, size_t pitch_bytes,
                       float* const* u_out, float* const* w_out, float* const* depth_out, float* const* z_out,
                       uint8_t* const* valid_out, const vfs_params* params, const double* betas,
                       const double* etas, bool outputs, char* state, const PairLayout& lay, Slot* slots,
                       hipStream_t s);

// A probed pair of a solve (vfs_solve_probe): the caller's request and where
// the pair's state lives.
struct Probe {
    vfs_probe req;
    const char* region;     // the pair's state region (device)
    PairLayout lay;
};

// Whole method on the n pairs whose descriptors are at slots (device, all of
// geometry g), enqueued on stream s.  Profiling events, if prof is not NULL
// and enabled, go to prof.  With a probe, the solve copies the probed pair's
// state at the requested warp and stops after that warp's clip.
vfs_status solve_slots(const Slot* slots, int n, const Geometry& g, const vfs_params& params, hipStream_t s,
                       vfs_rig* prof, const Probe* probe = nullptr);

}  // namespace vfs
